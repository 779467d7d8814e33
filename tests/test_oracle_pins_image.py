"""Pins of the oracle's image-space operators of the training objective (Eq. 9, Eq. 11):
the cross-bilateral denoiser and its adjoint, the map regulariser, the L1 data term and
the guide features, each against a library routine, a closed form, an invariant or
finite differences rather than against its own formula."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import oracle as O

from . import scenes


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _window_sum(img, kern):
    """sum over the window, clipped to the image (zero padding), per channel."""
    img = np.asarray(img, np.float64)
    if img.ndim == 2:
        return ndimage.correlate(img, kern, mode="constant", cval=0.0)
    return np.stack([ndimage.correlate(img[..., c], kern, mode="constant", cval=0.0)
                     for c in range(img.shape[2])], -1)


# --------------------------------------------------------------------------- D

def test_denoise_constant_image_is_fixed():
    """A weighted mean of equal values is that value, whatever the guide."""
    rng = np.random.default_rng(1)
    img = np.broadcast_to(np.array([0.3, 1.7, -2.0]), (9, 13, 3)).copy()
    guide = rng.normal(size=(9, 13, 4))
    out = O.denoise(img, guide, [0.5, 2.0, 0.0, 7.0], 0.1, 3)
    np.testing.assert_allclose(out, img, rtol=1e-14, atol=0)


def test_denoise_radius_zero_is_identity():
    rng = np.random.default_rng(2)
    img = rng.normal(size=(5, 6, 3))
    out = O.denoise(img, rng.normal(size=(5, 6, 2)), [1.0, 1.0], 0.3, 0)
    np.testing.assert_array_equal(out, img)


@pytest.mark.parametrize("r", [1, 2, 4])
def test_denoise_without_guide_or_distance_is_clipped_box_mean(r):
    """All factors 0: every weight is 1, so D is the box mean over the part of the
    window inside the image (scipy correlate of the image and of ones)."""
    rng = np.random.default_rng(3 + r)
    img = rng.normal(size=(11, 7, 3))        # non-square: a swapped x/y fails
    box = np.ones((2 * r + 1, 2 * r + 1))
    want = _window_sum(img, box) / _window_sum(np.ones(img.shape[:2]), box)[..., None]
    out = O.denoise(img, rng.normal(size=(11, 7, 1)), [0.0], 0.0, r)
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-13)


def test_denoise_distance_only_is_normalised_gaussian():
    """Guide factors 0: D is a truncated Gaussian convolution renormalised at the
    borders; the kernel is built from the separable 1-D Gaussian."""
    rng = np.random.default_rng(8)
    img = rng.normal(size=(10, 12, 3))
    r, sigma = 3, 1.3
    g1 = np.exp(-np.arange(-r, r + 1) ** 2 / (2 * sigma ** 2))
    kern = np.outer(g1, g1)
    want = _window_sum(img, kern) / _window_sum(np.ones(img.shape[:2]), kern)[..., None]
    out = O.denoise(img, np.zeros((10, 12, 2)), [0.0, 0.0], 1.0 / (2 * sigma ** 2), r)
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-13)


def test_denoise_strong_guide_edge_does_not_mix():
    """A guide step with a huge factor on its channel (and noise with factor 0 on the
    other) cuts the weights across the step: each side is the box mean over its own
    side of the window (masked correlate)."""
    rng = np.random.default_rng(5)
    H, W, r = 9, 14, 2
    img = rng.normal(size=(H, W, 3))
    side = np.zeros((H, W))
    side[:, 6:] = 1.0
    side[7:, :] = 1.0                         # an L-shaped region
    guide = np.stack([rng.normal(size=(H, W)), side], -1)
    out = O.denoise(img, guide, [0.0, 1e4], 0.0, r)
    box = np.ones((2 * r + 1, 2 * r + 1))
    want = np.zeros_like(img)
    for s in (0.0, 1.0):
        m = (side == s).astype(np.float64)
        with np.errstate(invalid="ignore"):   # windows without a pixel of this side are unused
            mean = _window_sum(img * m[..., None], box) / _window_sum(m, box)[..., None]
        want[side == s] = mean[side == s]
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-12)


def test_denoise_vjp_is_the_transpose():
    """<D(I), G> = <I, D^T(G)> for random I, G (dot-product test), and D^T of a unit
    cotangent at pixel p is the column of weights p spreads, via finite differences."""
    rng = np.random.default_rng(6)
    H, W, r = 8, 11, 3
    guide = rng.normal(size=(H, W, 3))
    coef, sp = [0.7, 0.2, 1.5], 0.15
    img, G = rng.normal(size=(H, W, 3)), rng.normal(size=(H, W, 3))
    lhs = np.sum(O.denoise(img, guide, coef, sp, r) * G)
    rhs = np.sum(img * O.denoise_vjp(G, guide, coef, sp, r))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # derivative of one output value w.r.t. every input value by finite differences
    e = np.zeros((H, W, 3))
    e[3, 5, 1] = 1.0
    col = O.denoise_vjp(e, guide, coef, sp, r)
    fd = np.zeros_like(col)
    for y in range(H):
        for x in range(W):
            d = np.zeros((H, W, 3))
            d[y, x, 1] = 1.0
            fd[y, x, 1] = (O.denoise(img + d, guide, coef, sp, r) - O.denoise(img - d, guide, coef, sp, r))[3, 5, 1] / 2
    np.testing.assert_allclose(col, fd, rtol=1e-10, atol=1e-13)
    assert np.all(col[..., 0] == 0) and np.all(col[..., 2] == 0)
    assert np.count_nonzero(col[..., 1]) == (2 * r + 1) * (2 * r + 1)


def test_denoise_rejects_mismatched_coefficients():
    with pytest.raises(ValueError):
        O.denoise(np.zeros((3, 3, 3)), np.zeros((3, 3, 2)), [1.0], 0.0, 1)


# --------------------------------------------------------------------------- L(m)

def test_tv_constant_map_is_zero():
    loss, g = O.tv(np.full((6, 5, 3), 0.42))
    assert loss == 0.0 and np.all(g == 0.0)


@pytest.mark.parametrize("shape", [(7, 9), (7, 9, 3), (1, 9), (7, 1)])
def test_tv_ramp_closed_form(shape):
    """m = a x + b y (+ a per-channel offset): every horizontal pair differs by a and
    every vertical pair by b, so the two means are |a| and |b| (0 without pairs)."""
    a, b = -0.37, 1.25
    h, w = shape[:2]
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    m = a * x + b * y
    if len(shape) == 3:
        m = m[..., None] + np.array([0.0, 3.0, -1.0])
    loss, g = O.tv(m)
    want = (abs(a) if w > 1 else 0.0) + (abs(b) if h > 1 else 0.0)
    assert loss == pytest.approx(want, rel=1e-13, abs=1e-15)
    # gradient of the horizontal term: -sign(a) / nh on the first column, +sign(a) / nh
    # on the last, 0 between (each interior value gains and loses one pair)
    c = 1 if len(shape) == 2 else shape[2]
    gx = np.zeros((h, w))
    if w > 1:
        nh = c * h * (w - 1)
        gx[:, 0] -= np.sign(a) / nh
        gx[:, -1] += np.sign(a) / nh
    gy = np.zeros((h, w))
    if h > 1:
        nv = c * (h - 1) * w
        gy[0, :] -= np.sign(b) / nv
        gy[-1, :] += np.sign(b) / nv
    want_g = gx + gy
    if len(shape) == 3:
        want_g = np.repeat(want_g[..., None], c, -1)
    np.testing.assert_allclose(g, want_g, rtol=1e-13, atol=1e-16)


def test_tv_checkerboard_is_two():
    y, x = np.mgrid[0:6, 0:8]
    loss, _ = O.tv(((x + y) % 2).astype(np.float64))
    assert loss == pytest.approx(2.0, rel=1e-15)


def test_tv_gradient_by_finite_differences():
    rng = np.random.default_rng(12)
    m = rng.normal(size=(5, 6, 2))            # no two neighbours equal: L is smooth here
    _, g = O.tv(m)
    h = 1e-7
    fd = np.zeros_like(m)
    for idx in np.ndindex(m.shape):
        d = np.zeros_like(m)
        d[idx] = h
        fd[idx] = (O.tv(m + d)[0] - O.tv(m - d)[0]) / (2 * h)
    # rounding of the central difference: ~1e-16 * L / h ~ 1e-9; gradient entries are ~1/50
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


# --------------------------------------------------------------------------- L1

def test_l1_closed_form_and_gradient():
    a = np.array([1.0, -2.0, 0.5, 3.0])
    b = np.array([0.0, -2.0, 1.0, 1.0])
    loss, g = O.l1(a, b)
    assert loss == pytest.approx((1.0 + 0.0 + 0.5 + 2.0) / 4, rel=1e-15)
    np.testing.assert_array_equal(g, np.array([1.0, 0.0, -1.0, 1.0]) / 4)


# --------------------------------------------------------------------------- guide features

def test_gbuffer_plane_closed_form():
    """Camera over the textured plane z = 0: each pixel-centre ray meets the plane at
    t = -o_z / d_z (plane equation, not the triangle test); the normal is +z (toward
    the camera); the albedo is the texture bilinearly sampled (scipy map_coordinates)
    at the affine UV of the hit; rays that miss the quad give zeros."""
    rng = np.random.default_rng(4)
    tex = rng.uniform(0.1, 0.9, (16, 16, 3)).astype(np.float32)
    w = scenes.plane_workload(tex=tex, half=0.3, cam_eye=(0.05, 0.1, 0.6), res=24, cam_fov=70.0)
    sc = O.Scene(w)
    out, margin = O.gbuffer(sc)
    K, R, t = (np.asarray(v, np.float64) for v in (w.camera.K, w.camera.R, w.camera.t))
    o = -R.T @ t
    hf = float(np.float32(0.3))
    hits = misses = 0
    for j in range(w.camera.height):
        for i in range(w.camera.width):
            row = out[j * w.camera.width + i]
            if margin[j * w.camera.width + i] < 1.0:
                continue                      # too close to the quad's border or diagonal
            d = R.T @ np.linalg.solve(K, np.array([i + 0.5, j + 0.5, 1.0]))
            d /= np.linalg.norm(d)
            tt = -o[2] / d[2]
            x = o + tt * d
            if abs(x[0]) > hf or abs(x[1]) > hf:
                np.testing.assert_array_equal(row, np.zeros(8))
                misses += 1
                continue
            u, v = (x[0] + hf) / (2 * hf), (x[1] + hf) / (2 * hf)
            alb = [ndimage.map_coordinates(tex[..., c].astype(np.float64), [[v * 16 - 0.5], [u * 16 - 0.5]],
                                           order=1, mode="nearest")[0] for c in range(3)]
            np.testing.assert_allclose(row[0:3], alb, rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(row[3:6], [0.0, 0.0, 1.0], atol=1e-12)
            assert row[6] == pytest.approx(tt, rel=1e-12)
            assert row[7] == 1.0
            hits += 1
    assert hits > 200 and misses > 50
