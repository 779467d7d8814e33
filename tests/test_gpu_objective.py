"""The training objective's device operators (Eq. 9, Eq. 11) against the FP64 oracle,
through the C ABI: the cross-bilateral denoiser and its VJP, the guide features, the
map regulariser and the L1 data term, and the torch Functions over them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes
from .gpu_util import ctx, dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24   # FP32 unit roundoff


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    O.build(force=False)


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _denoise_dev(img, guide, coef, spatial, r, vjp=False):
    import torch
    from paper_2503_12174_amd import dpcs
    c = ctx()
    H, W = img.shape[:2]
    p = dpcs.denoise_params(W, H, r, spatial, coef)
    out = torch.full((H, W, 3), np.nan, dtype=torch.float32, device="cuda")
    g = dev(guide, torch.float32) if guide.shape[2] else None
    (dpcs.dpcs_denoise_vjp if vjp else dpcs.dpcs_denoise)(c, p, dev(img, torch.float32), g, out)
    c.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _fwd_bound(r, scale):
    """|D_dev - D| <= (7n + 4) u max|I| for n = (2r+1)^2 taps: each FP32 weight carries a
    relative error <= 8u e + 2u from its exponent e and exp2 (so an absolute error
    <= 3u + 2u w, since w e <= 1/e), the normalised sum turns that into <= 2(3nu + 2uW)/W
    times max|I| with W >= 1 (the centre weight is 1), and the two FP32 sums add n u."""
    n = (2 * r + 1) ** 2
    return (7 * n + 4) * U32 * scale


def _vjp_bound(r, scale):
    """D^T: u_p = G_p / W_p carries (3n + 3)u relative error (W_p as above); the gather of
    n unnormalised weights (sum <= n) adds n (3n + 3)u + (3n + 2n)u + n^2 u, times max|G|."""
    n = (2 * r + 1) ** 2
    return (4 * n * n + 8 * n) * U32 * scale


def _tol(bound, want):
    """Both the derived worst-case bound and the path's stated bar, 1e-4 relative to the
    output's scale, must hold (the bound of D^T grows as n^2 and is the looser one from
    r = 2 on; measured errors are ~5e-7 relative)."""
    return min(bound, 1e-4 * np.abs(want).max())


CASES = [  # (H, W, G, r): ragged tiles, several tiles, every guide packing, radius 0..8
    (1, 1, 0, 2),
    (5, 3, 1, 0),
    (37, 53, 3, 1),
    (40, 33, 4, 3),
    (70, 45, 7, 3),
    (33, 70, 8, 5),
    (19, 41, 5, 8),
]


def _case(H, W, G, seed):
    rng = np.random.default_rng(seed)
    img = _f32(rng.uniform(0, 1, (H, W, 3)))
    # guides with structure: smooth ramps + steps + noise; large offsets on one channel
    y, x = np.mgrid[0:H, 0:W]
    gs = []
    for k in range(G):
        g = 0.3 * np.sin(0.2 * x + k) + 0.2 * (y > H // 2) + 0.05 * rng.normal(size=(H, W))
        if k == G - 1:
            g = g + 5.0          # a distance-like channel: large values, small differences
        gs.append(g)
    guide = _f32(np.stack(gs, -1) if G else np.zeros((H, W, 0)))
    coef = _f32(rng.uniform(0.5, 30.0, G))
    return img, guide, coef


@pytest.mark.parametrize("H,W,G,r", CASES)
def test_denoise_matches_oracle(H, W, G, r):
    img, guide, coef = _case(H, W, G, H * 131 + W)
    sp = float(np.float32(0.2))
    got = _denoise_dev(img, guide, coef, sp, r)
    want = O.denoise(img, guide, coef, sp, r)
    np.testing.assert_allclose(got, want, rtol=0, atol=_tol(_fwd_bound(r, np.abs(img).max()), want))


@pytest.mark.parametrize("H,W,G,r", CASES)
def test_denoise_vjp_matches_oracle(H, W, G, r):
    img, guide, coef = _case(H, W, G, H * 7 + W)
    G_ = _f32(np.random.default_rng(H + W).normal(size=(H, W, 3)))
    sp = float(np.float32(0.2))
    got = _denoise_dev(G_, guide, coef, sp, r, vjp=True)
    want = O.denoise_vjp(G_, guide, coef, sp, r)
    np.testing.assert_allclose(got, want, rtol=0, atol=_tol(_vjp_bound(r, np.abs(G_).max()), want))


def test_denoise_adjoint_identity_at_scale():
    """<D(I), G> = <D^T(G), I> on a 1024 x 768 image with an 8-channel guide (a property
    that holds at any size), within the FP32 bounds of the two sides."""
    H, W, r = 768, 1024, 3
    img, guide, coef = _case(H, W, 8, 5)
    G_ = _f32(np.random.default_rng(6).normal(size=(H, W, 3)))
    sp = float(np.float32(0.125))
    a = _denoise_dev(img, guide, coef, sp, r)
    b = _denoise_dev(G_, guide, coef, sp, r, vjp=True)
    lhs, rhs = np.sum(a * G_), np.sum(img * b)
    tol = H * W * 3 * (_fwd_bound(r, 1.0) * np.abs(G_).max() + _vjp_bound(r, np.abs(G_).max()))
    assert abs(lhs - rhs) <= tol
    assert abs(lhs - rhs) <= 1e-4 * np.sum(np.abs(a * G_))   # in practice far inside the bound
    # sampled pixels against the oracle on a crop whose windows lie inside the crop
    y0, x0, h, w = 300, 500, 24, 40
    crop = O.denoise(img[y0 - r:y0 + h + r, x0 - r:x0 + w + r], guide[y0 - r:y0 + h + r, x0 - r:x0 + w + r],
                     coef, sp, r)[r:-r, r:-r]
    np.testing.assert_allclose(a[y0:y0 + h, x0:x0 + w], crop, rtol=0, atol=_tol(_fwd_bound(r, 1.0), crop))


def test_denoise_of_the_benchmark_rendering():
    """D with its default parameters on a 256 x 256 rendering of the 50k-triangle corner,
    steered by that scene's guide features, and its VJP, against the oracle over the
    whole image."""
    import torch
    from paper_2503_12174_amd import dpcs
    from paper_2503_12174_amd import objective as Ob
    c = ctx()
    w = synth.corner_50k(spp=4)
    sc = dpcs.Scene(c, w.mesh, bvh="sah")
    f = torch.float32
    alb, rough, spec, proj = dev(w.albedo, f), dev(w.roughness, f), dev(w.specular, f), dev(w.proj_image, f)
    p = dpcs.params_from(w, alb, rough, spec)
    img = torch.zeros((256, 256, 3), device="cuda")
    dpcs.dpcs_render(c, sc, p, proj, img)
    guide = Ob.gbuffer(c, sc, p)
    cfg = Ob.DenoiseConfig()
    x = img.clone().requires_grad_(True)
    den = Ob.denoise(c, x, guide, cfg)
    G = torch.as_tensor(np.random.default_rng(51).normal(size=(256, 256, 3)).astype(np.float32)).cuda()
    den.backward(G)
    c.synchronize()
    f64 = lambda t: t.detach().cpu().numpy().astype(np.float64)
    coef, sp = _f32(cfg.guide), float(np.float32(cfg.spatial))
    want = O.denoise(f64(img), f64(guide), coef, sp, cfg.radius)
    np.testing.assert_allclose(f64(den), want, rtol=0, atol=_tol(_fwd_bound(cfg.radius, np.abs(f64(img)).max()), want))
    want_g = O.denoise_vjp(f64(G), f64(guide), coef, sp, cfg.radius)
    np.testing.assert_allclose(f64(x.grad), want_g, rtol=0,
                               atol=_tol(_vjp_bound(cfg.radius, np.abs(f64(G)).max()), want_g))
    # the camera sees the surface almost everywhere (coverage channel)
    assert float(guide[..., 7].mean()) > 0.9


def test_denoise_rejects_bad_params():
    import torch
    from paper_2503_12174_amd import dpcs
    c = ctx()
    img = torch.zeros((8, 8, 3), device="cuda")
    out = torch.zeros_like(img)
    guide = torch.zeros((8, 8, 2), device="cuda")
    for p in (dpcs.denoise_params(8, 8, 9, 0.1, (1.0, 1.0)),       # radius > 8
              dpcs.denoise_params(8, 8, 2, -1.0, (1.0, 1.0)),      # negative factor
              dpcs.denoise_params(8, 8, 2, 0.1, (1.0, float("nan"))),
              dpcs.denoise_params(0, 8, 2, 0.1, (1.0, 1.0))):
        with pytest.raises(Exception):
            dpcs.dpcs_denoise(c, p, img, guide, out)
    with pytest.raises(Exception):   # guide channels without a guide
        dpcs.dpcs_denoise(c, dpcs.denoise_params(8, 8, 2, 0.1, (1.0, 1.0)), img, None, out)
    with pytest.raises(Exception):   # in place
        dpcs.dpcs_denoise(c, dpcs.denoise_params(8, 8, 2, 0.1, (1.0, 1.0)), img, guide, img)
    with pytest.raises(Exception):   # beyond the largest image side
        dpcs.dpcs_denoise(c, dpcs.denoise_params(16385, 1, 2, 0.1, (1.0, 1.0)), img, guide, out)
    loss = torch.zeros((), device="cuda")
    with pytest.raises(Exception):   # an empty map
        c.check(dpcs.lib().dpcs_tv_loss(c.h, dpcs._ptr(img), 0, 8, 3, dpcs._ptr(loss)))
    with pytest.raises(Exception):   # no values
        c.check(dpcs.lib().dpcs_l1_loss(c.h, dpcs._ptr(img), dpcs._ptr(out), 0, dpcs._ptr(loss)))
    # the context still works after rejected calls
    dpcs.dpcs_denoise(c, dpcs.denoise_params(8, 8, 2, 0.1, (1.0, 1.0)), img, guide, out)
    c.synchronize()


# ------------------------------------------------------------------ guide features

def _gbuffer_dev(w, scene=None):
    import torch
    from paper_2503_12174_amd import dpcs
    from paper_2503_12174_amd.objective import gbuffer
    c = ctx()
    sc = scene or dpcs.Scene(c, w.mesh)
    alb = dev(w.albedo, torch.float32)
    rough, spec = dev(w.roughness, torch.float32), dev(w.specular, torch.float32)
    p = dpcs.params_from(w, alb, rough, spec)
    g = gbuffer(c, sc, p)
    c.synchronize()
    return g.cpu().numpy().reshape(-1, 8).astype(np.float64)


def _compare_gbuffer(got, want, margin):
    clean = margin >= 1.0
    assert clean.mean() > 0.95
    a, b = got[clean], want[clean]
    assert np.array_equal(a[:, 7], b[:, 7]), "hit / miss differs on robust pixels"
    # FP64 attributes rounded once to FP32 on the device: a few units of 2^-24
    np.testing.assert_allclose(a, b, rtol=4 * U32, atol=4 * U32)
    return int(clean.sum())


@pytest.mark.parametrize("name", ["quad+cube", "plane", "sphere"])
def test_gbuffer_matches_oracle(name):
    tex = np.random.default_rng(4).uniform(0.1, 0.9, (16, 16, 3)).astype(np.float32)
    if name == "quad+cube":
        w = synth.quad_cube()
    else:
        w = scenes.plane_workload(tex=tex, half=0.3, cam_eye=(0.05, 0.1, 0.6), res=48, cam_fov=70.0)
        if name == "sphere":   # 1,280 facets, silhouette against the background
            w.mesh = synth.icosphere(3, 0.25)
    got = _gbuffer_dev(w)
    want, margin = O.gbuffer(O.Scene(w))
    n = _compare_gbuffer(got, want, margin)
    assert n > 1000
    assert 0 < got[:, 7].mean() < 1 or name == "quad+cube"


def test_gbuffer_full_size_sampled():
    """The 256 x 256 camera of the 50k-triangle scene, 1500 sampled pixels by brute force."""
    w = synth.corner_50k()
    got = _gbuffer_dev(w)
    pix = np.random.default_rng(3).choice(256 * 256, 1500, replace=False)
    want, margin = O.gbuffer(O.Scene(w), pix)
    _compare_gbuffer(got[pix], want, margin)


# ------------------------------------------------------------------ L(m), L1

def _tv_dev(m, grad_scale=0.7):
    import torch
    from paper_2503_12174_amd import dpcs
    c = ctx()
    t = dev(m, torch.float32)
    loss = torch.zeros((), device="cuda")
    g = torch.full_like(t, np.nan)
    dpcs.dpcs_tv_loss(c, t, loss)
    dpcs.dpcs_tv_vjp(c, t, dev(np.float32(grad_scale)), g)
    c.synchronize()
    return float(loss.cpu()), g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (7, 1, 3), (33, 65), (50, 70, 3), (512, 512, 3), (1024, 1024)])
def test_tv_matches_oracle(shape):
    rng = np.random.default_rng(sum(shape))
    m = _f32(rng.uniform(0, 1, shape))
    m[::5] = m[::5].round(1)   # ties: sign(0) = 0 on both sides
    got_l, got_g = _tv_dev(m)
    want_l, want_g = O.tv(m)
    # FP64 sums in different orders, rounded once to FP32
    assert abs(got_l - want_l) <= 2 * U32 * abs(want_l) + 1e-30
    # the oracle adds +-1/n terms one at a time: where they cancel it leaves FP64 residue
    # of a few 2^-53 / n, the device sums the signs first and gets 0
    np.testing.assert_allclose(got_g, _f32(0.7) * want_g, rtol=2 * U32, atol=1e-12 * np.abs(want_g).max() + 1e-30)


@pytest.mark.parametrize("n", [1, 255, 256 * 256 * 3, 3 * 10 ** 6 + 17])
def test_l1_matches_oracle(n):
    import torch
    from paper_2503_12174_amd import dpcs
    rng = np.random.default_rng(n)
    a, b = _f32(rng.normal(size=n)), _f32(rng.normal(size=n))
    b[::7] = a[::7]            # equal values: sign(0) = 0
    c = ctx()
    ta, tb = dev(a, torch.float32), dev(b, torch.float32)
    loss = torch.zeros((), device="cuda")
    g = torch.full_like(ta, np.nan)
    dpcs.dpcs_l1_loss(c, ta, tb, loss)
    dpcs.dpcs_l1_vjp(c, ta, tb, dev(np.float32(1.5)), g)
    c.synchronize()
    want_l, want_g = O.l1(a, b)
    assert abs(float(loss.cpu()) - want_l) <= 2 * U32 * want_l
    np.testing.assert_allclose(g.cpu().numpy(), 1.5 * want_g, rtol=2 * U32, atol=1e-30)


def test_losses_are_deterministic():
    import torch
    from paper_2503_12174_amd import dpcs
    c = ctx()
    m = dev(np.random.default_rng(0).uniform(0, 1, (1000, 999, 3)), torch.float32)
    outs = []
    for _ in range(3):
        loss = torch.zeros((), device="cuda")
        dpcs.dpcs_tv_loss(c, m, loss)
        outs.append(float(loss.cpu()))
    assert outs[0] == outs[1] == outs[2]


# ------------------------------------------------------------------ torch Functions

def test_objective_functions_backpropagate():
    """torch.autograd through L1(D(x), target) + 0.1 TV(m) equals the oracle's gradients."""
    import torch
    from paper_2503_12174_amd import objective as Ob
    c = ctx()
    rng = np.random.default_rng(9)
    H, W = 29, 45
    img, guide, _ = _case(H, W, 8, 77)
    tgt = _f32(rng.uniform(0, 1, (H, W, 3)))
    m = _f32(rng.uniform(0, 1, (16, 12, 3)))
    cfg = Ob.DenoiseConfig()
    x = dev(img, torch.float32).requires_grad_(True)
    mm = dev(m, torch.float32).requires_grad_(True)
    loss = Ob.l1(c, Ob.denoise(c, x, dev(guide, torch.float32), cfg), dev(tgt, torch.float32)) + 0.1 * Ob.tv(c, mm)
    loss.backward()
    coef = _f32(cfg.guide)
    sp = float(np.float32(cfg.spatial))
    d = O.denoise(img, guide, coef, sp, cfg.radius)
    l1, g1 = O.l1(d, tgt)
    tvl, gt = O.tv(m)
    # |D_dev - D| is within the forward bound; the mean moves by at most that much
    assert abs(float(loss.detach().cpu()) - (l1 + 0.1 * tvl)) <= _fwd_bound(cfg.radius, 1.0) + 1e-6
    np.testing.assert_allclose(mm.grad.cpu().numpy(), _f32(0.1) * gt, rtol=4 * U32, atol=1e-12)
    # the L1 gradient's signs: the device's D(x) takes the oracle's decision everywhere here
    dd = _denoise_dev(img, guide, coef, sp, cfg.radius)
    assert np.array_equal(np.sign(dd - tgt), np.sign(d - tgt))
    gx = O.denoise_vjp(g1, guide, coef, sp, cfg.radius)
    np.testing.assert_allclose(x.grad.cpu().numpy(), gx, rtol=0, atol=_tol(_vjp_bound(cfg.radius, np.abs(g1).max()), gx))
