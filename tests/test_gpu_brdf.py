"""The device BRDF, its derivatives, the bounce density and the bounce sampler (through
dpcs_debug_brdf) against the oracle's FP64 routines, row by row."""
import numpy as np
import pytest

from oracle import oracle as O

from .gpu_util import ctx, dev

pytestmark = pytest.mark.gpu

# Relative tolerance for everything that goes through the GGX distribution D: the oracle
# writes D's denominator as (n.h)^2 (alpha^2 - 1) + 1, which cancels near the lobe peak,
# so its relative rounding there is ~2u/alpha^2 per rounding (u = 2^-53, alpha >= 1e-3:
# ~2e-10); the device forms sin^2 from |n x v|^2, without the cancellation.  A few such
# roundings stay below 1e-8.
RTOL_D = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    O.build(force=False)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _rows(rng, m):
    """m input rows: random frames, directions on both sides of the surface, the
    specular peak, grazing directions, roughness under the alpha floor."""
    n = _unit(rng.normal(size=(m, 3)))
    wo = _unit(rng.normal(size=(m, 3)))
    wo = np.where((np.sum(wo * n, 1) < 0)[:, None] & (rng.uniform(size=(m, 1)) < 0.9), -wo, wo)
    wi = _unit(rng.normal(size=(m, 3)))
    k = m // 8
    wi[:k] = 2.0 * np.sum(wo[:k] * n[:k], 1)[:, None] * n[:k] - wo[:k]          # mirror direction
    g = _unit(np.cross(n[k:2 * k], rng.normal(size=(k, 3))))                      # grazing
    wi[k:2 * k] = _unit(g + 1e-4 * n[k:2 * k])
    wi[2 * k:3 * k] = wo[2 * k:3 * k]                                             # wi = wo
    alb = rng.uniform(0, 1, (m, 3))
    r = rng.uniform(0, 1, m)
    r[3 * k:4 * k] = rng.uniform(0, 0.03, k)                                      # r^2 below the floor
    sp = rng.uniform(0, 1, m)
    u = rng.uniform(0, 1, (m, 3))
    return np.concatenate([n, wo, wi, alb, r[:, None], sp[:, None], u], 1)


def _device(kind, x):
    import torch
    from paper_2503_12174_amd import dpcs
    c = ctx()
    out = torch.zeros((x.shape[0], 11), dtype=torch.float64, device="cuda")
    dpcs.dpcs_debug_brdf(c, kind, dev(x, torch.float64), out)
    c.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
def test_brdf_matches_oracle(kind):
    rng = np.random.default_rng(11 + kind)
    x = _rows(rng, 2048)
    y = _device(kind, x)
    ref = np.array([O.brdf(kind, r[0:3], r[3:6], r[6:9], r[9:12], r[12], r[13]) for r in x])
    pdf = np.array([O.pdf(kind, r[0:3], r[3:6], r[6:9], r[12]) for r in x])
    # f and both derivatives: FP64 on both sides, different but equivalent arithmetic
    for c in range(5):
        scale = np.abs(ref[:, c]).max() + 1e-300
        np.testing.assert_allclose(y[:, c], ref[:, c], rtol=RTOL_D, atol=1e-12 * scale, err_msg=f"column {c}")
    np.testing.assert_allclose(y[:, 5], pdf, rtol=RTOL_D, atol=1e-12 * (np.abs(pdf).max() + 1e-300))
    # the forward's evaluation and the replay's agree bit for bit
    assert np.array_equal(y[:, 10], y[:, 0])
    if kind == 0:
        assert np.all(y[:, 3] == 0) and np.all(y[:, 4] == 0)


@pytest.mark.parametrize("kind", [0, 1])
def test_bounce_sampler_matches_oracle(kind):
    rng = np.random.default_rng(21 + kind)
    x = _rows(rng, 1024)
    y = _device(kind, x)
    for row, out in zip(x, y):
        wi, pdf = O.sample(kind, row[0:3], row[3:6], row[12], row[14:17][None, :])
        np.testing.assert_allclose(out[6:9], wi[0], rtol=0, atol=1e-12)
        np.testing.assert_allclose(out[9], pdf[0], rtol=RTOL_D, atol=1e-300)
    # a sampled direction is a unit vector
    np.testing.assert_allclose(np.linalg.norm(y[:, 6:9], axis=1), 1.0, atol=1e-12)


def test_brdf_rejects_bad_kind():
    import torch
    from paper_2503_12174_amd import dpcs
    c = ctx()
    x = torch.zeros((4, 17), dtype=torch.float64, device="cuda")
    out = torch.zeros((4, 11), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        dpcs.dpcs_debug_brdf(c, 7, x, out)
