"""torch.autograd wrapper and the thin optimisation drivers on the GPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes
from .gpu_util import compare_grads, ctx, dev

pytestmark = pytest.mark.gpu


def _tensors(w):
    import torch
    f = torch.float32
    return (dev(w.proj_image, f).requires_grad_(True), dev(w.albedo, f).requires_grad_(True),
            dev(w.roughness, f).requires_grad_(True), dev(w.specular, f).requires_grad_(True))


def test_autograd_backward_matches_oracle_vjp():
    from paper_2503_12174_amd import autograd, dpcs
    w = scenes.c3_ggx(spp=4, seed=31, max_depth=3)
    w.clip, w.clip_k = True, 0.5
    sc = O.Scene(w)
    allc = (O.render(sc, want=("margin_clip",))["margin_clip"] >= 1).all(1)
    G = np.random.default_rng(0).normal(size=(64 * 64, 3))
    G[~allc] = 0
    G = G.reshape(64, 64, 3)
    ref = O.render_vjp(sc, G)
    scene = dpcs.Scene(ctx(), w.mesh)
    ip, alb, rough, spec = _tensors(w)
    scal = autograd.scalars_from(w).requires_grad_(True)
    out = autograd.render(ctx(), scene, w, ip, alb, rough, spec, scal)
    (out * dev(G, out.dtype)).sum().backward()
    s = scal.grad.cpu().numpy()
    gpu = dict(Ip=ip.grad.cpu().numpy(), albedo=alb.grad.cpu().numpy(), roughness=rough.grad.cpu().numpy(),
               specular=spec.grad.cpu().numpy(), prf_gamma=s[0:3], prf_mix=s[3:12].reshape(3, 3),
               crf_gamma=s[12:15], white_balance=s[15:18])
    compare_grads(gpu, ref)


def test_compensation_reduces_the_loss():
    """Eq. 13 by Adam: a 128^2 compensation on a 10k-triangle corner."""
    import torch
    from paper_2503_12174_amd import drivers, dpcs
    w = synth.corner_200k(spp=4, n_quads=50, res=128)
    scene = dpcs.Scene(ctx(), w.mesh)
    f = torch.float32
    target = dev(synth.blob_image(128, 128, 402, lo=0.1, hi=0.9), f)
    ip, losses = drivers.compensate(ctx(), scene, w, target, dev(w.albedo, f), dev(w.roughness, f),
                                    dev(w.specular, f), steps=30, lr=0.05)
    # regions outside the projector frustum or in shadow cannot match the target: a floor remains
    assert losses[-1] < 0.75 * losses[0], losses
    assert all(b <= a * 1.02 for a, b in zip(losses, losses[1:])), losses
    assert float(ip.min()) >= 0.0 and float(ip.max()) <= 1.0


_FIT = {}


def _fit_problem():
    """Targets rendered by the FP64 oracle from hidden maps and responses (cached)."""
    if not _FIT:
        truth = synth.fit_truth(301)
        imgs = synth.fit_images(0, count=2)
        targets = []
        for im in imgs:
            tw = synth.fit_scene(spp=64)
            for k, v in truth.items():
                setattr(tw, {"roughness": "roughness", "specular": "specular"}.get(k, k), v)
            targets.append(O.render(O.Scene(tw, proj_image=im), want=("Ic",))["Ic"].reshape(64, 64, 3))
        _FIT.update(imgs=imgs, targets=targets)
    return _FIT["imgs"], _FIT["targets"]


def test_scene_fit_reduces_the_loss_on_oracle_targets():
    """Eq. 9 scene-parameter fit from the initial guess with fwd + VJP steps."""
    import torch
    from paper_2503_12174_amd import drivers, dpcs
    imgs, targets = _fit_problem()
    w = synth.fit_scene(spp=8)
    scene = dpcs.Scene(ctx(), w.mesh)
    f = torch.float32
    params, losses = drivers.fit(ctx(), scene, w, [dev(i, f) for i in imgs], [dev(t, f) for t in targets],
                                 steps=25, lr=0.03, clamp_gamma_p=False)
    assert losses[-1] < 0.5 * losses[0], losses


def test_batched_fit_steps_equal_one_render_per_pair():
    """The L2 fit with its pairs batched through the request loop computes the same
    gradients as one autograd render + VJP per pair (same Philox samples; the two differ
    only in summation order), and the same losses over a few steps, with and without the
    TV term.  (The maps after several Adam steps are not compared: Adam moves a texel whose
    gradient is near zero by up to the learning rate either way.)"""
    import copy

    import torch
    from paper_2503_12174_amd import autograd, drivers, dpcs
    imgs, targets = _fit_problem()
    w = synth.fit_scene(spp=8)
    scene = dpcs.Scene(ctx(), w.mesh)
    f = torch.float32
    ims, tgs = [dev(i, f) for i in imgs], [dev(t, f) for t in targets]
    th, tw = w.albedo.shape[:2]
    mk = lambda v, shape: torch.full(shape, v, dtype=f, device="cuda").requires_grad_(True)
    # one step's gradients
    grads = {}
    for batched in (True, False):
        alb, rough, spec = mk(0.5, (th, tw, 3)), mk(0.5, (th, tw)), mk(0.5, (th, tw))
        scal = autograd.scalars_from(w).clone().requires_grad_(True)
        c = copy.copy(w)
        c.seed = 7
        if batched:
            srv = dpcs.Server(ctx(), budget_bytes=1 << 30, max_slots=len(ims))
            loss = drivers._l2_step_batched(srv, scene, c, ims, tgs, alb, rough, spec, scal, 0)
            srv.close()
        else:
            loss = sum(((autograd.render(ctx(), scene, c, ip, alb, rough, spec, scal) - t) ** 2).mean()
                       for ip, t in zip(ims, tgs)) / len(ims)
            loss.backward()
        grads[batched] = [float(loss)] + [t.grad.cpu().numpy() for t in (alb, rough, spec, scal)]
    np.testing.assert_allclose(grads[True][0], grads[False][0], rtol=1e-5)
    for k, name in enumerate(("albedo", "roughness", "specular", "scalars")):
        x, y = grads[True][k + 1], grads[False][k + 1]
        np.testing.assert_allclose(x, y, rtol=1e-3, atol=1e-4 * np.abs(y).max(), err_msg=name)
    # the fit's losses step by step
    for tv in (0.0, 0.02):
        _, la = drivers.fit(ctx(), scene, w, ims, tgs, steps=4, lr=0.03, clamp_gamma_p=False, tv_weight=tv,
                            batched=True)
        _, lb = drivers.fit(ctx(), scene, w, ims, tgs, steps=4, lr=0.03, clamp_gamma_p=False, tv_weight=tv,
                            batched=False)
        np.testing.assert_allclose(la, lb, rtol=1e-4)


def test_scene_fit_with_the_papers_objective():
    """Eq. 9 as written: L1 of denoised renderings (Eq. 11) + lambda_reg L(m).  The loss
    falls, and a large lambda_reg leaves smoother maps than lambda_reg = 0."""
    import torch
    from paper_2503_12174_amd import drivers, dpcs
    from paper_2503_12174_amd import objective as Ob
    imgs, targets = _fit_problem()
    w = synth.fit_scene(spp=8)
    scene = dpcs.Scene(ctx(), w.mesh)
    f = torch.float32
    tv = {}
    for lam in (0.0, 0.05):
        params, losses = drivers.fit(ctx(), scene, w, [dev(i, f) for i in imgs], [dev(t, f) for t in targets],
                                     steps=25, lr=0.03, clamp_gamma_p=False, objective="paper", tv_weight=lam)
        assert all(np.isfinite(losses))
        # the maps start constant (L(m) = 0), so with lambda_reg > 0 the total falls less
        assert losses[-1] < (0.8 if lam == 0.0 else 0.95) * losses[0], (lam, losses)
        tv[lam] = sum(float(Ob.tv(ctx(), params[k])) for k in ("albedo", "roughness", "specular"))
    assert tv[0.05] < tv[0.0], tv
