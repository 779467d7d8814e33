"""Thin optimisation drivers over the differentiable renderer (paper Sec. 3.2).

compensate()  projector compensation, Eq. 13: find I_p whose rendering matches a
              target camera image, by Adam on an L2 loss, I_p clamped to [0, 1]
compensate_morphing()  the same on a moving surface, frame by frame (Sec. 4.4), the
              BVH refitted on the device for each frame's vertex positions
refine_camera()  camera-pose refinement (R_c, t_c of theta, Sec. 3.2): a rotation
              vector and a translation offset about the calibrated pose, by Adam on an L2
              loss against captures, the maps and responses held
fit()         scene-parameter fit, Eq. 9: BRDF maps and PRF/CRF scalars from image
              pairs, with the paper's constraints on gamma_p, gamma_c, w
              (Sec. 3.2: gamma_p in [2, 3], gamma_c in [1/3, 1], w in (0.2, 2.5));
              objective "l2": mean squared error of the raw renderings; "paper": Eq. 9
              as written, the L1 distance of denoised renderings (Eq. 11, guided by the
              scene's first-hit features under the current albedo) plus tv_weight times
              the total variation of the three BRDF maps
Each optimisation step uses its own Philox seed (base seed + step), so a run is
reproducible and resumable from any step.
"""
from __future__ import annotations

import copy

import torch

from . import dpcs
from . import objective as Ob
from .autograd import render, scalars_from


def compensate(ctx, scene, cfg, target, albedo, roughness, specular, steps=100, lr=0.01, init=0.5,
               base_seed=0, callback=None):
    scal = scalars_from(cfg)
    H, W = cfg.projector.height, cfg.projector.width
    ip = torch.full((H, W, 3), init, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([ip], lr=lr)
    losses = []
    for k in range(steps):
        c = copy.copy(cfg)
        c.seed = base_seed + k
        out = render(ctx, scene, c, ip, albedo, roughness, specular, scal)
        loss = ((out - target) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            ip.clamp_(0.0, 1.0)
        losses.append(float(loss.detach()))
        if callback:
            callback(k, losses[-1], ip)
    return ip.detach(), losses


def compensate_morphing(ctx, scene, cfg, frames, target, albedo, roughness, specular, steps_per_frame=10,
                        lr=0.01, init=0.5, base_seed=0):
    """Projector compensation on a moving surface (Sec. 4.4): for each frame's vertex
    positions (device tensors on the scene's topology) the scene's BVH is refitted on
    the device and the projector image, warm-started from the previous frame, takes
    steps_per_frame Adam steps of Eq. 13 toward the target.  Returns the images and
    the per-frame losses."""
    scal = scalars_from(cfg)
    H, W = cfg.projector.height, cfg.projector.width
    ip = torch.full((H, W, 3), init, device="cuda", requires_grad=True)
    images, losses = [], []
    for f, pos in enumerate(frames):
        scene.refit(pos)
        opt = torch.optim.Adam([ip], lr=lr)
        fl = []
        for k in range(steps_per_frame):
            c = copy.copy(cfg)
            c.seed = base_seed + f * steps_per_frame + k
            out = render(ctx, scene, c, ip, albedo, roughness, specular, scal)
            loss = ((out - target) ** 2).mean()
            opt.zero_grad()
            loss.backward()
            opt.step()
            with torch.no_grad():
                ip.clamp_(0.0, 1.0)
            fl.append(float(loss.detach()))
        images.append(ip.detach().clone())
        losses.append(fl)
    return images, losses


def project_constraints(scal: torch.Tensor, clamp_gamma_p=True):
    with torch.no_grad():
        if clamp_gamma_p:
            scal[0:3].clamp_(2.0, 3.0)
        scal[12:15].clamp_(1.0 / 3.0, 1.0)
        scal[15:18].clamp_(0.2 + 1e-4, 2.5 - 1e-4)


def pose_from(omega, dt, R0, t0):
    """The 12 pose values (R row-major, t) of R = exp([omega]x) R0, t = t0 + dt (Rodrigues),
    differentiable in omega and dt (float64 tensors on the host)."""
    th = torch.sqrt((omega * omega).sum() + 1e-30)
    k = omega / th
    Kx = torch.zeros((3, 3), dtype=omega.dtype)
    Kx = Kx.index_put((torch.tensor([0, 0, 1, 1, 2, 2]), torch.tensor([1, 2, 0, 2, 0, 1])),
                      torch.stack([-k[2], k[1], k[2], -k[0], -k[1], k[0]]))
    Rw = torch.eye(3, dtype=omega.dtype) + torch.sin(th) * Kx + (1 - torch.cos(th)) * (Kx @ Kx)
    R = Rw @ torch.as_tensor(R0, dtype=omega.dtype)
    t = torch.as_tensor(t0, dtype=omega.dtype) + dt
    return torch.cat([R.reshape(-1), t])


def refine_camera(ctx, scene, cfg, images, targets, albedo, roughness, specular, steps=40, lr=2e-3, base_seed=0,
                  scalars=None, edge_density=4.0):
    """Refine the camera pose about cfg.camera so renderings of `images` match `targets`.
    The pose gradient has its interior part and, with edge_density > 0 (points per pixel of
    edge length), the boundary part where silhouettes, creases and seams move in the image.
    Returns (R, t) and the losses."""
    omega = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    dt = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([omega, dt], lr=lr)
    scal = scalars_from(cfg) if scalars is None else scalars
    R0, t0 = cfg.camera.R, cfg.camera.t
    losses = []
    for k in range(steps):
        c = copy.copy(cfg)
        c.seed = base_seed + k
        pose = pose_from(omega, dt, R0, t0)
        loss = 0.0
        for ip, tgt in zip(images, targets):
            out = render(ctx, scene, c, ip, albedo, roughness, specular, scal, camera_pose=pose.float(),
                         camera_edge_density=edge_density)
            loss = loss + ((out - tgt) ** 2).mean()
        loss = loss / len(images)
        opt.zero_grad()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    pose = pose_from(omega, dt, R0, t0).detach().numpy()
    return (pose[:9].reshape(3, 3), pose[9:]), losses


def _l2_step_batched(srv, scene, c, images, targets, alb, rough, spec, scal, first_id):
    """Forward + VJP of the mean L2 loss over all (image, target) pairs as compensation
    requests of the request loop, which packs them into shared launch waves; the maps'
    and scalars' gradients (averaged over the pairs) land in their .grad.  Returns the loss."""
    p = dpcs.params_from(c, alb.detach(), rough.detach(), spec.detach(), device_scalars=scal.detach())
    outs, grads = [], []
    for b, (ip, tgt) in enumerate(zip(images, targets)):
        out = torch.empty_like(tgt)
        g = dict(d_albedo=torch.zeros_like(alb), d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                 d_scalars=torch.zeros_like(scal))
        st = srv.submit(first_id + b, scene, p, ip.contiguous(), out, target=tgt.contiguous(), grads=g)
        if st != dpcs.OK:
            raise dpcs.DpcsError(f"fit step request {b}: status {st}")
        outs.append(out)
        grads.append(g)
    done = 0
    while done < len(images):
        for _, st, _ in srv.poll():
            if st != dpcs.OK:
                raise dpcs.DpcsError(f"fit step request failed: status {st}")
            done += 1
    n = float(len(images))
    for t, key in ((alb, "d_albedo"), (rough, "d_roughness"), (spec, "d_specular"), (scal, "d_scalars")):
        t.grad = sum(g[key] for g in grads) / n
    return sum(((o - t) ** 2).mean() for o, t in zip(outs, targets)) / n


def fit(ctx, scene, cfg, images, targets, steps=50, lr=0.02, base_seed=0, clamp_gamma_p=True, init=None,
        objective="l2", tv_weight=0.0, denoise: Ob.DenoiseConfig | None = None, batched=True):
    """Fit albedo/roughness/specular maps and the 18 response scalars to (image, target) pairs.
    With the L2 objective and several pairs (batched=True), each step runs the pairs as
    compensation requests of one request loop, so their samples share launch waves
    instead of one render + VJP per pair; the same Philox samples either way."""
    if objective not in ("l2", "paper"):
        raise ValueError("objective must be 'l2' or 'paper'")
    th, tw = cfg.albedo.shape[:2]
    dev = lambda x: torch.as_tensor(x, dtype=torch.float32, device="cuda").clone().requires_grad_(True)
    init = init or {}
    alb = dev(init.get("albedo", torch.full((th, tw, 3), 0.5)))
    rough = dev(init.get("roughness", torch.full((th, tw), 0.5)))
    spec = dev(init.get("specular", torch.full((th, tw), 0.5)))
    scal = scalars_from(cfg).clone().requires_grad_(True)
    opt = torch.optim.Adam([alb, rough, spec, scal], lr=lr)
    losses = []
    srv = None
    if batched and objective == "l2" and len(images) > 1:
        paths = sum(int(t.shape[0]) * int(t.shape[1]) for t in targets) * cfg.spp
        # queues for every pair's paths in one wave (~600 B per path) within a quarter of the budget
        srv = dpcs.Server(ctx, budget_bytes=max(1 << 30, 4 * 640 * paths + (256 << 20)), max_slots=len(images))
    try:
        for k in range(steps):
            c = copy.copy(cfg)
            c.seed = base_seed + k
            if srv is not None:
                opt.zero_grad()
                loss = _l2_step_batched(srv, scene, c, images, targets, alb, rough, spec, scal, k * len(images))
                if tv_weight:
                    tv = tv_weight * (Ob.tv(ctx, alb) + Ob.tv(ctx, rough) + Ob.tv(ctx, spec))
                    tv.backward()
                    loss = loss + tv.detach()
                opt.step()
                with torch.no_grad():
                    alb.clamp_(0.0, 1.0)
                    rough.clamp_(0.05, 1.0)
                    spec.clamp_(0.0, 1.0)
                project_constraints(scal, clamp_gamma_p)
                losses.append(float(loss))
                continue
            _fit_step(ctx, scene, c, images, targets, alb, rough, spec, scal, opt, objective, tv_weight, denoise,
                      clamp_gamma_p, losses)
    finally:
        if srv is not None:
            srv.close()
    return dict(albedo=alb.detach(), roughness=rough.detach(), specular=spec.detach(), scalars=scal.detach()), losses


def _fit_step(ctx, scene, c, images, targets, alb, rough, spec, scal, opt, objective, tv_weight, denoise,
              clamp_gamma_p, losses):
    """One step of fit, one autograd render + VJP per pair."""
    loss = 0.0
    guide = None
    if objective == "paper":   # guide features under the current albedo (a constant of D)
        guide = Ob.gbuffer(ctx, scene, dpcs.params_from(c, alb.detach(), rough.detach(), spec.detach()))
    for ip, tgt in zip(images, targets):
        out = render(ctx, scene, c, ip, alb, rough, spec, scal)
        if objective == "paper":
            loss = loss + Ob.l1(ctx, Ob.denoise(ctx, out, guide, denoise), tgt)
        else:
            loss = loss + ((out - tgt) ** 2).mean()
    loss = loss / len(images)
    if tv_weight:
        loss = loss + tv_weight * (Ob.tv(ctx, alb) + Ob.tv(ctx, rough) + Ob.tv(ctx, spec))
    opt.zero_grad()
    loss.backward()
    opt.step()
    with torch.no_grad():
        alb.clamp_(0.0, 1.0)
        rough.clamp_(0.05, 1.0)
        spec.clamp_(0.0, 1.0)
    project_constraints(scal, clamp_gamma_p)
    losses.append(float(loss.detach()))
