"""torch.autograd.Function over dpcs_render / dpcs_render_vjp (argument marshalling only).

Forward keeps each camera sample's radiance and the path records (hit leaf and
shadow visibility per vertex, 4 B) so backward replays the same Philox paths
without recomputing the forward samples or tracing.  Differentiable inputs: projector
image, albedo, roughness, specular maps, the 18 response scalars
(gamma_p[3], M[9], gamma_c[3], w[3]) as one device tensor, optionally the metallic
map and the normal map (stored values) of the principled BRDF, and optionally the
camera pose (R_c row-major then t_c, 12 values; read back to the host for each call;
its gradient is the interior part, plus the boundary part at the images of mesh edges
when camera_edge_density > 0).
"""
from __future__ import annotations

import torch

from . import dpcs


def scalars_from(w, device="cuda") -> torch.Tensor:
    """The 18 differentiable response scalars of a workload-like object as a device tensor."""
    import numpy as np
    v = np.concatenate([np.ravel(w.prf_gamma), np.ravel(w.prf_mix), np.ravel(w.crf_gamma), np.ravel(w.white_balance)])
    return torch.tensor(v, dtype=torch.float32, device=device)


def _with_pose(cfg, pose):
    """cfg with its camera's R, t replaced by the 12 values of pose (None: unchanged)."""
    if pose is None:
        return cfg
    import copy

    import numpy as np
    v = pose.detach().double().cpu().numpy()
    c = copy.copy(cfg)
    cam = cfg.camera
    c.camera = type(cam)(cam.K, v[:9].reshape(3, 3), v[9:12], cam.width, cam.height)
    return c


class DPCSRender(torch.autograd.Function):
    @staticmethod
    def forward(fctx, proj_image, albedo, roughness, specular, scalars, metallic, normal_map, camera_pose, ctx, scene,
                cfg, camera_edge_density):
        proj_image, albedo = proj_image.contiguous(), albedo.contiguous()
        roughness, specular, scalars = roughness.contiguous(), specular.contiguous(), scalars.contiguous()
        metallic = None if metallic is None else metallic.contiguous()
        normal_map = None if normal_map is None else normal_map.contiguous()
        cfg = _with_pose(cfg, camera_pose)
        p = dpcs.params_from(cfg, albedo, roughness, specular, device_scalars=scalars, metallic=metallic,
                             normal_map=normal_map)
        H, W = p.camera.height, p.camera.width
        out = torch.empty((H, W, 3), dtype=torch.float32, device=proj_image.device)
        L = torch.empty((H, W, p.spp, 3), dtype=torch.float32, device=proj_image.device)
        rec = torch.empty((H, W, p.spp, p.max_depth), dtype=torch.int32, device=proj_image.device)
        dpcs.dpcs_render(ctx, scene, p, proj_image, out, sample_radiance=L, path_records=rec)
        fctx.save_for_backward(proj_image, albedo, roughness, specular, scalars, metallic, normal_map, L, rec)
        fctx.ctx, fctx.scene, fctx.cfg = ctx, scene, cfg
        fctx.pose_like = None if camera_pose is None else camera_pose.detach()
        fctx.edge_density = float(camera_edge_density)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        proj_image, albedo, roughness, specular, scalars, metallic, normal_map, L, rec = fctx.saved_tensors
        p = dpcs.params_from(fctx.cfg, albedo, roughness, specular, device_scalars=scalars, metallic=metallic,
                             normal_map=normal_map)
        need = fctx.needs_input_grad
        z = lambda t, k: torch.empty_like(t) if (t is not None and need[k]) else None
        d_proj, d_alb, d_rough, d_spec = z(proj_image, 0), z(albedo, 1), z(roughness, 2), z(specular, 3)
        d_scal, d_metal, d_nmap = z(scalars, 4), z(metallic, 5), z(normal_map, 6)
        pose = fctx.pose_like
        d_cam = torch.zeros(12, dtype=torch.float32, device=proj_image.device) if (pose is not None and need[7]) else None
        dpcs.dpcs_render_vjp(fctx.ctx, fctx.scene, p, proj_image, grad_out.contiguous(), sample_radiance=L,
                             path_records=rec, d_proj_image=d_proj, d_albedo=d_alb, d_roughness=d_rough, d_specular=d_spec,
                             d_scalars=d_scal, d_metallic=d_metal, d_normal_map=d_nmap, d_camera=d_cam,
                             camera_edge_density=fctx.edge_density if d_cam is not None else 0.0)
        if d_cam is not None:
            d_cam = d_cam.to(device=pose.device, dtype=pose.dtype)
        return d_proj, d_alb, d_rough, d_spec, d_scal, d_metal, d_nmap, d_cam, None, None, None, None


def render(ctx, scene, cfg, proj_image, albedo, roughness, specular, scalars, metallic=None, normal_map=None,
           camera_pose=None, camera_edge_density=0.0):
    """I_c = R(I_p, theta) (paper Eq. 7) with gradients for every tensor argument
    (camera_pose: 12 values, R_c row-major then t_c, overriding cfg's camera;
    camera_edge_density: points per pixel of edge length for the pose gradient's boundary
    part, 0: interior part only)."""
    return DPCSRender.apply(proj_image, albedo, roughness, specular, scalars, metallic, normal_map, camera_pose, ctx,
                            scene, cfg, camera_edge_density)
