"""ctypes binding of libdpcs.so (include/dpcs.h): argument marshalling only.

Every computation happens in the HIP library; this module converts torch tensors
to device pointers, mirrors the C structs and raises on non-OK statuses.  Loading
fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpcs.so")

OK, E_INVALID, E_OOM, E_DEVICE, E_UNSUPPORTED, E_BUSY, E_REJECTED = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "OK", -1: "INVALID", -2: "OOM", -3: "DEVICE", -4: "UNSUPPORTED", -5: "BUSY", -6: "REJECTED"}
LAMBERT, GGX = 0, 1
NUM_SCALARS = 18
NOALLOC_SCRATCH_BYTES = 64 << 20


class DpcsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dpcs status {STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("positions", C.c_void_p), ("num_vertices", C.c_int32), ("triangles", C.c_void_p),
                ("num_triangles", C.c_int32), ("corner_uvs", C.c_void_p), ("emission", C.c_void_p),
                ("bvh_kind", C.c_int32)]


BVH_LBVH, BVH_SAH, BVH_PLOC = 0, 1, 2


class SceneInfo(C.Structure):
    _fields_ = [("num_triangles", C.c_int32), ("num_nodes", C.c_int32), ("max_depth", C.c_int32),
                ("wide_nodes", C.c_int32), ("device_bytes", C.c_int64), ("build_ms", C.c_double),
                ("bbox_lo", C.c_float * 3), ("bbox_hi", C.c_float * 3), ("tmin", C.c_float)]


class Pinhole(C.Structure):
    _fields_ = [("K", C.c_double * 9), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("width", C.c_int32), ("height", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("camera", Pinhole), ("projector", Pinhole), ("brdf", C.c_int32),
                ("albedo", C.c_void_p), ("roughness", C.c_void_p), ("specular", C.c_void_p),
                ("tex_w", C.c_int32), ("tex_h", C.c_int32),
                ("prf_gamma", C.c_float * 3), ("prf_gain", C.c_float), ("prf_mix", C.c_float * 9),
                ("crf_gamma", C.c_float * 3), ("crf_gain", C.c_float), ("white_balance", C.c_float * 3),
                ("device_scalars", C.c_void_p), ("env_radiance", C.c_float * 3),
                ("clip_enable", C.c_int32), ("clip_k", C.c_float), ("spp", C.c_int32), ("max_depth", C.c_int32),
                ("seed", C.c_uint64), ("sample_offset", C.c_uint32), ("metallic", C.c_void_p),
                ("normal_map", C.c_void_p)]


class RenderAux(C.Structure):
    _fields_ = [("linear", C.c_void_p), ("sample_radiance", C.c_void_p), ("hit_prims", C.c_void_p),
                ("path_records", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("d_proj_image", C.c_void_p), ("d_albedo", C.c_void_p), ("d_roughness", C.c_void_p),
                ("d_specular", C.c_void_p), ("d_scalars", C.c_void_p), ("d_metallic", C.c_void_p),
                ("d_normal_map", C.c_void_p), ("d_camera", C.c_void_p), ("camera_edge_density", C.c_double)]


NUM_STAGES = 9
STAGES = ["raygen", "trace", "shade", "shadow", "finalize", "adj_pixel", "adj_shade", "adj_shadow", "other"]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * NUM_STAGES), ("ms", C.c_double * NUM_STAGES),
                ("items", C.c_int64 * NUM_STAGES), ("nodes", C.c_int64 * NUM_STAGES),
                ("tris", C.c_int64 * NUM_STAGES)]

    def as_dict(self):
        return {name: dict(launches=self.launches[k], ms=self.ms[k], items=self.items[k], nodes=self.nodes[k],
                           tris=self.tris[k]) for k, name in enumerate(STAGES)}


class Request(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("params", RenderParams), ("proj_image", C.c_void_p),
                ("out_image", C.c_void_p), ("grad_image", C.c_void_p), ("target", C.c_void_p),
                ("grads", C.POINTER(Grads)), ("request_id", C.c_uint64), ("input_stream", C.c_void_p)]


class DenoiseParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("guide_channels", C.c_int32), ("radius", C.c_int32),
                ("spatial", C.c_float), ("guide", C.c_float * 8)]


def denoise_params(width: int, height: int, radius: int, spatial: float, guide=()) -> DenoiseParams:
    """Window radius r, a_s = 1 / (2 sigma_s^2), and a_k = 1 / (2 sigma_k^2) per guide channel."""
    g = [float(x) for x in guide]
    if len(g) > 8:
        raise ValueError("at most 8 guide channels")
    p = DenoiseParams()
    p.width, p.height, p.radius, p.spatial = int(width), int(height), int(radius), float(spatial)
    p.guide_channels = len(g)
    for k, x in enumerate(g):
        p.guide[k] = x
    return p


# every symbol the header declares (a test checks the library exports all of them)
SYMBOLS = ["dpcs_context_create", "dpcs_context_destroy", "dpcs_last_error", "dpcs_context_synchronize",
           "dpcs_context_set_capacity", "dpcs_scene_create", "dpcs_scene_get_info", "dpcs_scene_destroy",
           "dpcs_render", "dpcs_render_vjp", "dpcs_debug_intersect", "dpcs_debug_philox", "dpcs_debug_brdf",
           "dpcs_context_set_profiling", "dpcs_context_get_profile", "dpcs_server_create",
           "dpcs_server_submit", "dpcs_server_poll", "dpcs_server_stats", "dpcs_server_destroy",
           "dpcs_denoise", "dpcs_denoise_vjp", "dpcs_render_gbuffer", "dpcs_tv_loss", "dpcs_tv_vjp",
           "dpcs_l1_loss", "dpcs_l1_vjp", "dpcs_render_noalloc", "dpcs_scene_refit"]

_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_12174_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, S, I32, I64 = C.c_void_p, C.c_int32, C.c_int32, C.c_int64
        sig = {
            "dpcs_context_create": ([I32, P, C.c_size_t, C.POINTER(P)], S),
            "dpcs_context_destroy": ([P], None),
            "dpcs_last_error": ([P], C.c_char_p),
            "dpcs_context_synchronize": ([P], S),
            "dpcs_context_set_capacity": ([P, I64], S),
            "dpcs_scene_create": ([P, C.POINTER(MeshDesc), C.POINTER(P)], S),
            "dpcs_scene_get_info": ([P, C.POINTER(SceneInfo)], S),
            "dpcs_scene_destroy": ([P], S),
            "dpcs_scene_refit": ([P, P, P], S),
            "dpcs_render": ([P, P, C.POINTER(RenderParams), P, P, C.POINTER(RenderAux)], S),
            "dpcs_render_noalloc": ([P, P, C.POINTER(RenderParams), P, P, C.POINTER(RenderAux)], S),
            "dpcs_render_vjp": ([P, P, C.POINTER(RenderParams), P, P, P, P, C.POINTER(Grads)], S),
            "dpcs_debug_intersect": ([P, P, P, I64, I32, P, P, P, P], S),
            "dpcs_debug_philox": ([P, C.c_uint64, P, I64, P], S),
            "dpcs_debug_brdf": ([P, I32, P, I64, P], S),
            "dpcs_context_set_profiling": ([P, I32], S),
            "dpcs_context_get_profile": ([P, C.POINTER(Profile)], S),
            "dpcs_server_create": ([P, C.c_size_t, I32, C.POINTER(P)], S),
            "dpcs_server_submit": ([P, C.POINTER(Request)], S),
            "dpcs_server_poll": ([P, P, P, P, I32], I32),
            "dpcs_server_stats": ([P, P], S),
            "dpcs_server_destroy": ([P], S),
            "dpcs_denoise": ([P, C.POINTER(DenoiseParams), P, P, P], S),
            "dpcs_denoise_vjp": ([P, C.POINTER(DenoiseParams), P, P, P], S),
            "dpcs_render_gbuffer": ([P, P, C.POINTER(RenderParams), P], S),
            "dpcs_tv_loss": ([P, P, I32, I32, I32, P], S),
            "dpcs_tv_vjp": ([P, P, I32, I32, I32, P, P], S),
            "dpcs_l1_loss": ([P, P, P, I64, P], S),
            "dpcs_l1_vjp": ([P, P, P, I64, P, P], S),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(t):
    """Device (or host) pointer of a contiguous tensor / array; None stays NULL."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return t.data_ptr()
    return t.ctypes.data


class Context:
    """dpcs_context on one device and the torch stream current at creation."""

    def __init__(self, device: int = 0, stream=None, scratch_limit: int = 0, capacity: int | None = None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = lib().dpcs_context_create(device, C.c_void_p(stream.cuda_stream), scratch_limit, C.byref(h))
        if st != OK:
            raise DpcsError(st, "dpcs_context_create")
        self.h = h
        if capacity is not None:
            self.check(lib().dpcs_context_set_capacity(self.h, int(capacity)))

    def check(self, st):
        if st != OK:
            raise DpcsError(st, lib().dpcs_last_error(self.h).decode())
        return st

    def synchronize(self):
        return self.check(lib().dpcs_context_synchronize(self.h))

    def set_profiling(self, mode: int):
        return self.check(lib().dpcs_context_set_profiling(self.h, int(mode)))

    def profile(self) -> dict:
        p = Profile()
        self.check(lib().dpcs_context_get_profile(self.h, C.byref(p)))
        return p.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().dpcs_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    """Resident mesh + BVH (dpcs_scene) built from a synth.Mesh-like object;
    bvh = "lbvh" (Morton radix tree), "sah" (binned SAH) or "ploc" (clustering); all built on the device."""

    def __init__(self, ctx: Context, mesh, bvh: str = "lbvh"):
        self.ctx = ctx
        V = np.ascontiguousarray(mesh.vertices, np.float32)
        F = np.ascontiguousarray(mesh.triangles, np.int32)
        UV = np.ascontiguousarray(mesh.corner_uvs, np.float32)
        E = None if mesh.emission is None else np.ascontiguousarray(mesh.emission, np.float32)
        kind = {"lbvh": BVH_LBVH, "sah": BVH_SAH, "ploc": BVH_PLOC}[bvh]
        d = MeshDesc(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], UV.ctypes.data,
                     None if E is None else E.ctypes.data, kind)
        h = C.c_void_p()
        ctx.check(lib().dpcs_scene_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    def refit(self, positions):
        """New vertex positions (device tensor, num_vertices x 3 float32) on the same
        topology: the BVH is refitted on the device."""
        if positions.dtype != __import__("torch").float32 or not positions.is_contiguous():
            raise ValueError("positions must be a contiguous float32 device tensor")
        return self.ctx.check(lib().dpcs_scene_refit(self.ctx.h, self.h, _ptr(positions)))

    def info(self) -> SceneInfo:
        i = SceneInfo()
        self.ctx.check(lib().dpcs_scene_get_info(self.h, C.byref(i)))
        return i

    def close(self):
        if getattr(self, "h", None):
            st = lib().dpcs_scene_destroy(self.h)
            if st == OK:
                self.h = None
            return st
        return OK

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pinhole(p) -> Pinhole:
    ph = Pinhole()
    ph.K[:] = [float(x) for x in np.ravel(p.K)]
    ph.R[:] = [float(x) for x in np.ravel(p.R)]
    ph.t[:] = [float(x) for x in np.ravel(p.t)]
    ph.width, ph.height = int(p.width), int(p.height)
    return ph


def params_from(w, albedo, roughness=None, specular=None, device_scalars=None, metallic=None, normal_map=None,
                **over) -> RenderParams:
    """RenderParams from a synth.Workload-like object and device tensors for the maps
    (metallic and normal_map: optional device tensors of the further principled maps)."""
    g = lambda k: over[k] if k in over else getattr(w, k)
    p = RenderParams()
    p.camera = pinhole(g("camera"))
    p.projector = pinhole(g("projector"))
    p.brdf = int(g("brdf"))
    p.albedo, p.roughness, p.specular = _ptr(albedo), _ptr(roughness), _ptr(specular)
    p.tex_h, p.tex_w = int(albedo.shape[0]), int(albedo.shape[1])
    p.prf_gamma[:] = [float(x) for x in g("prf_gamma")]
    p.prf_gain = float(g("prf_gain"))
    p.prf_mix[:] = [float(x) for x in np.ravel(g("prf_mix"))]
    p.crf_gamma[:] = [float(x) for x in g("crf_gamma")]
    p.crf_gain = float(g("crf_gain"))
    p.white_balance[:] = [float(x) for x in g("white_balance")]
    p.device_scalars = _ptr(device_scalars)
    p.env_radiance[:] = [float(x) for x in g("env")]
    p.clip_enable = int(bool(g("clip")))
    p.clip_k = float(g("clip_k"))
    p.spp = int(g("spp"))
    p.max_depth = int(g("max_depth"))
    p.seed = int(g("seed"))
    p.sample_offset = int(g("sample_offset"))
    p.metallic, p.normal_map = _ptr(metallic), _ptr(normal_map)
    return p


# ------------------------------------------------------------------ entry points

def dpcs_render(ctx: Context, scene: Scene, params: RenderParams, proj_image, out_image, linear=None,
                sample_radiance=None, hit_prims=None, path_records=None):
    aux = RenderAux(_ptr(linear), _ptr(sample_radiance), _ptr(hit_prims), _ptr(path_records))
    return ctx.check(lib().dpcs_render(ctx.h, scene.h, C.byref(params), _ptr(proj_image), _ptr(out_image),
                                       C.byref(aux)))


def dpcs_render_noalloc(ctx: Context, scene: Scene, params: RenderParams, proj_image, out_image, linear=None,
                        sample_radiance=None, hit_prims=None, path_records=None):
    aux = RenderAux(_ptr(linear), _ptr(sample_radiance), _ptr(hit_prims), _ptr(path_records))
    return ctx.check(lib().dpcs_render_noalloc(ctx.h, scene.h, C.byref(params), _ptr(proj_image),
                                               _ptr(out_image), C.byref(aux)))


def dpcs_render_vjp(ctx: Context, scene: Scene, params: RenderParams, proj_image, grad_image, sample_radiance=None,
                    d_proj_image=None, d_albedo=None, d_roughness=None, d_specular=None, d_scalars=None,
                    path_records=None, d_metallic=None, d_normal_map=None, d_camera=None,
                    camera_edge_density=0.0):
    """d_camera: 12 floats, d/dR_c (row-major) then d/dt_c of the camera pose: the interior
    part, plus the boundary part at the images of mesh edges when camera_edge_density > 0
    (points per pixel of edge length)."""
    g = Grads(_ptr(d_proj_image), _ptr(d_albedo), _ptr(d_roughness), _ptr(d_specular), _ptr(d_scalars),
              _ptr(d_metallic), _ptr(d_normal_map), _ptr(d_camera), float(camera_edge_density))
    return ctx.check(lib().dpcs_render_vjp(ctx.h, scene.h, C.byref(params), _ptr(proj_image), _ptr(grad_image),
                                           _ptr(sample_radiance), _ptr(path_records), C.byref(g)))


def dpcs_debug_intersect(ctx: Context, scene: Scene, rays, use_bvh, prim, t=None, b1=None, b2=None):
    """use_bvh: 0 / False brute force, 1 / True the renderer's BVH, 2 the binary BVH,
    3 any hit through the renderer's BVH, 4 any hit by brute force."""
    return ctx.check(lib().dpcs_debug_intersect(ctx.h, scene.h, _ptr(rays), int(rays.shape[0]), int(use_bvh),
                                                _ptr(prim), _ptr(t), _ptr(b1), _ptr(b2)))


def dpcs_debug_philox(ctx: Context, seed: int, ctr, out):
    return ctx.check(lib().dpcs_debug_philox(ctx.h, int(seed), _ptr(ctr), int(ctr.shape[0]), _ptr(out)))


def dpcs_debug_brdf(ctx: Context, brdf: int, inputs, out):
    """inputs: device float64 (n, 17); out: device float64 (n, 11) (layout in dpcs.h)."""
    return ctx.check(lib().dpcs_debug_brdf(ctx.h, int(brdf), _ptr(inputs), int(inputs.shape[0]), _ptr(out)))


def dpcs_denoise(ctx: Context, p: DenoiseParams, image, guide, out):
    return ctx.check(lib().dpcs_denoise(ctx.h, C.byref(p), _ptr(image), _ptr(guide), _ptr(out)))


def dpcs_denoise_vjp(ctx: Context, p: DenoiseParams, grad_out, guide, grad_image):
    return ctx.check(lib().dpcs_denoise_vjp(ctx.h, C.byref(p), _ptr(grad_out), _ptr(guide), _ptr(grad_image)))


def dpcs_render_gbuffer(ctx: Context, scene: Scene, params: RenderParams, gbuffer):
    return ctx.check(lib().dpcs_render_gbuffer(ctx.h, scene.h, C.byref(params), _ptr(gbuffer)))


def _map_shape(m):
    h, w = int(m.shape[0]), int(m.shape[1])
    return h, w, (1 if m.dim() == 2 else int(m.shape[2]))


def dpcs_tv_loss(ctx: Context, m, loss):
    h, w, c = _map_shape(m)
    return ctx.check(lib().dpcs_tv_loss(ctx.h, _ptr(m), h, w, c, _ptr(loss)))


def dpcs_tv_vjp(ctx: Context, m, grad_loss, grad_m):
    h, w, c = _map_shape(m)
    return ctx.check(lib().dpcs_tv_vjp(ctx.h, _ptr(m), h, w, c, _ptr(grad_loss), _ptr(grad_m)))


def dpcs_l1_loss(ctx: Context, a, b, loss):
    return ctx.check(lib().dpcs_l1_loss(ctx.h, _ptr(a), _ptr(b), int(a.numel()), _ptr(loss)))


def dpcs_l1_vjp(ctx: Context, a, b, grad_loss, grad_a):
    return ctx.check(lib().dpcs_l1_vjp(ctx.h, _ptr(a), _ptr(b), int(a.numel()), _ptr(grad_loss), _ptr(grad_a)))


class Server:
    """dpcs_server: continuous-batching request loop on a context's device."""

    def __init__(self, ctx: Context, budget_bytes: int, max_slots: int = 64):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.check(lib().dpcs_server_create(ctx.h, int(budget_bytes), int(max_slots), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, request_id: int, scene: Scene, params: RenderParams, proj_image, out_image, grad_image=None,
               target=None, grads: dict | None = None, keep=None, stream=None) -> int:
        """Queues one request; its first launch waits for the work queued on `stream`
        (default: torch's current stream) at this call, so inputs written there are ready."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        g = None
        if grads is not None:
            g = Grads(_ptr(grads.get("d_proj_image")), _ptr(grads.get("d_albedo")), _ptr(grads.get("d_roughness")),
                      _ptr(grads.get("d_specular")), _ptr(grads.get("d_scalars")))
        rq = Request(scene.h, params, _ptr(proj_image), _ptr(out_image), _ptr(grad_image), _ptr(target),
                     C.pointer(g) if g is not None else None, int(request_id), C.c_void_p(stream.cuda_stream))
        st = lib().dpcs_server_submit(self.h, C.byref(rq))
        if st == OK:
            self._keep[int(request_id)] = (params, proj_image, out_image, grad_image, target, grads, g, keep)
        return st

    def poll(self, max_items: int = 256):
        ids = (C.c_uint64 * max_items)()
        sts = (C.c_int32 * max_items)()
        lat = (C.c_double * max_items)()
        n = lib().dpcs_server_poll(self.h, ids, sts, lat, max_items)
        out = []
        for k in range(n):
            out.append((int(ids[k]), int(sts[k]), float(lat[k])))
            self._keep.pop(int(ids[k]), None)
        return out

    def stats(self) -> dict:
        v = (C.c_int64 * 14)()
        self.ctx.check(lib().dpcs_server_stats(self.h, v))
        keys = ["submitted", "completed", "rejected", "active", "queued", "waves", "samples", "peak_bytes",
                "replayed_waves", "retraced_waves", "wait_us", "admit_us", "run_us", "binned_waves"]
        return dict(zip(keys, [int(x) for x in v]))

    def close(self):
        if getattr(self, "h", None):
            st = lib().dpcs_server_destroy(self.h)
            self.h = None
            self._keep.clear()
            return st
        return OK

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
