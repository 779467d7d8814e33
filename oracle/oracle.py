"""ctypes wrapper of the FP64 CPU oracle (oracle/dpcs_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the CPU
baseline of the benchmark.  Nothing on the product path imports this module.
It takes the plain arrays the seeded generators produce and shares no code
with the GPU library.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dpcs_oracle.c")
LIB = os.path.join(HERE, "libdpcs_oracle.so")


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (plain C99, FP64, OpenMP over pixels)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class Desc(C.Structure):
    _fields_ = [
        ("nv", C.c_int32), ("nt", C.c_int32),
        ("V", C.c_void_p), ("F", C.c_void_p), ("UV", C.c_void_p), ("Le", C.c_void_p),
        ("Kc", C.c_double * 9), ("Rc", C.c_double * 9), ("tc", C.c_double * 3),
        ("Wc", C.c_int32), ("Hc", C.c_int32),
        ("Kp", C.c_double * 9), ("Rp", C.c_double * 9), ("tp", C.c_double * 3),
        ("Wp", C.c_int32), ("Hp", C.c_int32),
        ("brdf", C.c_int32), ("tw", C.c_int32), ("th", C.c_int32),
        ("albedo", C.c_void_p), ("rough", C.c_void_p), ("spec", C.c_void_p), ("rough_sample", C.c_void_p),
        ("Ip", C.c_void_p),
        ("prf_gamma", C.c_double * 3), ("prf_gain", C.c_double), ("prf_mix", C.c_double * 9),
        ("crf_gamma", C.c_double * 3), ("crf_gain", C.c_double), ("wb", C.c_double * 3),
        ("env", C.c_double * 3),
        ("clip", C.c_int32), ("clip_k", C.c_double),
        ("spp", C.c_int32), ("max_depth", C.c_int32),
        ("seed", C.c_uint64), ("sample_offset", C.c_uint32),
        ("nthreads", C.c_int32),
        ("tmin", C.c_double),
        ("metal", C.c_void_p), ("nmap", C.c_void_p), ("nmap_sample", C.c_void_p),
        ("edge_density", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _load(LIB)
    return _lib


@contextlib.contextmanager
def library(path: str):
    """Run the wrapper on another build of the oracle for the duration of the block (the
    tests that plant a mistake in a copy of the source and check that a pin catches it)."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def _load(path: str):
    L = C.CDLL(path)
    P = C.c_void_p
    L.orc_render.argtypes = [C.POINTER(Desc), C.c_int32, P, P, P, P, P, P, P, P]
    L.orc_render_vjp.argtypes = [C.POINTER(Desc), P, C.c_int32, P, P, P, P, P, P, P, P, P, P]
    L.orc_brdf_full.argtypes = [C.c_int32, P, P, P, P, P, C.c_double, C.c_double, C.c_double, P]
    L.orc_shading_frame.argtypes = [C.POINTER(Desc), C.c_int32, P, P, P]
    L.orc_philox_batch.argtypes = [C.c_uint64, C.c_int64, P, P]
    L.orc_intersect.argtypes = [C.POINTER(Desc), C.c_int64, P, P, P, P, P, P]
    L.orc_brdf.argtypes = [C.c_int32, P, P, P, P, C.c_double, C.c_double, P]
    L.orc_sample.argtypes = [C.c_int32, P, P, C.c_double, C.c_int64, P, P, P]
    L.orc_pdf.argtypes = [C.c_int32, P, P, P, C.c_double]
    L.orc_pdf.restype = C.c_double
    L.orc_ggx_D.argtypes = [C.c_double, C.c_double]
    L.orc_ggx_D.restype = C.c_double
    L.orc_ggx_G1.argtypes = [C.c_double, C.c_double]
    L.orc_ggx_G1.restype = C.c_double
    L.orc_prf.argtypes = [C.POINTER(Desc), P]
    L.orc_bilinear.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int64, P, P]
    L.orc_threads.argtypes = [C.POINTER(Desc)]
    L.orc_first_hit.argtypes = [C.POINTER(Desc), C.c_int32, C.c_int32, P]
    L.orc_camera_boundary.argtypes = [C.POINTER(Desc), P, P, C.POINTER(C.c_int64)]
    L.orc_pdf_batch.argtypes = [C.c_int32, P, P, C.c_double, C.c_int64, P, P]
    L.orc_denoise.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, P, C.c_double, C.c_int32, P]
    L.orc_denoise_vjp.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, P, C.c_double, C.c_int32, P]
    L.orc_tv.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P]
    L.orc_tv.restype = C.c_double
    L.orc_l1.argtypes = [P, P, C.c_int64, P]
    L.orc_l1.restype = C.c_double
    L.orc_gbuffer.argtypes = [C.POINTER(Desc), C.c_int32, P, P, P]
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Scene:
    """Everything the oracle needs, as contiguous arrays kept alive for the C side.

    `w` is a `synth.Workload`-like object; keyword overrides replace its fields.
    Textures and the projector image are held in float64 so that finite
    differences can perturb them.
    """

    def __init__(self, w, **over):
        g = lambda k: over[k] if k in over else getattr(w, k)
        mesh = g("mesh")
        self.V = np.ascontiguousarray(mesh.vertices, np.float32)
        self.F = np.ascontiguousarray(mesh.triangles, np.int32)
        self.UV = np.ascontiguousarray(mesh.corner_uvs, np.float32)
        self.Le = None if mesh.emission is None else np.ascontiguousarray(mesh.emission, np.float32)
        self.camera = g("camera")
        self.projector = g("projector")
        self.brdf = int(g("brdf"))
        self.albedo = np.ascontiguousarray(g("albedo"), np.float64)
        self.rough = np.ascontiguousarray(g("roughness"), np.float64)
        self.spec = np.ascontiguousarray(g("specular"), np.float64)
        self.rough_sample = None if over.get("rough_sample") is None else \
            np.ascontiguousarray(over["rough_sample"], np.float64)
        mt = over["metallic"] if "metallic" in over else getattr(w, "metallic", None)
        nm = over["normal_map"] if "normal_map" in over else getattr(w, "normal_map", None)
        self.metal = None if mt is None else np.ascontiguousarray(mt, np.float64)
        self.nmap = None if nm is None else np.ascontiguousarray(nm, np.float64)
        self.nmap_sample = None if over.get("normal_sample") is None else \
            np.ascontiguousarray(over["normal_sample"], np.float64)
        self.Ip = np.ascontiguousarray(g("proj_image"), np.float64)
        self.prf_gamma = np.asarray(g("prf_gamma"), np.float64)
        self.prf_gain = float(g("prf_gain"))
        self.prf_mix = np.asarray(g("prf_mix"), np.float64)
        self.crf_gamma = np.asarray(g("crf_gamma"), np.float64)
        self.crf_gain = float(g("crf_gain"))
        self.wb = np.asarray(g("white_balance"), np.float64)
        self.env = np.asarray(g("env"), np.float64)
        self.clip = bool(g("clip"))
        self.clip_k = float(g("clip_k"))
        self.spp = int(g("spp"))
        self.max_depth = int(g("max_depth"))
        self.seed = int(g("seed"))
        self.sample_offset = int(g("sample_offset"))
        self.nthreads = int(over.get("nthreads", 0))
        self.tmin = float(over.get("tmin", 0.0))
        self.edge_density = float(over.get("edge_density", 0.0))

    def desc(self) -> Desc:
        d = Desc()
        d.nv, d.nt = self.V.shape[0], self.F.shape[0]
        d.V, d.F, d.UV, d.Le = _p(self.V), _p(self.F), _p(self.UV), _p(self.Le)
        cam, prj = self.camera, self.projector
        d.Kc[:] = list(np.ravel(cam.K)); d.Rc[:] = list(np.ravel(cam.R)); d.tc[:] = list(cam.t)
        d.Wc, d.Hc = cam.width, cam.height
        d.Kp[:] = list(np.ravel(prj.K)); d.Rp[:] = list(np.ravel(prj.R)); d.tp[:] = list(prj.t)
        d.Wp, d.Hp = prj.width, prj.height
        d.brdf = self.brdf
        d.th, d.tw = self.albedo.shape[0], self.albedo.shape[1]
        d.albedo, d.rough, d.spec = _p(self.albedo), _p(self.rough), _p(self.spec)
        d.rough_sample = _p(self.rough_sample)
        d.Ip = _p(self.Ip)
        d.prf_gamma[:] = list(self.prf_gamma); d.prf_gain = self.prf_gain
        d.prf_mix[:] = list(np.ravel(self.prf_mix))
        d.crf_gamma[:] = list(self.crf_gamma); d.crf_gain = self.crf_gain; d.wb[:] = list(self.wb)
        d.env[:] = list(self.env)
        d.clip = int(self.clip); d.clip_k = self.clip_k
        d.spp, d.max_depth = self.spp, self.max_depth
        d.seed, d.sample_offset = self.seed, self.sample_offset
        d.nthreads = self.nthreads
        d.tmin = self.tmin
        d.metal, d.nmap, d.nmap_sample = _p(self.metal), _p(self.nmap), _p(self.nmap_sample)
        d.edge_density = self.edge_density
        self._d = d
        return d


def render(sc: Scene, pixels=None, want=("Ec", "Ic", "L", "hits", "margin", "margin_clip")):
    """Forward render of all pixels (pixels=None) or of the listed pixel indices j*W+i."""
    d = sc.desc()
    n = sc.camera.width * sc.camera.height if pixels is None else len(pixels)
    px = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
    out = {}
    out["Ec"] = np.zeros((n, 3)) if "Ec" in want else None
    out["Ic"] = np.zeros((n, 3)) if "Ic" in want else None
    out["L"] = np.zeros((n, sc.spp, 3)) if "L" in want else None
    out["hits"] = np.zeros((n, sc.spp, sc.max_depth), np.int32) if "hits" in want else None
    out["margin"] = np.zeros((n, sc.spp)) if "margin" in want else None
    out["margin_clip"] = np.zeros((n, sc.spp)) if "margin_clip" in want else None
    out["reason"] = np.zeros((n, sc.spp), np.int32) if "reason" in want else None
    lib().orc_render(C.byref(d), n, _p(px), _p(out["Ec"]), _p(out["Ic"]), _p(out["L"]), _p(out["hits"]),
                     _p(out["margin"]), _p(out["margin_clip"]), _p(out["reason"]))
    return {k: v for k, v in out.items() if v is not None}


def render_vjp(sc: Scene, G, pixels=None, camera=False):
    """VJP of the rendered image I_c with cotangent G (Hc x Wc x 3); camera=True adds the
    camera-pose gradient (camera_R, camera_t): its interior part, plus the boundary part at
    the images of mesh edges when the scene has edge_density > 0."""
    d = sc.desc()
    G = np.ascontiguousarray(G, np.float64)
    px = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
    n = 0 if pixels is None else len(pixels)
    th, tw = sc.albedo.shape[:2]
    out = dict(Ip=np.zeros(sc.Ip.shape), albedo=np.zeros((th, tw, 3)), roughness=np.zeros((th, tw)),
               specular=np.zeros((th, tw)), scalars=np.zeros(18), Ep=np.zeros(sc.Ip.shape),
               metallic=np.zeros((th, tw)), normal_map=np.zeros((th, tw, 3)), camera=np.zeros(12))
    lib().orc_render_vjp(C.byref(d), _p(G), n, _p(px), _p(out["Ip"]), _p(out["albedo"]), _p(out["roughness"]),
                         _p(out["specular"]), _p(out["scalars"]), _p(out["Ep"]), _p(out["metallic"]),
                         _p(out["normal_map"]), _p(out["camera"]) if camera else None)
    s = out.pop("scalars")
    cam = out.pop("camera")
    out.update(prf_gamma=s[0:3], prf_mix=s[3:12].reshape(3, 3), crf_gamma=s[12:15], white_balance=s[15:18])
    if camera:   # the camera-pose gradient: d/dR (row-major 3x3) and d/dt
        out.update(camera_R=cam[:9].reshape(3, 3), camera_t=cam[9:])
    return out


def camera_boundary(sc: Scene, dE):
    """The boundary part of the camera-pose gradient alone, for per-pixel cotangents dE
    (Hc x Wc x 3) of the pixel means of the clipped sample radiance; uses the scene's
    edge_density.  Returns (12-vector: d/dR row-major then d/dt, number of edge samples)."""
    d = sc.desc()
    dE = np.ascontiguousarray(dE, np.float64)
    out = np.zeros(12)
    n = C.c_int64(0)
    lib().orc_camera_boundary(C.byref(d), _p(dE), _p(out), C.byref(n))
    return out, int(n.value)


def philox(seed: int, counters: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(counters, np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    lib().orc_philox_batch(seed, c.shape[0], _p(c), _p(out))
    return out


def intersect(sc: Scene, rays: np.ndarray, with_margin=False):
    """rays: n x 8 (o, d, tmax, skip) -> prim, t, b1, b2 (brute force, FP64)."""
    d = sc.desc()
    r = np.ascontiguousarray(rays, np.float64)
    n = r.shape[0]
    prim = np.zeros(n, np.int32)
    t, b1, b2 = np.zeros(n), np.zeros(n), np.zeros(n)
    m = np.zeros(n) if with_margin else None
    lib().orc_intersect(C.byref(d), n, _p(r), _p(prim), _p(t), _p(b1), _p(b2), _p(m))
    return (prim, t, b1, b2, m) if with_margin else (prim, t, b1, b2)


def brdf(kind, n, wo, wi, a, r, sp):
    out = np.zeros(5)
    f = lambda v: np.ascontiguousarray(v, np.float64)
    lib().orc_brdf(kind, _p(f(n)), _p(f(wo)), _p(f(wi)), _p(f(a)), float(r), float(sp), _p(out))
    return out


def brdf_full(kind, ng, ns, wo, wi, a, r, sp, mu):
    """The principled BRDF with metallic mu and shading normal ns: dict of f (3), the cosine
    about ns, df/da, df/dr (3), df/dsp, df/dmu (3) and d(f_c cos)/dns (3 x 3, row c)."""
    out = np.zeros(21)
    f = lambda v: np.ascontiguousarray(v, np.float64)
    lib().orc_brdf_full(kind, _p(f(ng)), _p(f(ns)), _p(f(wo)), _p(f(wi)), _p(f(a)), float(r), float(sp), float(mu),
                        _p(out))
    return dict(f=out[0:3], c=out[3], dfa=out[4], dfr=out[5:8], dfs=out[8], dfm=out[9:12],
                dfcn=out[12:21].reshape(3, 3))


def shading_frame(sc: Scene, prim: int, direction, uv):
    """Tangent frame (T, B, n) and shading normal of a hit on triangle prim."""
    d = sc.desc()
    out = np.zeros(12)
    f = lambda v: np.ascontiguousarray(v, np.float64)
    lib().orc_shading_frame(C.byref(d), int(prim), _p(f(direction)), _p(f(uv)), _p(out))
    return dict(T=out[0:3], B=out[3:6], n=out[6:9], ns=out[9:12])


def sample(kind, n, wo, r, u):
    u = np.ascontiguousarray(u, np.float64).reshape(-1, 3)
    wi = np.zeros((u.shape[0], 3))
    pdf = np.zeros(u.shape[0])
    f = lambda v: np.ascontiguousarray(v, np.float64)
    lib().orc_sample(kind, _p(f(n)), _p(f(wo)), float(r), u.shape[0], _p(u), _p(wi), _p(pdf))
    return wi, pdf


def pdf(kind, n, wo, wi, r):
    f = lambda v: np.ascontiguousarray(v, np.float64)
    return lib().orc_pdf(kind, _p(f(n)), _p(f(wo)), _p(f(wi)), float(r))


def ggx_D(nh, r):
    return lib().orc_ggx_D(float(nh), float(r))


def ggx_G1(c, r):
    return lib().orc_ggx_G1(float(c), float(r))


def prf(sc: Scene):
    d = sc.desc()
    out = np.zeros(sc.Ip.shape)
    lib().orc_prf(C.byref(d), _p(out))
    return out


def bilinear(img, xy):
    img = np.ascontiguousarray(img, np.float64)
    H, W = img.shape[:2]
    Cc = 1 if img.ndim == 2 else img.shape[2]
    xy = np.ascontiguousarray(xy, np.float64).reshape(-1, 2)
    out = np.zeros((xy.shape[0], Cc))
    lib().orc_bilinear(_p(img), W, H, Cc, xy.shape[0], _p(xy), _p(out))
    return out


def threads(sc: Scene) -> int:
    return lib().orc_threads(C.byref(sc.desc()))


def first_hit(sc: Scene, pixel: int, s: int):
    """Camera ray and first-hit attributes of one camera sample."""
    d = sc.desc()
    out = np.zeros(18)
    lib().orc_first_hit(C.byref(d), int(pixel), int(s), _p(out))
    return dict(o=out[0:3], d=out[3:6], t=out[6], prim=int(out[7]), x=out[8:11], n=out[11:14],
                uv=out[14:16], puv=out[16:18])


def pdf_batch(kind, n, wo, r, wi):
    f = lambda v: np.ascontiguousarray(v, np.float64)
    wi = f(wi).reshape(-1, 3)
    out = np.zeros(wi.shape[0])
    lib().orc_pdf_batch(kind, _p(f(n)), _p(f(wo)), float(r), wi.shape[0], _p(wi), _p(out))
    return out


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def _guide(img, guide, coef):
    img = _f64(img)
    H, W = img.shape[:2]
    guide = _f64(np.zeros((H, W, 0)) if guide is None else guide).reshape(H, W, -1)
    coef = _f64(np.zeros(0) if coef is None else coef).reshape(-1)
    if coef.shape[0] != guide.shape[2]:
        raise ValueError("one guide coefficient per guide channel")
    return img, guide, coef, H, W


def denoise(img, guide, coef, spatial, radius):
    """Eq. 11: cross-bilateral filter of an H x W x 3 image steered by an H x W x G guide;
    coef[k] and spatial are the 1 / (2 sigma^2) factors of the weights."""
    img, guide, coef, H, W = _guide(img, guide, coef)
    out = np.zeros_like(img)
    lib().orc_denoise(_p(img), _p(guide), W, H, guide.shape[2], _p(coef), float(spatial), int(radius), _p(out))
    return out


def denoise_vjp(grad, guide, coef, spatial, radius):
    """Transpose of denoise() (the guide is a constant): cotangent of the input image."""
    grad, guide, coef, H, W = _guide(grad, guide, coef)
    out = np.zeros_like(grad)
    lib().orc_denoise_vjp(_p(grad), _p(guide), W, H, guide.shape[2], _p(coef), float(spatial), int(radius),
                          _p(out))
    return out


def tv(m):
    """Eq. 9 regulariser of an h x w (x c) map: (loss, dloss/dm)."""
    m = _f64(m)
    h, w = m.shape[:2]
    c = 1 if m.ndim == 2 else m.shape[2]
    g = np.zeros_like(m)
    loss = lib().orc_tv(_p(m), h, w, c, _p(g))
    return loss, g


def l1(a, b):
    """Eq. 9 data term: (mean |a - b|, d/da)."""
    a, b = _f64(a), _f64(b)
    g = np.zeros_like(a)
    loss = lib().orc_l1(_p(a), _p(b), a.size, _p(g))
    return loss, g


def gbuffer(sc: Scene, pixels=None):
    """Guide features through each pixel centre: (npix x 8 features, npix margins)."""
    d = sc.desc()
    npix = d.Wc * d.Hc if pixels is None else len(pixels)
    px = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
    out = np.zeros((npix, 8))
    margin = np.zeros(npix)
    lib().orc_gbuffer(C.byref(d), npix, _p(px), _p(out), _p(margin))
    return out, margin
