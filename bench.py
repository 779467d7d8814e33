"""Benchmark of the DPCS hot path on one MI355X.

One step = one pass of the whole path over one batch: forward render of the
paper-scale scene (50k-triangle displaced folded corner + 3 box occluders, GGX
512^2 maps, 256x256 camera, 256x256 projector, 64 spp, depth 4) and its
vector-Jacobian product by path replay of the same samples.

Prints ONE JSON line.  Inputs are synthetic and resident in HBM before timing.
  value          path samples/s of the timed fwd+VJP steps (fwd_samples_per_s: forward alone)
  roofline       live HIP-event timing of the dominant kernel (closest-hit
                 traversal) against its algorithmic operations and the vector-ALU
                 issue peak (its DRAM traffic is ~0.1 of HBM: the tree lives in L2 / MALL),
                 with the HBM byte model and the counters' DRAM bytes beside it
  cpu_baseline   the FP64 CPU oracle timed on a bounded pixel sample
  objective      the training objective's operators (denoiser D and its VJP, guide
                 features, L1 data term, map regulariser), timed apart from the step
  configs        the other synthetic setups end to end (quad+cube forward, 200k-triangle
                 512^2 forward and fwd+VJP, 100 compensation steps, a scene-fit step)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "path samples/s fwd and fwd+adjoint (1 GPU, ≤1e-4 rel err); p50/p99 relight latency"
HBM_PEAK_GBS = 8000.0
# vector ALU issue of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit VALU
# operation per lane per clock (the published 157.3 TFLOP/s counts an FMA as two flops and
# packed FP32 as two lanes' worth, neither of which a traversal loop issues)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "trace_traffic_corner50k_256px.md")
COUNTER_FILE = os.path.join(ROOT, "profiles", "hot_kernel_counters_corner50k_256px.md")
KERNEL_SOURCES = ["render.hip", "trace.hpp", "shade.hpp", "common.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_12174_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# algorithmic bytes of one closest-hit query in this layout: path origin and
# direction read (PathO + PathD = 64 B), each visited BVH node (64 B binary, 128 B
# 4-wide), each tested triangle record (48 B), the hit index written (4 B)
RAY_IO_BYTES = 64 + 4
NODE_BYTES = 64       # binary BVH node: two child boxes + two child references
NODE4_BYTES = 128     # 4-wide BVH node: four child boxes (SoA) + four references + pad
TRI_BYTES = 48
UV_BYTES = 32          # corner UVs of a triangle
SHADE_STATE_IN = 84    # PathO + PathD + throughput + hit index
PATH_STATE = 80        # PathO + PathD + throughput written for a continuing path
SHADOW_RECORD = 52     # shadow origin, direction, contribution float4s + t_max

# algorithmic FP32 operations of one closest-hit query (each add, mul, FMA, min, max,
# compare or select is one operation; a component permutation is a register choice):
#   per ray      box setup (3 reciprocals, 3 products, 3 error bounds, 6 offsets), the
#                watertight setup (axis choice 4, 3 quotients), the exact test of the
#                winner for t and the barycentrics (33 + 3) = 15 + 7 + 36
#   per node     4 children x (6 slab FMAs, 4 ops of the two 3-way max / min, 2 widenings,
#                2 clamps, 1 compare) + 5 compare-exchanges ordering the children (3 each)
#   per triangle 9 subtractions, 6 FMAs of the shear, 6 of the edge functions, 2 of the
#                sign test, 2 for the determinant, 3 for T, 3 for t = T Sz / det, 2 range
#                compares
OPS_RAY, OPS_NODE4, OPS_NODE2, OPS_TRI = 58, 75, 31, 33


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--quick", action="store_true", help="skip the profiled passes")
    ap.add_argument("--serving-requests", type=int, default=2000, help="0 disables the serving run")
    ap.add_argument("--serving-alone", type=int, default=60, help="requests also timed alone")
    ap.add_argument("--no-serving-sweep", action="store_true", help="skip the serving runs at higher rates")
    ap.add_argument("--no-objective", action="store_true", help="skip the training-objective operators")
    ap.add_argument("--no-configs", action="store_true", help="skip the other setups (quad+cube, 200k corner, fit)")
    return ap.parse_args()


FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (packed); the build disables packed FP32: 78.6


def objective_bench(ctx, scene, params, image, maps, reps=50):
    """The training objective's device operators on this workload (Eq. 9, 11): guide
    features, D and its VJP on the 256 x 256 rendering, L1 against a capture and L(m) of
    the three BRDF maps with their VJPs, each timed with events on the context's stream
    (the torch stream it was created on); D alone also on a 2048 x 2048 image, where the
    launch fills the chip, against its arithmetic model (4G + 9 FP32 flops per window
    tap: G guide channels of sub, mul, fma; exp2; the weight sum; three fmas)."""
    import numpy as np
    import torch

    from paper_2503_12174_amd import dpcs
    from paper_2503_12174_amd import objective as Ob

    cfg = Ob.DenoiseConfig()
    H, W = image.shape[:2]
    guide = Ob.gbuffer(ctx, scene, params)
    p = cfg.params(W, H, guide.shape[2])
    den, gimg = torch.empty_like(image), torch.empty_like(image)
    tgt = torch.as_tensor(np.random.default_rng(8).uniform(0, 1, (H, W, 3)).astype(np.float32)).cuda()
    loss, gl, gl1 = torch.empty((), device="cuda"), torch.ones((), device="cuda"), torch.empty_like(image)
    gmaps = [torch.empty_like(m) for m in maps]

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ops = {
        "gbuffer": lambda: dpcs.dpcs_render_gbuffer(ctx, scene, params, guide),
        "denoise": lambda: dpcs.dpcs_denoise(ctx, p, image, guide, den),
        "l1": lambda: dpcs.dpcs_l1_loss(ctx, den, tgt, loss),
        "l1_vjp": lambda: dpcs.dpcs_l1_vjp(ctx, den, tgt, gl, gl1),
        "denoise_vjp": lambda: dpcs.dpcs_denoise_vjp(ctx, p, gl1, guide, gimg),
        "tv_3maps": lambda: [dpcs.dpcs_tv_loss(ctx, m, loss) for m in maps],
        "tv_vjp_3maps": lambda: [dpcs.dpcs_tv_vjp(ctx, m, gl, g) for m, g in zip(maps, gmaps)],
    }
    res = {k: round(timed(f), 5) for k, f in ops.items()}
    res["objective_step_ms"] = round(sum(v for k, v in res.items() if k != "gbuffer"), 4)

    # D on a 2048 x 2048 image with an 8-channel guide: arithmetic throughput
    N = 2048
    g = torch.Generator(device="cuda").manual_seed(9)
    big = torch.rand((N, N, 3), device="cuda", generator=g)
    bguide = torch.rand((N, N, 8), device="cuda", generator=g)
    bout = torch.empty_like(big)
    bp = cfg.params(N, N, 8)
    ms = timed(lambda: dpcs.dpcs_denoise(ctx, bp, big, bguide, bout))
    r = cfg.radius
    taps = float(N * (2 * r + 1) - r * (r + 1)) ** 2   # window taps summed over pixels (clipped at borders)
    flops = taps * (4 * 8 + 9)
    tf = flops / (ms * 1e-3) / 1e12
    res["denoise_2048"] = {"ms": round(ms, 4), "taps_per_s": round(taps / (ms * 1e-3), 1),
                           "bound": "alu", "achieved": round(tf, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4)}
    return res


def configs_bench(ctx, steps=5):
    """The other synthetic setups, timed end to end (context beside the headline step):
    the oracle-scale quad-and-cube forward, the 200k-triangle 512^2 compensation-scale
    forward and forward + VJP step at 16 spp, 100 Adam steps of projector compensation
    on it, a relighting render at the paper's capture resolutions, one scene-fit step
    (8 image pairs, 32 spp forward + VJP each), and the VJP on the headline scene with the
    camera-pose gradient's interior and boundary parts."""
    import copy

    import numpy as np
    import torch

    from paper_2503_12174_amd import drivers, dpcs, synth

    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float32)).cuda()

    def wall(fn, k):
        fn()
        ctx.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        ctx.synchronize()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    res = {}
    # quad + cube, 64^2, 4 spp, depth 3 (launch-bound: a render is ~16k samples)
    w = synth.quad_cube()
    sc = dpcs.Scene(ctx, w.mesh)
    alb, rough, spec, proj = dev(w.albedo), dev(w.roughness), dev(w.specular), dev(w.proj_image)
    p = dpcs.params_from(w, alb, rough, spec)
    out = torch.zeros((64, 64, 3), device="cuda")
    ms = wall(lambda: dpcs.dpcs_render(ctx, sc, p, proj, out), 50)
    res["quad_cube_forward"] = {"ms": round(ms, 4), "samples_per_s": round(64 * 64 * w.spp / (ms * 1e-3), 1)}

    # 200k-triangle corner, 512^2 camera and projector, 16 spp, depth 4
    w = synth.corner_200k()
    sc = dpcs.Scene(ctx, w.mesh, bvh="sah")
    alb, rough, spec, proj = dev(w.albedo), dev(w.roughness), dev(w.specular), dev(w.proj_image)
    p = dpcs.params_from(w, alb, rough, spec)
    H, W = w.camera.height, w.camera.width
    n = H * W * w.spp
    out = torch.zeros((H, W, 3), device="cuda")
    Ls = torch.zeros((H, W, w.spp, 3), device="cuda")
    rec = torch.zeros((H, W, w.spp, w.max_depth), dtype=torch.int32, device="cuda")
    G = dev(np.random.default_rng(11).normal(size=(H, W, 3)))
    grads = dict(d_proj_image=torch.zeros_like(proj), d_albedo=torch.zeros_like(alb),
                 d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                 d_scalars=torch.zeros(18, device="cuda"))

    def step():
        dpcs.dpcs_render(ctx, sc, p, proj, out, sample_radiance=Ls, path_records=rec)
        dpcs.dpcs_render_vjp(ctx, sc, p, proj, G, sample_radiance=Ls, path_records=rec, **grads)

    ms_f = wall(lambda: dpcs.dpcs_render(ctx, sc, p, proj, out), steps)
    ms_s = wall(step, steps)
    res["corner_200k_512px_16spp"] = {"triangles": int(sc.info().num_triangles),
                                      "forward_ms": round(ms_f, 4), "forward_samples_per_s": round(n / (ms_f * 1e-3), 1),
                                      "fwd_vjp_ms": round(ms_s, 4), "fwd_vjp_samples_per_s": round(n / (ms_s * 1e-3), 1)}
    del Ls, rec
    # projector compensation: 100 Adam steps (lr 0.01) of fwd + VJP at 16 spp
    tgt = dev(synth.compensation_target(512))
    drivers.compensate(ctx, sc, w, tgt, alb, rough, spec, steps=3, lr=0.01)   # scratch and allocator warm-up
    torch.cuda.synchronize()
    stamps = []
    t0 = time.perf_counter()
    _, losses = drivers.compensate(ctx, sc, w, tgt, alb, rough, spec, steps=100, lr=0.01,
                                   callback=lambda k, l, ip: stamps.append(time.perf_counter()))
    torch.cuda.synchronize()
    res["compensation_100_steps"] = {"s": round(time.perf_counter() - t0, 3),
                                     "median_step_ms": round(float(np.median(np.diff(stamps))) * 1e3, 3),
                                     "loss_first_last": [round(losses[0], 5), round(losses[-1], 5)]}
    del sc

    # relighting render at the paper's capture resolutions (camera 640x360, projector
    # 800x600, 16 spp): the paper's own figure for one such render is 2.48 s on an
    # RTX 3090 (real scene, render resolution unstated) -- context, not a like-for-like
    w = synth.corner_capture_res()
    sc = dpcs.Scene(ctx, w.mesh, bvh="sah")
    alb, rough, spec, proj = dev(w.albedo), dev(w.roughness), dev(w.specular), dev(w.proj_image)
    p = dpcs.params_from(w, alb, rough, spec)
    out = torch.zeros((w.camera.height, w.camera.width, 3), device="cuda")
    ms = wall(lambda: dpcs.dpcs_render(ctx, sc, p, proj, out), steps)
    n = w.camera.width * w.camera.height * w.spp
    res["relight_640x360_proj800x600_16spp"] = {"ms": round(ms, 4), "samples_per_s": round(n / (ms * 1e-3), 1)}
    del sc

    # scene fit step: 8 pairs at 64^2, 32 spp, GGX maps and 18 scalars
    w = synth.fit_scene(spp=32)
    sc = dpcs.Scene(ctx, w.mesh)
    imgs = [dev(i) for i in synth.fit_images(0, 8)]
    tg = [dev(np.random.default_rng(40 + k).uniform(0, 1, (64, 64, 3))) for k in range(8)]
    c = copy.copy(w)
    drivers.fit(ctx, sc, c, imgs, tg, steps=2, lr=0.02)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    drivers.fit(ctx, sc, c, imgs, tg, steps=10, lr=0.02)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 10
    res["fit_step_8x64px_32spp"] = {"ms": round(ms, 3), "samples_per_s": round(8 * 64 * 64 * 32 / (ms * 1e-3), 1)}
    del sc

    # camera-pose gradient on the headline scene (VJP replaying the forward's records):
    # without it, its interior part, and with the boundary part at 1 and 4 points per
    # pixel of edge length
    w = synth.corner_50k()
    sc = dpcs.Scene(ctx, w.mesh, bvh="sah")
    alb, rough, spec, proj = dev(w.albedo), dev(w.roughness), dev(w.specular), dev(w.proj_image)
    p = dpcs.params_from(w, alb, rough, spec)
    H, W = w.camera.height, w.camera.width
    out = torch.zeros((H, W, 3), device="cuda")
    Ls = torch.zeros((H, W, w.spp, 3), device="cuda")
    rec = torch.zeros((H, W, w.spp, w.max_depth), dtype=torch.int32, device="cuda")
    dpcs.dpcs_render(ctx, sc, p, proj, out, sample_radiance=Ls, path_records=rec)
    G = dev(np.random.default_rng(12).normal(size=(H, W, 3)))
    grads = dict(d_proj_image=torch.zeros_like(proj), d_albedo=torch.zeros_like(alb),
                 d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                 d_scalars=torch.zeros(18, device="cuda"))
    d_cam = torch.zeros(12, device="cuda")
    cam = {}
    for key, pose, dens in (("vjp_ms", False, 0.0), ("with_interior_ms", True, 0.0), ("with_edges_1_ms", True, 1.0),
                            ("with_edges_4_ms", True, 4.0)):
        kw = dict(d_camera=d_cam, camera_edge_density=dens) if pose else {}
        cam[key] = round(wall(lambda: dpcs.dpcs_render_vjp(ctx, sc, p, proj, G, sample_radiance=Ls, path_records=rec,
                                                           **grads, **kw), steps), 4)
    res["camera_pose_vjp_corner50k_256px_64spp"] = cam
    del Ls, rec, sc
    return res


def serving_bench(ctx, n_req, n_alone, warmup=100, rate=50.0, sweep=(30.0, 40.0, 100.0, 200.0), n_sweep=400,
                  max_slots=64):
    """Serving run: 4 resident corners (10k/50k/200k/500k triangles), Poisson arrivals,
    resolution in {128, 256, 512}^2, spp in {16, 64, 256}, depth 4, half relighting and
    half compensation steps (fwd + VJP of an L2 loss).  n_req requests after `warmup` at
    `rate` req/s, then shorter runs at the `sweep` rates (n_sweep requests each after 50
    warm-up) for the highest rate whose p99 stays bounded, then n_alone of the same
    requests alone through the plain entry points."""
    import threading

    import numpy as np
    import torch

    from paper_2503_12174_amd import dpcs, synth

    t = time.perf_counter()
    meshes = synth.serving_scenes()
    scenes = [dpcs.Scene(ctx, m, bvh="sah") for m in meshes]
    infos = [sc.info() for sc in scenes]
    alb, rough, spec = (torch.as_tensor(x).cuda() for x in synth.ggx_textures(503, 512))
    # inputs and outputs from pools (16 images per resolution; one output set per
    # request slot of 128 in rotation: requests 128 apart are never in flight together
    # below the saturated rates, and above them only the timing is read)
    pool = {}
    for res in (128, 256, 512):
        rng = np.random.default_rng(res)
        pool[res] = dict(
            ip=[torch.as_tensor(rng.uniform(0, 1, (res, res, 3)).astype(np.float32)).cuda() for _ in range(16)],
            target=[torch.as_tensor(synth.blob_image(res, res, 700 + k, lo=0.1, hi=0.9)).cuda() for k in range(4)])
    outs = {}

    def out_for(k, res, comp):
        key = (k % 128, res)
        if key not in outs:
            outs[key] = dict(out=torch.zeros((res, res, 3), device="cuda"),
                             grads=dict(d_proj_image=torch.zeros((res, res, 3), device="cuda"),
                                        d_albedo=torch.zeros_like(alb), d_roughness=torch.zeros_like(rough),
                                        d_specular=torch.zeros_like(spec), d_scalars=torch.zeros(18, device="cuda")))
        o = outs[key]
        return o["out"], (o["grads"] if comp else None)

    templates = {}
    for res in (128, 256, 512):   # camera, projector and response parameters per resolution
        w = synth.corner_50k(res=res)
        w.projector = synth.pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, res, res)
        templates[res] = w

    def prepare(reqs):
        prep = []
        for k, rq in enumerate(reqs):
            res = rq["res"]
            p = dpcs.params_from(templates[res], alb, rough, spec, spp=rq["spp"], max_depth=rq["depth"], seed=k)
            ip = pool[res]["ip"][rq["image_seed"] % 16]
            out, grads = out_for(k, res, rq["compensation"])
            target = pool[res]["target"][rq["image_seed"] % 4] if rq["compensation"] else None
            prep.append((k, rq, p, ip, out, target, grads, res * res * rq["spp"]))
        return prep

    def run(reqs, warmup):
        prep = prepare(reqs)
        torch.cuda.synchronize()
        srv = dpcs.Server(ctx, budget_bytes=64 << 30, max_slots=max_slots)
        lat = {}
        t0 = time.perf_counter()

        def client():
            for k, rq, p, ip, out, target, grads, _ in prep:
                dt = rq["arrival"] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                st = srv.submit(k, scenes[rq["scene"]], p, ip, out, target=target, grads=grads)
                if st != dpcs.OK:
                    lat[k] = None

        th = threading.Thread(target=client)
        th.start()
        last_print = time.perf_counter()
        while len(lat) < len(prep):
            for k, st, ms in srv.poll():
                lat[k] = ms if st == dpcs.OK else None
            if time.perf_counter() - last_print > 10:
                print(f"[bench] serving: {len(lat)}/{len(prep)} done", file=sys.stderr, flush=True)
                last_print = time.perf_counter()
            time.sleep(0.001)
        th.join()
        wall = time.perf_counter() - t0
        stats = srv.stats()
        srv.close()
        measured = [k for k, *_ in prep[warmup:]]
        ok = [lat[k] for k in measured if lat[k] is not None]
        span = wall - reqs[warmup]["arrival"]
        samples = sum(x[-1] * (2 if x[1]["compensation"] else 1) for x in prep[warmup:])
        offered = sum(x[-1] * (2 if x[1]["compensation"] else 1) for x in prep) / reqs[-1]["arrival"]
        done = max(stats["completed"], 1)
        return prep, {
            "requests": len(measured), "warmup_requests": warmup, "completed_ok": len(ok),
            "p50_ms": round(float(np.percentile(ok, 50)), 2), "p99_ms": round(float(np.percentile(ok, 99)), 2),
            "mean_ms": round(float(np.mean(ok)), 2), "achieved_req_s": round(len(ok) / span, 2),
            "samples_per_s": round(samples / span, 1), "offered_samples_per_s": round(offered, 1),
            "mean_queue_wait_ms": round(stats["wait_us"] / done / 1e3, 3),
            "mean_admit_to_first_wave_ms": round(stats["admit_us"] / done / 1e3, 3),
            "mean_first_wave_to_done_ms": round(stats["run_us"] / done / 1e3, 3),
            "waves": stats["waves"], "peak_admitted_bytes": stats["peak_bytes"]}

    setup_s = time.perf_counter() - t
    reqs = synth.serving_requests(warmup + n_req, seed=501, rate=rate)
    prep, main = run(reqs, warmup)
    main["rate_req_s"] = rate

    # the same requests alone through the plain entry points (a subset, back to back)
    alone = []
    for k, rq, p, ip, out, target, grads, _ in prep[warmup:warmup + n_alone]:
        sc = scenes[rq["scene"]]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        if grads is None:
            dpcs.dpcs_render(ctx, sc, p, ip, out)
        else:
            L = torch.empty((rq["res"], rq["res"], rq["spp"], 3), device="cuda")
            rc = torch.empty((rq["res"], rq["res"], rq["spp"], p.max_depth), dtype=torch.int32, device="cuda")
            dpcs.dpcs_render(ctx, sc, p, ip, out, sample_radiance=L, path_records=rc)
            G = (2.0 * (out - target) / out.numel()).contiguous()
            dpcs.dpcs_render_vjp(ctx, sc, p, ip, G, sample_radiance=L, path_records=rc, **grads)
        ctx.synchronize()
        alone.append((time.perf_counter() - ta) * 1e3)
    alone_p99 = float(np.percentile(alone, 99))
    main.update(alone_p50_ms=round(float(np.percentile(alone, 50)), 2), alone_p99_ms=round(alone_p99, 2),
                alone_requests=len(alone))

    # rate sweep: bounded = the loop keeps up (>= 95 % of the offered request rate) and
    # p99 stays within 3x the p99 of the same request mix run alone
    table = [{"rate_req_s": rate, "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"],
              "achieved_req_s": main["achieved_req_s"], "samples_per_s": main["samples_per_s"]}]
    for r in sweep:
        rq = synth.serving_requests(50 + n_sweep, seed=601 + int(r), rate=r)
        _, st = run(rq, 50)
        table.append({"rate_req_s": r, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                      "achieved_req_s": st["achieved_req_s"], "samples_per_s": st["samples_per_s"]})
        print(f"[bench] serving sweep {r} req/s: p50 {st['p50_ms']} p99 {st['p99_ms']} ms, "
              f"{st['achieved_req_s']} req/s", file=sys.stderr, flush=True)
    for row in table:
        row["bounded"] = bool(row["achieved_req_s"] >= 0.95 * row["rate_req_s"] and row["p99_ms"] <= 3 * alone_p99)
    ok_rates = [row["rate_req_s"] for row in table if row["bounded"]]
    main.update(sweep=table, max_rate_bounded_p99=max(ok_rates) if ok_rates else None,
                bounded_rule="achieved >= 0.95 x offered req/s and p99 <= 3 x alone p99",
                scenes_tris=[int(i.num_triangles) for i in infos],
                scenes_wide_nodes=[int(i.wide_nodes) for i in infos],
                scenes_bvh_depth=[int(i.max_depth) for i in infos],
                bvh_build_ms=[round(i.build_ms, 2) for i in infos], setup_s=round(setup_s, 1),
                note="samples count fwd + replay for compensation steps; latency = submit to device completion")
    return main


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(the path would shard by pixels and samples across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2503_12174_amd import dpcs, synth

    w = synth.corner_50k()
    ctx = dpcs.Context(0)
    scene = dpcs.Scene(ctx, w.mesh, bvh="sah")
    info = scene.info()
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float32)).cuda()
    alb, rough, spec, proj = dev(w.albedo), dev(w.roughness), dev(w.specular), dev(w.proj_image)
    params = dpcs.params_from(w, alb, rough, spec)
    H, W = w.camera.height, w.camera.width
    out = torch.zeros((H, W, 3), device="cuda")
    Ls = torch.zeros((H, W, w.spp, 3), device="cuda")
    rec = torch.zeros((H, W, w.spp, w.max_depth), dtype=torch.int32, device="cuda")
    G = torch.as_tensor(np.random.default_rng(7).normal(size=(H, W, 3)).astype(np.float32)).cuda()
    grads = dict(d_proj_image=torch.zeros_like(proj), d_albedo=torch.zeros_like(alb),
                 d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                 d_scalars=torch.zeros(18, device="cuda"))
    samples = H * W * w.spp

    def fwd():
        dpcs.dpcs_render(ctx, scene, params, proj, out)

    def step():   # the whole path: forward (keeping per-sample radiance and path records) + VJP by replay
        dpcs.dpcs_render(ctx, scene, params, proj, out, sample_radiance=Ls, path_records=rec)
        dpcs.dpcs_render_vjp(ctx, scene, params, proj, G, sample_radiance=Ls, path_records=rec, **grads)

    def step_retrace():   # the same step when the forward keeps only per-sample radiance: the VJP re-traces
        dpcs.dpcs_render(ctx, scene, params, proj, out, sample_radiance=Ls)
        dpcs.dpcs_render_vjp(ctx, scene, params, proj, G, sample_radiance=Ls, **grads)

    def timed(fn, k):
        for _ in range(a.warmup):
            fn()
        ctx.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        ctx.synchronize()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    ms_fwd = timed(fwd, a.steps)
    fwd_sps = samples / (ms_fwd * 1e-3)
    ms_step = timed(step, a.steps)
    step_sps = samples / (ms_step * 1e-3)
    ms_rt = timed(step_retrace, a.steps)
    rt_sps = samples / (ms_rt * 1e-3)
    print(f"[bench] forward {ms_fwd:.3f} ms, {fwd_sps:.4e} samples/s; fwd+vjp {ms_step:.3f} ms, "
          f"{step_sps:.4e} samples/s; fwd+vjp re-tracing {ms_rt:.3f} ms", file=sys.stderr, flush=True)

    roof = None
    stages = None
    if not a.quick:
        # live per-kernel timing: HIP events around every stage launch on the context's stream
        ctx.set_profiling(1)
        for _ in range(3):
            step()
        prof = ctx.profile()
        # traversal work per query (instrumented kernels, same rays; not timed)
        ctx.set_profiling(2)
        step()
        vis = ctx.profile()
        ctx.set_profiling(0)
        tr = prof["trace"]
        nodes_per_ray = vis["trace"]["nodes"] / max(vis["trace"]["items"], 1)
        tris_per_ray = vis["trace"]["tris"] / max(vis["trace"]["items"], 1)
        node_bytes = NODE4_BYTES if info.wide_nodes else NODE_BYTES
        per_ray = RAY_IO_BYTES + node_bytes * nodes_per_ray + TRI_BYTES * tris_per_ray
        rays_per_launch = tr["items"] / max(tr["launches"], 1)
        avg_ms = tr["ms"] / max(tr["launches"], 1)
        model_GBps = per_ray * rays_per_launch / (avg_ms * 1e-3) / 1e9
        ops_per_ray = OPS_RAY + (OPS_NODE4 if info.wide_nodes else OPS_NODE2) * nodes_per_ray + OPS_TRI * tris_per_ray
        achieved = ops_per_ray * rays_per_launch / (avg_ms * 1e-3) / 1e12

        def summary_json(path):
            """The fenced json block that ends a profile summary, if it was taken on
            the kernels as they are now (same source hash), else None."""
            if not os.path.exists(path):
                return None
            txt = open(path).read()
            if "```json" not in txt:
                return None
            blk = json.loads(txt.rsplit("```json", 1)[-1].split("```", 1)[0])
            return blk if blk.get("kernel_hash") == kernel_hash() else None

        tf = summary_json(TRAFFIC_FILE)
        traffic = tf.get("bytes_per_launch") if tf else None
        cf = summary_json(COUNTER_FILE)
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic,
                "kernel": "k_trace (closest-hit traversal, %s BVH)" % ("4-wide" if info.wide_nodes else "binary"),
                "ops_per_ray": round(ops_per_ray, 1), "nodes_per_ray": round(nodes_per_ray, 2),
                "tris_per_ray": round(tris_per_ray, 2), "rays_per_launch": round(rays_per_launch),
                "avg_launch_ms": round(avg_ms, 4),
                "hbm_model_bytes_per_ray": round(per_ray, 1), "hbm_model_GBps": round(model_GBps, 1)}
        if traffic:
            roof["dram_GBps"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
            roof["dram_frac"] = round(roof["dram_GBps"] / HBM_PEAK_GBS, 4)
        if cf:
            # the issue-bound decomposition from the counters of the same kernel:
            # frac ~= VALU busy x lane utilisation x (algorithmic / issued lane operations)
            issued = cf["valu_insts_per_launch"] * 64 * cf["lane_util"] / rays_per_launch
            roof.update(valu_busy=cf["valu_busy"], lane_util=cf["lane_util"],
                        valu_wave_insts_per_ray=round(cf["valu_insts_per_launch"] / rays_per_launch, 2),
                        valu_lane_ops_per_node=round(issued / max(nodes_per_ray, 1e-9), 1),
                        algorithmic_per_issued=round(ops_per_ray / issued, 3))
        stages = {k: {"launches": v["launches"], "ms": round(v["ms"], 3), "items": v["items"]}
                  for k, v in prof.items() if v["launches"]}
        sh = vis["shadow"]
        if sh["items"]:
            stages["shadow"]["nodes_per_ray"] = round(sh["nodes"] / sh["items"], 2)
            stages["shadow"]["tris_per_ray"] = round(sh["tris"] / sh["items"], 2)
        roof["rays_per_s"] = round(rays_per_launch / (avg_ms * 1e-3), 1)
        # shading's model bytes over the profiled steps (layout above): every vertex reads its
        # path state, triangle and UV records, 4 packed albedo/roughness texels, 4 specular
        # texels and writes a path record; each projector shadow record adds 4 projector
        # texels read and the record written; each continuing path writes its next state
        sd = prof["shade"]
        cont = tr["items"] - prof["raygen"]["items"]
        shade_bytes = (sd["items"] * (SHADE_STATE_IN + TRI_BYTES + UV_BYTES + 4 * 16 + 4 * 4 + 4)
                       + prof["shadow"]["items"] * (4 * 16 + SHADOW_RECORD) + cont * PATH_STATE)
        roof["shade_model_GBps"] = round(shade_bytes / (sd["ms"] * 1e-3) / 1e9, 1)
        # measured device-copy bandwidth (1 GiB read + 1 GiB written), beside the spec peak
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        roof["copy_GBps"] = round(5 * 2 * x.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        if traffic:
            roof["dram_frac_of_copy"] = round(roof["dram_GBps"] / roof["copy_GBps"], 4)
        del x, y

    if a.calib_copy:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(2):
            y.copy_(x)
        torch.cuda.synchronize()

    objective = None
    if not a.no_objective:
        objective = objective_bench(ctx, scene, params, out, (alb, rough, spec))
        print(f"[bench] objective {objective['objective_step_ms']} ms per step; D at 2048^2 "
              f"{objective['denoise_2048']['ms']} ms", file=sys.stderr, flush=True)

    configs = None
    if not a.no_configs:
        configs = configs_bench(ctx)
        print(f"[bench] configs {json.dumps(configs)}", file=sys.stderr, flush=True)

    serving = None
    if a.serving_requests > 0:
        serving = serving_bench(ctx, a.serving_requests, a.serving_alone,
                                sweep=() if a.no_serving_sweep else (30.0, 40.0, 100.0, 200.0))
        print(f"[bench] serving p50 {serving['p50_ms']} ms p99 {serving['p99_ms']} ms", file=sys.stderr, flush=True)

    cpu = None
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        O.build(force=False)
        sc = O.Scene(w)
        rng = np.random.default_rng(12345)
        order = rng.permutation(H * W)
        Gc = G.cpu().numpy().astype(np.float64)

        def oracle_step(px):   # the same step as the GPU's: forward render + VJP of the same samples
            O.render(sc, pixels=px, want=("Ec",))
            O.render_vjp(sc, Gc, pixels=px)

        t = time.perf_counter()
        oracle_step(order[:8])
        dt = time.perf_counter() - t
        n = int(max(8, min(H * W, 8 * a.cpu_seconds / max(dt, 1e-6))))
        t = time.perf_counter()
        oracle_step(order[8:8 + n])
        dt = time.perf_counter() - t
        model = "unknown"
        if os.path.exists("/proc/cpuinfo"):
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        cpu = {"value": round(n * w.spp / dt, 2), "unit": "samples/s", "cores": O.threads(sc), "kind": "oracle",
               "cpu_model": model, "host_cpus": os.cpu_count(),
               "sample": f"forward + VJP of {n} random pixels x {w.spp} spp of the same scene "
                         f"({n * w.spp} samples, {dt:.1f} s)"}
        print(f"[bench] oracle {cpu['value']:.1f} samples/s on {cpu['cores']} threads", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(step_sps, 1), "unit": "samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 traversal + f64 shading", "data": "synthetic",
        "config": {"workload": w.name, "camera": [W, H], "projector": [w.projector.width, w.projector.height],
                   "spp": w.spp, "max_depth": w.max_depth, "triangles": info.num_triangles,
                   "bvh": "binned SAH built on the device, collapsed to 4-wide", "bvh_build_ms": round(info.build_ms, 3),
                   "bvh_wide_nodes": int(info.wide_nodes),
                   "step": "forward render keeping per-sample radiance and 4-byte path records + VJP "
                           "replaying the same samples"},
        "fwd_samples_per_s": round(fwd_sps, 1), "fwd_ms": round(ms_fwd, 4),
        "fwd_adj_samples_per_s": round(step_sps, 1),
        "fwd_adj_retrace_samples_per_s": round(rt_sps, 1), "fwd_adj_retrace_ms": round(ms_rt, 4),
        "roofline": roof, "cpu_baseline": cpu, "serving": serving, "stages": stages, "objective": objective,
        "configs": configs,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
