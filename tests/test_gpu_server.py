"""Continuous-batching request loop: results alone == in the mix, admission, completion."""
import time

import numpy as np
import pytest

from paper_2503_12174_amd import synth

from .gpu_util import ctx, dev

pytestmark = pytest.mark.gpu


def _setup(n_scenes=2):
    import torch
    from paper_2503_12174_amd import dpcs
    scenes = [dpcs.Scene(ctx(), synth.folded_corner(n, 600 + n, 700 + n)) for n in (12, 30)][:n_scenes]
    albedo, rough, spec = (dev(x, torch.float32) for x in synth.ggx_textures(7, 128))
    return scenes, albedo, rough, spec


def _request(k, rng, albedo, rough, spec):
    res = int(rng.choice([16, 24, 40]))
    w = synth.corner_50k(spp=int(rng.choice([2, 4, 8])), max_depth=int(rng.integers(1, 5)), res=res, n_quads=8)
    w.projector = synth.pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, res, res)
    w.seed = k
    if k % 3 == 0:
        w.env = np.full(3, 0.03)
    img = synth.blob_image(res, res, 900 + k)
    return w, img


def _wait(srv, n, timeout=60):
    done = []
    t0 = time.time()
    while len(done) < n and time.time() - t0 < timeout:
        done += srv.poll()
        time.sleep(0.002)
    return done


def test_results_alone_equal_results_in_the_mix():
    import torch
    from paper_2503_12174_amd import dpcs
    scenes, albedo, rough, spec = _setup()
    rng = np.random.default_rng(0)
    reqs = []
    for k in range(24):
        w, img = _request(k, rng, albedo, rough, spec)
        sc = scenes[k % len(scenes)]
        p = dpcs.params_from(w, albedo, rough, spec)
        ip = dev(img, torch.float32)
        out = torch.zeros((w.camera.height, w.camera.width, 3), device="cuda")
        comp = k % 2 == 1
        grads = target = None
        if comp:
            target = dev(synth.blob_image(w.camera.height, w.camera.width, 50 + k, lo=0.1, hi=0.9), torch.float32)
            grads = dict(d_proj_image=torch.zeros_like(ip), d_albedo=torch.zeros_like(albedo),
                         d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                         d_scalars=torch.zeros(18, device="cuda"))
        reqs.append((k, w, sc, p, ip, out, target, grads))
    torch.cuda.synchronize()
    srv = dpcs.Server(ctx(), budget_bytes=8 << 30, max_slots=8)
    for k, w, sc, p, ip, out, target, grads in reqs:   # arrivals overlap the requests in flight
        assert srv.submit(k, sc, p, ip, out, target=target, grads=grads) == dpcs.OK
    done = _wait(srv, len(reqs))
    assert sorted(d[0] for d in done) == list(range(24))
    assert all(d[1] == dpcs.OK and d[2] > 0 for d in done)
    st = srv.stats()
    assert st["waves"] < 24   # requests shared launch waves
    assert st["replayed_waves"] > 0 and st["retraced_waves"] == 0   # depth <= 4: records fit
    srv.close()
    # every request alone through the plain entry points
    for k, w, sc, p, ip, out, target, grads in reqs:
        alone = torch.zeros_like(out)
        L = torch.zeros((w.camera.height, w.camera.width, w.spp, 3), device="cuda")
        dpcs.dpcs_render(ctx(), sc, p, ip, alone, sample_radiance=L)
        ctx().synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), alone.cpu().numpy(), err_msg=f"request {k}")
        if grads is not None:
            n = 3 * w.camera.height * w.camera.width
            G = 2.0 * (alone - target) / n
            g2 = {k2: torch.zeros_like(v) for k2, v in grads.items()}
            dpcs.dpcs_render_vjp(ctx(), sc, p, ip, G.contiguous(), sample_radiance=L, **g2)
            ctx().synchronize()
            for name in grads:
                a, b = grads[name].cpu().numpy(), g2[name].cpu().numpy()
                scale = np.abs(b).max() + 1e-30
                np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * scale, err_msg=f"request {k} {name}")


def test_full_waves_with_overlapped_shadow_rays():
    """Waves of 2^21 paths put their shadow rays (forward, and the re-traced adjoint's) on
    a second stream beside the next depth's closest hit: a large relight request (env on:
    both shadow queues) and a depth-20 compensation step (its path records exceed the
    loop's record buffer of 8 words per path: re-traced) through the loop equal the plain
    entry points."""
    import torch
    from paper_2503_12174_amd import dpcs
    scene = dpcs.Scene(ctx(), synth.folded_corner(30, 630, 730))
    albedo, rough, spec = (dev(x, torch.float32) for x in synth.ggx_textures(7, 128))
    reqs = []
    for k, (spp, depth, comp) in enumerate([(64, 3, False), (32, 20, True)]):
        w = synth.corner_50k(spp=spp, max_depth=depth, res=256, n_quads=8)
        w.seed = 40 + k
        w.env = np.full(3, 0.03)
        p = dpcs.params_from(w, albedo, rough, spec)
        ip = dev(synth.blob_image(256, 256, 910 + k), torch.float32)
        out = torch.zeros((256, 256, 3), device="cuda")
        grads = target = None
        if comp:
            target = dev(synth.blob_image(256, 256, 60 + k, lo=0.1, hi=0.9), torch.float32)
            grads = dict(d_proj_image=torch.zeros_like(ip), d_albedo=torch.zeros_like(albedo),
                         d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                         d_scalars=torch.zeros(18, device="cuda"))
        reqs.append((k, w, p, ip, out, target, grads))
    torch.cuda.synchronize()
    srv = dpcs.Server(ctx(), budget_bytes=16 << 30, max_slots=4)
    for k, w, p, ip, out, target, grads in reqs:
        assert srv.submit(k, scene, p, ip, out, target=target, grads=grads) == dpcs.OK
    done = _wait(srv, len(reqs), timeout=120)
    assert sorted(d[0] for d in done) == [0, 1] and all(d[1] == dpcs.OK for d in done)
    assert srv.stats()["retraced_waves"] > 0
    srv.close()
    for k, w, p, ip, out, target, grads in reqs:
        alone = torch.zeros_like(out)
        L = torch.zeros((256, 256, w.spp, 3), device="cuda")
        dpcs.dpcs_render(ctx(), scene, p, ip, alone, sample_radiance=L)
        ctx().synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), alone.cpu().numpy(), err_msg=f"request {k}")
        if grads is not None:
            G = 2.0 * (alone - target) / (3 * 256 * 256)
            g2 = {k2: torch.zeros_like(v) for k2, v in grads.items()}
            dpcs.dpcs_render_vjp(ctx(), scene, p, ip, G.contiguous(), sample_radiance=L, **g2)
            ctx().synchronize()
            for name in grads:
                a, b = grads[name].cpu().numpy(), g2[name].cpu().numpy()
                np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * (np.abs(b).max() + 1e-30), err_msg=name)


def test_one_request_waves_bin_their_gradients():
    """Compensation steps submitted one at a time run alone in their waves: their map
    cotangents are binned and flushed (no atomics), and the gradients equal the plain
    VJP's."""
    import torch
    from paper_2503_12174_amd import dpcs
    scenes, albedo, rough, spec = _setup(1)
    rng = np.random.default_rng(5)
    srv = dpcs.Server(ctx(), budget_bytes=8 << 30, max_slots=4)
    for k in range(3):
        w, img = _request(2 * k + 1, rng, albedo, rough, spec)
        w.max_depth = 2 + k   # depths 2, 3 and 4
        p = dpcs.params_from(w, albedo, rough, spec)
        ip = dev(img, torch.float32)
        out = torch.zeros((w.camera.height, w.camera.width, 3), device="cuda")
        target = dev(synth.blob_image(w.camera.height, w.camera.width, 70 + k, lo=0.1, hi=0.9), torch.float32)
        grads = dict(d_proj_image=torch.zeros_like(ip), d_albedo=torch.zeros_like(albedo),
                     d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                     d_scalars=torch.zeros(18, device="cuda"))
        before = srv.stats()["binned_waves"]
        assert srv.submit(k, scenes[0], p, ip, out, target=target, grads=grads) == dpcs.OK
        done = _wait(srv, 1)
        assert len(done) == 1 and done[0][1] == dpcs.OK
        assert srv.stats()["binned_waves"] > before
        L = torch.zeros((w.camera.height, w.camera.width, w.spp, 3), device="cuda")
        alone = torch.zeros_like(out)
        dpcs.dpcs_render(ctx(), scenes[0], p, ip, alone, sample_radiance=L)
        G = 2.0 * (alone - target) / (3 * w.camera.height * w.camera.width)
        g2 = {name: torch.zeros_like(v) for name, v in grads.items()}
        dpcs.dpcs_render_vjp(ctx(), scenes[0], p, ip, G.contiguous(), sample_radiance=L, **g2)
        ctx().synchronize()
        for name in grads:
            a, b = grads[name].cpu().numpy(), g2[name].cpu().numpy()
            np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * (np.abs(b).max() + 1e-30), err_msg=f"{k} {name}")
    srv.close()


def test_admission_by_memory_budget():
    import torch
    from paper_2503_12174_amd import dpcs
    scenes, albedo, rough, spec = _setup(1)
    rng = np.random.default_rng(1)
    w, img = _request(0, rng, albedo, rough, spec)
    p = dpcs.params_from(w, albedo, rough, spec)
    ip = dev(img, torch.float32)
    budget = 1 << 30
    srv = dpcs.Server(ctx(), budget_bytes=budget, max_slots=4)
    outs = []
    for k in range(6):
        out = torch.zeros((w.camera.height, w.camera.width, 3), device="cuda")
        outs.append(out)
        assert srv.submit(k, scenes[0], p, ip, out) == dpcs.OK
    done = _wait(srv, 6)
    assert len(done) == 6
    assert srv.stats()["peak_bytes"] <= budget
    # a compensation step with 4096^2 maps and projector needs > 1 GiB of request state:
    # rejected up front (every buffer it names exists, so nothing could be read out of bounds)
    n = 4096
    big = synth.corner_50k(spp=1, max_depth=1, res=16, n_quads=8)
    big.projector = synth.pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, n, n)
    alb_b = torch.full((n, n, 3), 0.5, device="cuda")
    r_b = torch.full((n, n), 0.5, device="cuda")
    s_b = torch.full((n, n), 0.5, device="cuda")
    ip_b = torch.full((n, n, 3), 0.5, device="cuda")
    pb = dpcs.params_from(big, alb_b, r_b, s_b)
    out_b = torch.zeros((16, 16, 3), device="cuda")
    grads = dict(d_proj_image=torch.zeros_like(ip_b), d_albedo=torch.zeros_like(alb_b),
                 d_roughness=torch.zeros_like(r_b), d_specular=torch.zeros_like(s_b),
                 d_scalars=torch.zeros(18, device="cuda"))
    st2 = srv.submit(99, scenes[0], pb, ip_b, out_b, target=torch.zeros_like(out_b), grads=grads)
    assert st2 == dpcs.E_REJECTED
    assert srv.stats()["rejected"] == 1
    assert srv.close() == dpcs.OK
    for o in outs[1:]:
        np.testing.assert_array_equal(o.cpu().numpy(), outs[0].cpu().numpy())


def test_scene_in_use_cannot_be_destroyed():
    import torch
    from paper_2503_12174_amd import dpcs
    scenes, albedo, rough, spec = _setup(1)
    w = synth.corner_50k(spp=256, max_depth=4, res=64, n_quads=8)
    p = dpcs.params_from(w, albedo, rough, spec)
    ip = dev(synth.blob_image(256, 256, 3), torch.float32)
    srv = dpcs.Server(ctx(), budget_bytes=4 << 30, max_slots=4)
    out = torch.zeros((64, 64, 3), device="cuda")
    assert srv.submit(1, scenes[0], p, ip, out) == dpcs.OK
    st = dpcs.lib().dpcs_scene_destroy(scenes[0].h)
    done = _wait(srv, 1)
    assert len(done) == 1
    srv.close()
    assert st in (dpcs.E_BUSY, dpcs.OK)
    if st == dpcs.OK:
        scenes[0].h = None


def test_retraced_adjoint_in_the_mix():
    """Compensation steps whose paths are too deep for the wave's path records (depth 10,
    records hold 8 vertices per path): the loop re-traces their adjoint instead of
    replaying records; each result still equals the request run alone.  Each request
    alone (128^2 x 16 samples) fills a wave, so its first wave re-traces whatever the
    arrival timing."""
    import torch
    from paper_2503_12174_amd import dpcs
    scenes, albedo, rough, spec = _setup(1)
    reqs = []
    for k in range(4):
        w = synth.corner_50k(spp=16, max_depth=10, res=128, n_quads=8)
        w.projector = synth.pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, 64, 64)
        w.seed = 40 + k
        p = dpcs.params_from(w, albedo, rough, spec)
        ip = dev(synth.blob_image(64, 64, 300 + k), torch.float32)
        out = torch.zeros((128, 128, 3), device="cuda")
        target = dev(synth.blob_image(128, 128, 400 + k, lo=0.1, hi=0.9), torch.float32)
        grads = dict(d_proj_image=torch.zeros_like(ip), d_albedo=torch.zeros_like(albedo),
                     d_roughness=torch.zeros_like(rough), d_specular=torch.zeros_like(spec),
                     d_scalars=torch.zeros(18, device="cuda"))
        reqs.append((k, w, p, ip, out, target, grads))
    torch.cuda.synchronize()
    # 512 MiB: ~228k paths per wave, records for 8 x that many vertices; a request of
    # 128^2 x 16 = 262k samples fills a wave with adjoint paths needing 10 vertices each
    srv = dpcs.Server(ctx(), budget_bytes=512 << 20, max_slots=8)
    for k, w, p, ip, out, target, grads in reqs:
        assert srv.submit(k, scenes[0], p, ip, out, target=target, grads=grads) == dpcs.OK
    done = _wait(srv, len(reqs))
    assert sorted(d[0] for d in done) == list(range(4))
    assert all(d[1] == dpcs.OK for d in done)
    assert srv.stats()["retraced_waves"] > 0
    srv.close()
    for k, w, p, ip, out, target, grads in reqs:
        alone = torch.zeros_like(out)
        L = torch.zeros((128, 128, w.spp, 3), device="cuda")
        dpcs.dpcs_render(ctx(), scenes[0], p, ip, alone, sample_radiance=L)
        ctx().synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), alone.cpu().numpy(), err_msg=f"request {k}")
        G = 2.0 * (alone - target) / (3 * 128 * 128)
        g2 = {k2: torch.zeros_like(v) for k2, v in grads.items()}
        dpcs.dpcs_render_vjp(ctx(), scenes[0], p, ip, G.contiguous(), sample_radiance=L, **g2)
        ctx().synchronize()
        for name in grads:
            a, b = grads[name].cpu().numpy(), g2[name].cpu().numpy()
            scale = np.abs(b).max() + 1e-30
            np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * scale, err_msg=f"request {k} {name}")


def test_request_waits_for_its_input_stream():
    """The projector image is written on a side stream behind ~10 ms of other work and
    the request is submitted at once with that stream: the loop's first launch waits for
    it, so the result equals a plain render of the final image; the latency parts of
    the completed request add up to no more than its latency."""
    import torch
    from paper_2503_12174_amd import dpcs
    scenes, albedo, rough, spec = _setup(1)
    w = synth.corner_50k(spp=4, max_depth=2, res=64, n_quads=8)
    w.projector = synth.pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, 64, 64)
    p = dpcs.params_from(w, albedo, rough, spec)
    final = dev(synth.blob_image(64, 64, 77), torch.float32)
    ip = torch.zeros_like(final)
    out = torch.zeros((64, 64, 3), device="cuda")
    a = torch.randn(4096, 4096, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    srv = dpcs.Server(ctx(), budget_bytes=512 << 20, max_slots=4)
    with torch.cuda.stream(side):
        acc = a
        for _ in range(8):
            acc = (acc @ a) * 1e-3
        ip.copy_(final)
    assert srv.submit(0, scenes[0], p, ip, out, stream=side) == dpcs.OK
    done = _wait(srv, 1)
    assert len(done) == 1 and done[0][1] == dpcs.OK
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    alone = torch.zeros_like(out)
    dpcs.dpcs_render(ctx(), scenes[0], p, final, alone)
    ctx().synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), alone.cpu().numpy())
    assert 0 <= st["wait_us"] and 0 <= st["admit_us"] and 0 <= st["run_us"]
    assert (st["wait_us"] + st["admit_us"] + st["run_us"]) * 1e-3 <= done[0][2] + 1.0
    del acc
