"""DPCS project-and-capture path tracing on MI355X (gfx950): forward rendering
I_c = R(I_p, theta), its vector-Jacobian product, the training objective's operators
and a continuous-batching request loop, as HIP kernels behind the C ABI of
include/dpcs.h (libdpcs.so, built by build.py).

    from paper_2503_12174_amd import dpcs, synth, autograd, objective
    w = synth.corner_50k()                      # seeded synthetic workload
    ctx = dpcs.Context(0)                       # device 0, torch's current stream
    scene = dpcs.Scene(ctx, w.mesh, bvh="sah")  # resident mesh + 4-wide BVH
    img = autograd.render(ctx, scene, w, proj, albedo, rough, spec, scalars)   # Eq. 7
    loss = objective.l1(ctx, objective.denoise(ctx, img, guide), target)       # Eq. 9, 11
    loss.backward()                             # path-replay VJP into every input

dpcs.py      ctypes binding of the C ABI (argument marshalling only; raises when the
             library is missing, there is no CPU fallback)
autograd.py  torch.autograd.Function over dpcs_render / dpcs_render_vjp
objective.py denoiser, guide features, L1 and map regulariser as autograd Functions
drivers.py   Adam loops for projector compensation (Eq. 13) and scene fitting (Eq. 9)
synth.py     seeded input generators (meshes, maps, images, request streams)
"""
