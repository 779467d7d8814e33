// vjp.cpp -- dpcs_render_vjp: per launch wave of whole pixels, forward samples with path
// records (unless the caller hands in the forward call's per-sample radiance), CRF/clip
// backward, path replay with gradient scatter; finally the PRF backward and scalar
// reductions.
#include <algorithm>

#include "runtime.hpp"

using namespace dpcs;

extern "C" dpcs_status dpcs_render_vjp(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                                       const float* proj_image, const float* grad_image, const float* sample_radiance,
                                       const uint32_t* path_records, const dpcs_grads* grads) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->sticky) return DPCS_E_DEVICE;
    if (!scene || scene->ctx != ctx) return fail(ctx, DPCS_E_INVALID, "scene is NULL or from another context");
    if (!grad_image) return fail(ctx, DPCS_E_INVALID, "grad_image is NULL");
    if (!grads) return fail(ctx, DPCS_E_INVALID, "grads is NULL");
    if (path_records && !sample_radiance)
        return fail(ctx, DPCS_E_INVALID, "path_records need the sample_radiance of the same forward call");
    (void)hipGetLastError();
    ReqDesc r;
    std::string why;
    if (!fill_desc(ctx, r, params, scene, proj_image, &why)) return fail(ctx, DPCS_E_INVALID, why);
    const bool ext = params->metallic || params->normal_map;
    if (ext && sample_radiance && !path_records)
        return fail(ctx, DPCS_E_UNSUPPORTED, "with the metallic or normal map the VJP replays path records: pass the "
                                             "forward's path_records with sample_radiance, or neither");
    if (grads->d_camera && sample_radiance && !path_records)
        return fail(ctx, DPCS_E_UNSUPPORTED, "the camera-pose gradient replays path records: pass the forward's "
                                             "path_records with sample_radiance, or neither");
    const double edge_density = grads->camera_edge_density;
    if (!(edge_density >= 0.0 && edge_density <= 1e6))
        return fail(ctx, DPCS_E_INVALID, "camera_edge_density must be in [0, 1e6]");
    if (edge_density > 0.0 && !grads->d_camera)
        return fail(ctx, DPCS_E_INVALID, "camera_edge_density needs d_camera");
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    r.grad_image = grad_image;
    dpcs_status st = DPCS_OK;
    if (!prepare_request(ctx, r, params, "vjp", &st)) return st;
    const size_t nEp = (size_t)r.Wp * r.Hp, nT = (size_t)r.tw * r.th;
    float* dEp = (float*)scratch(ctx, "vjp.dEp", sizeof(float) * 4 * nEp, &st);
    if (!dEp) return st;
    const int C = r.dtex_c;   // cotangent channels per texel: 5, or 9 with the metallic / normal maps
    float* dtex = (float*)scratch(ctx, "vjp.dtex", sizeof(float) * C * nT, &st);
    if (!dtex) return st;
    float* acc = (float*)scratch(ctx, "vjp.acc", sizeof(float) * 32, &st);
    if (!acc) return st;
    Launch l{ctx->stream, ctx->grid_cap};
    ZeroList zl(l);   // the accumulators, cleared by one launch before the first wave
    zl.add(dEp, 4 * (int64_t)nEp);
    zl.add(dtex, C * (int64_t)nT);
    zl.add(acc, 32);
    r.dEp = dEp;
    r.d_tex = dtex;
    r.d_acc = acc;
    const int64_t npix = (int64_t)r.Wc * r.Hc;
    const int64_t cap = std::min<int64_t>(std::max<int64_t>(ctx->capacity, r.spp), npix * r.spp);
    const int64_t ppw = std::max<int64_t>(1, cap / r.spp);
    // scalar sums reduced in a fixed order: the same gradients on every run
    r.d_part = (float*)scratch(ctx, "vjp.partials", sizeof(float) * partial_floats(ppw, (int64_t)nEp), &st);
    if (!r.d_part) return st;
    if (grads->d_camera) {
        r.d_cam_part = (float*)scratch(ctx, "vjp.camera_partials", sizeof(float) * cam_partial_floats(ppw * r.spp), &st);
        if (!r.d_cam_part) return st;
    }
    // the boundary part of the camera-pose gradient needs every pixel's cotangent
    float4* pix_dE = nullptr;
    if (edge_density > 0.0) {
        pix_dE = (float4*)scratch(ctx, "vjp.pixel_cotangents", sizeof(float4) * npix, &st);
        if (!pix_dE) return st;
        zl.add((float*)pix_dE, 4 * npix);
    }
    Queues q{};
    AdjQueues aq{};
    if (!make_queues(ctx, "fwd.queues", ppw * r.spp, q, &st)) return st;
    if (!make_adj_queues(ctx, "vjp.queues", ppw * r.spp, aq, &st, ext)) return st;
    // Path records: the caller's (whole image, from the forward call that produced
    // sample_radiance), or this call's own per wave when it runs the forward itself.
    // With sample_radiance alone the replay traces again.
    uint32_t* wave_rec = nullptr;
    const bool own_rec = !sample_radiance;
    if ((own_rec || path_records) && scene->nt >= (int)REC_LEAF)
        return fail(ctx, DPCS_E_UNSUPPORTED, "path records need < 2^30 triangles");
    if (own_rec) {
        wave_rec = (uint32_t*)scratch(ctx, "vjp.records", sizeof(uint32_t) * (size_t)(ppw * r.spp) * r.max_depth, &st);
        if (!wave_rec) return st;
    }
    {   // the replay bins its map cotangents: per group of k depths at most k + 1 texture
        // records per path (one per vertex, one more where a path ends) -- the re-tracing
        // replay writes one per vertex and one per unoccluded shadow ray, at most 3 per
        // vertex -- and one E_p record per vertex
        const int64_t k = std::min(r.max_depth, BIN_DEPTHS);
        const int64_t per = (own_rec || path_records) ? k + 1 : 3 * k;
        if (ext) make_map_bins(ctx, zl, aq.tb, "vjp.tex9_bins", r.tw, r.th, 9, 12, ppw * r.spp * per);
        else make_map_bins(ctx, zl, aq.tb, "vjp.tex_bins", r.tw, r.th, 5, 8, ppw * r.spp * per);
        make_map_bins(ctx, zl, aq.eb, "vjp.ep_bins", r.Wp, r.Hp, 3, 6, ppw * r.spp * k);
    }
    zl.launch();
    // the forward run here and the re-tracing replay put shadow rays on the side stream
    int* spill2 = (own_rec || !path_records) ? side_spill(ctx, q) : nullptr;
    for (int64_t a = 0; a < npix; a += ppw) {
        const uint32_t b = (uint32_t)std::min(npix, a + ppw);
        if (own_rec) {
            r.rec = wave_rec;
            r.rec_g0 = (uint32_t)a * (uint32_t)r.spp;
            forward_wave(ctx, q, r, (uint32_t)a, b, false, spill2);
        } else {
            r.rec = const_cast<uint32_t*>(path_records);   // read only in the adjoint
            r.rec_g0 = 0;
        }
        adjoint_wave(ctx, q, aq, r, (uint32_t)a, b, sample_radiance, pix_dE, spill2);
    }
    if (pix_dE) {
        st = camera_edge_term(ctx, scene, r, q, edge_density, params->camera.K, pix_dE, acc + 20);
        if (st != DPCS_OK) return st;
    }
    launch_adj_finish(l, r, grads->d_proj_image, grads->d_albedo, grads->d_roughness, grads->d_specular,
                      grads->d_scalars, acc, grads->d_metallic, grads->d_normal_map);
    if (grads->d_camera &&
        !hip_ok(ctx, hipMemcpyAsync(grads->d_camera, acc + 20, 12 * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream),
                "camera gradient copy"))
        return DPCS_E_DEVICE;
    if (!hip_ok(ctx, hipGetLastError(), "kernel launch")) return DPCS_E_DEVICE;
    ctx->err.clear();
    return DPCS_OK;
}
