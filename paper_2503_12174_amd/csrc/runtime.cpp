// runtime.cpp -- C ABI implementation: context, scratch pool, scene residency and BVH
// build, forward render orchestration, debug entry points.
#include "runtime.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace dpcs;

// Scratch of dpcs_render_noalloc: one copy per device, held until the process ends.  Host
// code never uses this name as an address (here it is a host-side stand-in); the device
// address of each GPU's copy is looked up once per device at context creation and kept in
// noalloc_ptr.
constexpr size_t NOALLOC_BYTES = size_t(DPCS_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char noalloc_scratch[NOALLOC_BYTES];
static std::mutex noalloc_mu;
static std::vector<void*> noalloc_ptr;          // per device, null until looked up
static std::vector<hipError_t> noalloc_status;  // per device: result of the lookup

namespace dpcs {

dpcs_status fail(dpcs_context ctx, dpcs_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

bool hip_ok(dpcs_context ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    if (ctx) {
        ctx->sticky = true;
        ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return false;
}

void* scratch(dpcs_context ctx, const char* name, size_t bytes, dpcs_status* st) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = ctx->pool.find(name);
    if (it != ctx->pool.end() && it->second.second >= bytes) return it->second.first;
    size_t old = it != ctx->pool.end() ? it->second.second : 0;
    if (ctx->scratch_limit && ctx->scratch_bytes - old + bytes > ctx->scratch_limit) {
        *st = fail(ctx, DPCS_E_OOM, std::string("scratch limit exceeded by buffer ") + name);
        return nullptr;
    }
    if (it != ctx->pool.end()) {
        // the old buffer may still be read by queued work
        if (!hip_ok(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize")) {
            *st = DPCS_E_DEVICE;
            return nullptr;
        }
        (void)hipFree(it->second.first);
        ctx->scratch_bytes -= old;
        ctx->pool.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *st = fail(ctx, DPCS_E_OOM, std::string("hipMalloc failed for buffer ") + name);
        return nullptr;
    }
    ctx->pool[name] = {p, bytes};
    ctx->scratch_bytes += bytes;
    return p;
}

size_t queue_bytes(int64_t cap, int trace_blocks) {
    // per path: 2 x (PathO 32 + PathD 32 + beta 16) + hit 4 + 2 x shadow (48 + 4) + L 16,
    // the traversal spill region of trace_blocks workgroups, and 256 bytes of alignment
    // slack per part (18 parts)
    return (size_t)cap * (2 * 80 + 4 + 2 * 52 + 16) + 4 * (size_t)trace_blocks * TRACE_TB * SPILL + 32 * 256;
}

void carve_queues(char* b, int64_t cap, int trace_blocks, Queues& q) {
    const size_t c = (size_t)cap;
    auto take = [&](size_t n) {   // 256-byte aligned parts
        char* p = b;
        b += (n + 255) & ~size_t(255);
        return (void*)p;
    };
    for (int k = 0; k < 2; ++k) {
        q.po[k] = (PathO*)take(32 * c);
        q.pd[k] = (PathD*)take(32 * c);
        q.pb[k] = (float4*)take(16 * c);
        q.so[k] = (float4*)take(16 * c);
        q.sd[k] = (float4*)take(16 * c);
        q.sc[k] = (float4*)take(16 * c);
        q.st[k] = (float*)take(4 * c);
    }
    q.hit = (int*)take(4 * c);
    q.L = (float4*)take(16 * c);
    q.cnt = (uint32_t*)take(4 * (SHADOW_CNT + 4));
    q.spill = (int*)take(4 * (size_t)trace_blocks * TRACE_TB * SPILL);
    q.trace_blocks = trace_blocks;
    q.cap = cap;
    q.stats = nullptr;
}

bool make_queues(dpcs_context ctx, const char* name, int64_t cap, Queues& q, dpcs_status* st) {
    const int tb = trace_grid_cap(ctx->grid_cap, TRACE_ROUNDS);
    char* b = (char*)scratch(ctx, name, queue_bytes(cap, tb), st);
    if (!b) return false;
    carve_queues(b, cap, tb, q);
    return true;
}

bool make_adj_queues(dpcs_context ctx, const char* name, int64_t cap, AdjQueues& aq, dpcs_status* st, bool ext) {
    const size_t c = (size_t)cap;
    // per path 2 x 144 + 16 bytes (+ 2 x 112 with the metallic / normal maps); + 256 bytes
    // of alignment slack per part (27 parts)
    const size_t bytes = c * (2 * 144 + 16 + (ext ? 2 * (sizeof(PendX) + 16) : 0)) + 32 * 256;
    char* b = (char*)scratch(ctx, name, bytes, st);
    if (!b) return false;
    auto take = [&](size_t n) {
        char* p = b;
        b += (n + 255) & ~size_t(255);
        return (void*)p;
    };
    for (int k = 0; k < 2; ++k) {
        aq.rl[k] = (float4*)take(16 * c);
        aq.puv[k] = (double2*)take(16 * c);
        aq.pend[k] = (float2*)take(8 * c);
        aq.penda[k] = (float4*)take(16 * c);
        aq.sproj[k] = (double2*)take(16 * c);
        aq.suv[k] = (double2*)take(16 * c);
        aq.sg[k] = (float4*)take(16 * c);
        aq.sa[k] = (float4*)take(16 * c);
        aq.ss[k] = (float*)take(4 * c);
        aq.pn[k] = (float4*)take(16 * c);
        aq.pns[k] = (float*)take(4 * c);
        aq.px[k] = ext ? (PendX*)take(sizeof(PendX) * c) : nullptr;
        aq.pnx[k] = ext ? (float4*)take(16 * c) : nullptr;
    }
    aq.delta = (float4*)take(16 * c);
    aq.tb = MapBins{};
    aq.eb = MapBins{};
    return true;
}

// Record buffers of the binned map-cotangent flush for a W x H map with C values per
// texel (their counters go on zl to be cleared); leaves mb empty (direct atomics) when
// the map has too many tiles or the scratch allocation fails.
void make_map_bins(dpcs_context ctx, ZeroList& zl, MapBins& mb, const char* name, int W, int H, int C, int RS,
                   int64_t cap) {
    mb = MapBins{};
    int T = 0, nbx = 0, nby = 0;
    if (!map_tiling(W, H, T, nbx, nby)) return;
    cap = std::min<int64_t>(cap, int64_t(1) << 31);
    const int nb = nbx * nby;
    const size_t rec = 4 * (size_t)RS * cap, stage = 8 * (size_t)((cap + ACC_CHUNK - 1) / ACC_CHUNK + nb) * (T + 1) * (T + 1) * C;
    const size_t rows = 4 * (size_t)((cap + BIN_CHUNK - 1) / BIN_CHUNK) * nb;
    const size_t bytes = 2 * rec + stage + rows + 4 * (3 * (size_t)nb + 2) + 8 * 256;
    dpcs_status st = DPCS_OK;
    char* b = (char*)scratch(ctx, name, bytes, &st);
    if (!b) {   // run without binning
        ctx->err.clear();
        return;
    }
    auto take = [&](size_t n) {
        char* p = b;
        b += (n + 255) & ~size_t(255);
        return (void*)p;
    };
    mb.rec = (float*)take(rec);
    mb.sorted = (float*)take(rec);
    mb.stage = (long long*)take(stage);
    mb.count = (uint32_t*)take(4);
    mb.bins = (uint32_t*)take(4 * (3 * (size_t)nb + 2));
    mb.rowbase = (uint32_t*)take(rows);
    mb.cap = cap;
    mb.W = W;
    mb.H = H;
    mb.T = T;
    mb.nbx = nbx;
    mb.nby = nby;
    mb.nb = nb;
    zl.add((float*)mb.count, 1);
    zl.add((float*)mb.bins, 3 * (int64_t)nb + 2);
}

static void inv3(const double* m, double* o) {
    const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7], i = m[8];
    const double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    const double det = a * A + b * B + c * C;
    o[0] = A / det;
    o[1] = -(b * i - c * h) / det;
    o[2] = (b * f - c * e) / det;
    o[3] = B / det;
    o[4] = (a * i - c * g) / det;
    o[5] = -(a * f - c * d) / det;
    o[6] = C / det;
    o[7] = -(a * h - b * g) / det;
    o[8] = (a * e - b * d) / det;
}

static double det3(const double* m) {
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

static bool pinhole_ok(const dpcs_pinhole& p, const char* what, std::string* why) {
    if (p.width <= 0 || p.height <= 0 || p.width > 16384 || p.height > 16384) {
        *why = std::string(what) + ": width/height must be in 1..16384";
        return false;
    }
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(p.K[k]) || !std::isfinite(p.R[k])) {
            *why = std::string(what) + ": K and R must be finite";
            return false;
        }
    if (!(std::fabs(det3(p.K)) > 1e-12)) {
        *why = std::string(what) + ": K is not invertible";
        return false;
    }
    return true;
}

bool fill_desc(dpcs_context, ReqDesc& r, const dpcs_render_params* p, dpcs_scene sc, const float* proj_image,
               std::string* why, bool need_proj) {
    std::memset(&r, 0, sizeof r);
    if (!p) return *why = "params is NULL", false;
    if (!pinhole_ok(p->camera, "camera", why) || !pinhole_ok(p->projector, "projector", why)) return false;
    if (p->brdf != DPCS_BRDF_LAMBERT && p->brdf != DPCS_BRDF_GGX) return *why = "brdf must be LAMBERT or GGX", false;
    if (!p->albedo) return *why = "albedo is NULL", false;
    if (p->brdf == DPCS_BRDF_GGX && (!p->roughness || !p->specular))
        return *why = "GGX needs roughness and specular maps", false;
    if (p->tex_w <= 0 || p->tex_h <= 0 || p->tex_w > 16384 || p->tex_h > 16384)
        return *why = "tex_w/tex_h must be in 1..16384", false;
    if (p->spp < 1 || p->spp > 65536) return *why = "spp must be in 1..65536", false;
    if (p->max_depth < 1 || p->max_depth > 64) return *why = "max_depth must be in 1..64", false;
    if (need_proj && !proj_image) return *why = "proj_image is NULL", false;
    if (!p->device_scalars) {
        for (int c = 0; c < 3; ++c) {
            if (!(p->prf_gamma[c] > 0.f) || !(p->crf_gamma[c] > 0.f)) return *why = "gammas must be > 0", false;
            if (!(p->white_balance[c] > 0.f)) return *why = "white balance must be > 0", false;
        }
    }
    if (!(p->prf_gain >= 0.f) || !(p->crf_gain >= 0.f)) return *why = "gains must be >= 0", false;
    if (p->clip_enable && !(p->clip_k > 0.f)) return *why = "clip_k must be > 0", false;
    const int64_t pix = (int64_t)p->camera.width * p->camera.height;
    if (pix * p->spp >= (int64_t(1) << 32)) return *why = "pixels x spp must be < 2^32", false;

    double Ki[9];
    inv3(p->camera.K, Ki);
    const double* R = p->camera.R;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.cam_M[3 * i + j] = R[i] * Ki[j] + R[3 + i] * Ki[3 + j] + R[6 + i] * Ki[6 + j];
    for (int i = 0; i < 3; ++i)
        r.cam_o[i] = -(R[i] * p->camera.t[0] + R[3 + i] * p->camera.t[1] + R[6 + i] * p->camera.t[2]);
    for (int k = 0; k < 9; ++k) {
        r.cam_R[k] = R[k];
        r.cam_Ki[k] = Ki[k];
    }
    for (int i = 0; i < 3; ++i) r.cam_t[i] = p->camera.t[i];
    r.Wc = p->camera.width;
    r.Hc = p->camera.height;
    const double* Rp = p->projector.R;
    for (int k = 0; k < 9; ++k) r.prj_R[k] = Rp[k];
    for (int i = 0; i < 3; ++i) {
        r.prj_t[i] = p->projector.t[i];
        r.prj_o[i] = -(Rp[i] * p->projector.t[0] + Rp[3 + i] * p->projector.t[1] + Rp[6 + i] * p->projector.t[2]);
    }
    for (int k = 0; k < 6; ++k) r.prj_K[k] = p->projector.K[k];
    r.Wp = p->projector.width;
    r.Hp = p->projector.height;
    r.nodes = sc->nodes;
    r.nodes4 = sc->nodes4;
    r.tris = sc->tris;
    r.top_nodes = sc->nodes4 ? std::min(TOP_NODES, sc->nnodes4) : 0;
    r.tri_uv = sc->tri_uv;
    r.emission = sc->emission;
    r.tmin = sc->tmin;
    r.brdf = p->brdf;
    r.tw = p->tex_w;
    r.th = p->tex_h;
    r.spec = p->brdf == DPCS_BRDF_GGX ? p->specular : nullptr;
    r.env_on = 0;
    for (int c = 0; c < 3; ++c) {
        r.env[c] = p->env_radiance[c];
        if (p->env_radiance[c] != 0.f) r.env_on = 1;
    }
    r.spp = p->spp;
    r.max_depth = p->max_depth;
    r.seed_lo = (uint32_t)p->seed;
    r.seed_hi = (uint32_t)(p->seed >> 32);
    r.sample_offset = p->sample_offset;
    r.prf_gain = p->prf_gain;
    r.crf_gain = p->crf_gain;
    r.clip = p->clip_enable ? 1 : 0;
    r.clip_k = p->clip_k;
    for (int c = 0; c < 3; ++c) {
        r.scal[c] = p->prf_gamma[c];
        r.scal[12 + c] = p->crf_gamma[c];
        r.scal[15 + c] = p->white_balance[c];
    }
    for (int k = 0; k < 9; ++k) r.scal[3 + k] = p->prf_mix[k];
    r.dscal = p->device_scalars;
    r.proj_image = proj_image;
    r.dtex_c = (p->metallic || p->normal_map) ? 9 : 5;   // tex4b is set where the maps are packed
    return true;
}


static hipEvent_t prof_event(dpcs_context ctx) {
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_used++];
}

int prof_begin(dpcs_context ctx, int stage) {
    if (!ctx->prof_mode) return -1;
    hipEvent_t a = prof_event(ctx), b = prof_event(ctx);
    if (!a || !b) return -1;
    (void)hipEventRecord(a, ctx->stream);
    ctx->prof.push_back({stage, a, b, -1, 0});
    return (int)ctx->prof.size() - 1;
}

void prof_end(dpcs_context ctx, int rec, const uint32_t* dev_count, int64_t host_count) {
    if (rec < 0) return;
    auto& r = ctx->prof[rec];
    (void)hipEventRecord(r.b, ctx->stream);
    r.host_count = host_count;
    if (dev_count && ctx->pinned && ctx->pinned_used < ctx->pinned_cap) {
        r.slot = ctx->pinned_used++;
        (void)hipMemcpyAsync(ctx->pinned + r.slot, dev_count, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream);
    }
}

unsigned long long* prof_stats(dpcs_context ctx, int stage) {
    return ctx->prof_mode >= 2 && ctx->dstats ? ctx->dstats + 2 * stage : nullptr;
}

}  // namespace dpcs

// ====================================================================== context
extern "C" dpcs_status dpcs_context_create(int32_t device, void* hip_stream, size_t scratch_limit_bytes,
                                           dpcs_context* out) {
    if (!out) return DPCS_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return DPCS_E_INVALID;
    }
    if (hipSetDevice(device) != hipSuccess) return DPCS_E_DEVICE;
    hipError_t na = hipSuccess;
    void* na_ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(noalloc_mu);
        if ((int)noalloc_ptr.size() < n) {
            noalloc_ptr.resize(n, nullptr);
            noalloc_status.resize(n, hipErrorNotReady);
        }
        if (!noalloc_ptr[device]) {
            void* p = nullptr;
            noalloc_status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
            if (noalloc_status[device] == hipSuccess) noalloc_ptr[device] = p;
            else (void)hipGetLastError();
        }
        na = noalloc_status[device];
        na_ptr = noalloc_ptr[device];
    }
    auto* c = new dpcs_context_s();
    c->device = device;
    c->noalloc = na_ptr;
    c->noalloc_err = (int)na;
    c->stream = (hipStream_t)hip_stream;
    c->scratch_limit = scratch_limit_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->grid_cap = std::max(1024, prop.multiProcessorCount * 16);
    *out = c;
    return DPCS_OK;
}

extern "C" void dpcs_context_destroy(dpcs_context ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->pool) (void)hipFree(kv.second.first);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->ev_shade) (void)hipEventDestroy(ctx->ev_shade);
    if (ctx->ev_shadow) (void)hipEventDestroy(ctx->ev_shadow);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->dstats) (void)hipFree(ctx->dstats);
    delete ctx;
}

extern "C" const char* dpcs_last_error(dpcs_context ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" dpcs_status dpcs_context_synchronize(dpcs_context ctx) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    if (!hip_ok(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize")) return DPCS_E_DEVICE;
    return ctx->sticky ? DPCS_E_DEVICE : DPCS_OK;
}

extern "C" dpcs_status dpcs_context_set_capacity(dpcs_context ctx, int64_t paths) {
    if (!ctx || paths < 1 || paths > (int64_t(1) << 30)) return DPCS_E_INVALID;
    ctx->capacity = paths;
    return DPCS_OK;
}

// ====================================================================== scene

extern "C" dpcs_status dpcs_scene_create(dpcs_context ctx, const dpcs_mesh_desc* m, dpcs_scene* out) {
    if (!ctx || !m || !out) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    *out = nullptr;
    if (ctx->sticky) return DPCS_E_DEVICE;
    (void)hipGetLastError();   // drop errors left by other libraries on this thread
    if (!m->positions || !m->triangles || !m->corner_uvs || m->num_vertices <= 0 || m->num_triangles <= 0)
        return fail(ctx, DPCS_E_INVALID, "mesh needs positions, triangles, corner_uvs and positive counts");
    if (m->num_triangles > (1 << 29)) return fail(ctx, DPCS_E_UNSUPPORTED, "too many triangles");
    if (m->bvh_kind != DPCS_BVH_LBVH && m->bvh_kind != DPCS_BVH_SAH && m->bvh_kind != DPCS_BVH_PLOC)
        return fail(ctx, DPCS_E_INVALID, "bvh_kind must be DPCS_BVH_LBVH, DPCS_BVH_SAH or DPCS_BVH_PLOC");
    const int nt = m->num_triangles, nv = m->num_vertices;
    for (int64_t i = 0; i < 3 * (int64_t)nt; ++i)
        if (m->triangles[i] < 0 || m->triangles[i] >= nv)
            return fail(ctx, DPCS_E_INVALID, "triangle index out of range");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) {
            const double v = m->positions[3 * i + k];
            if (!std::isfinite(v)) return fail(ctx, DPCS_E_INVALID, "non-finite vertex");
            lo[k] = std::min(lo[k], v);
            hi[k] = std::max(hi[k], v);
        }
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    for (int64_t p = 0; p < nt; ++p)
        for (int k = 0; k < 3; ++k) {
            const float c = (m->positions[3 * m->triangles[3 * p] + k] + m->positions[3 * m->triangles[3 * p + 1] + k] +
                             m->positions[3 * m->triangles[3 * p + 2] + k]) *
                            (1.0f / 3.0f);
            clo[k] = std::min(clo[k], (double)c);
            chi[k] = std::max(chi[k], (double)c);
        }
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    auto* sc = new dpcs_scene_s();
    sc->ctx = ctx;
    sc->nt = nt;
    const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
    sc->tmin = (float)(1e-5 * diag);
    for (int k = 0; k < 3; ++k) {
        sc->lo[k] = (float)lo[k];
        sc->hi[k] = (float)hi[k];
    }
    const int ni = std::max(nt - 1, 1);
    const int ntiles = (nt + 1023) / 1024;
    // resident arrays
    bool ok = true;
    auto dmalloc = [&](void** p, size_t b) {
        if (!ok) return;
        if (hipMalloc(p, std::max<size_t>(b, 16)) != hipSuccess) {
            (void)hipGetLastError();
            ok = false;
        }
    };
    dmalloc((void**)&sc->nodes, sizeof(float4) * 4 * ni);
    dmalloc((void**)&sc->tris, sizeof(float4) * 3 * (nt + 1));   // + the dummy leaf of empty BVH4 slots
    dmalloc((void**)&sc->tri_uv, sizeof(float4) * 2 * nt);
    if (m->emission) dmalloc((void**)&sc->emission, sizeof(float4) * nt);
    dmalloc((void**)&sc->leaf_of_prim, sizeof(int) * nt);
    dmalloc((void**)&sc->F, sizeof(int) * 3 * nt);
    dmalloc((void**)&sc->order, sizeof(uint32_t) * nt);
    dmalloc((void**)&sc->child, sizeof(int) * 2 * ni);
    dmalloc((void**)&sc->parent_int, sizeof(int) * ni);
    dmalloc((void**)&sc->parent_leaf, sizeof(int) * nt);
    sc->nv = nv;
    sc->nnodes = ni;
    sc->bytes = (int64_t)sizeof(float4) * (4 * ni + 3 * (nt + 1) + 2 * nt + (m->emission ? nt : 0)) + 4 * nt +
                4 * (3 * (int64_t)nt + nt + 2 * (int64_t)ni + ni + nt);
    // build temporaries: the uploaded vertices, uvs and emission, the sort and bounds
    // buffers carved from one allocation (each part rounded up to 256 bytes), and the
    // clustering / collapse scratch (used one after the other)
    const BvhBuild kind = m->bvh_kind == DPCS_BVH_SAH    ? BvhBuild::SAH
                          : m->bvh_kind == DPCS_BVH_PLOC ? BvhBuild::PLOC
                                                         : BvhBuild::LBVH;
    void *dV = nullptr, *dUV = nullptr, *dLe = nullptr, *tmp = nullptr, *bscr = nullptr;
    dmalloc(&dV, sizeof(float) * 3 * nv);
    dmalloc(&dUV, sizeof(float) * 6 * nt);
    if (m->emission) dmalloc(&dLe, sizeof(float) * 3 * nt);
    auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t tmp_parts[] = {4 * (size_t)nt, 4 * (size_t)nt, 4 * (size_t)nt, 4 * (size_t)nt,
                                4 * 256 * (size_t)ntiles, 4 * (size_t)ni, 24 * (size_t)ni};
    size_t tmp_bytes = 0;
    for (size_t b : tmp_parts) tmp_bytes += r256(b);
    dmalloc(&tmp, tmp_bytes);
    if (nt > 1) {
        const size_t hier = kind == BvhBuild::SAH    ? sah_scratch_bytes(nt)
                            : kind == BvhBuild::PLOC ? ploc_scratch_bytes(nt)
                                                     : 0;
        dmalloc(&bscr, std::max(hier, wide_scratch_bytes(nt)));
    }
    auto cleanup_tmp = [&]() {
        (void)hipStreamSynchronize(ctx->stream);   // no build kernel or copy still reads them
        (void)hipFree(dV);
        (void)hipFree(dUV);
        if (dLe) (void)hipFree(dLe);
        (void)hipFree(tmp);
        if (bscr) (void)hipFree(bscr);
    };
    auto destroy_scene = [&]() {
        (void)hipFree(sc->nodes);
        if (sc->nodes4) (void)hipFree(sc->nodes4);
        (void)hipFree(sc->tris);
        (void)hipFree(sc->tri_uv);
        if (sc->emission) (void)hipFree(sc->emission);
        (void)hipFree(sc->leaf_of_prim);
        for (void* q : {(void*)sc->F, (void*)sc->order, (void*)sc->child, (void*)sc->parent_int, (void*)sc->parent_leaf,
                        (void*)sc->map4})
            if (q) (void)hipFree(q);
        delete sc;
    };
    if (!ok) {
        cleanup_tmp();
        destroy_scene();
        return fail(ctx, DPCS_E_OOM, "device allocation failed while creating the scene");
    }
    BvhInputs in{};
    BvhOutputs bo{};
    char* t = (char*)tmp;
    int part = 0;
    auto take = [&]() {   // next part, in the order of tmp_parts
        char* p = t;
        t += r256(tmp_parts[part++]);
        return (void*)p;
    };
    in.keys[0] = (uint32_t*)take();
    in.keys[1] = (uint32_t*)take();
    in.vals[0] = (uint32_t*)take();
    in.vals[1] = (uint32_t*)take();
    in.hist = (uint32_t*)take();
    in.flags = (int*)take();
    in.node_box = (float*)take();
    in.child = sc->child;
    in.parent_int = sc->parent_int;
    in.parent_leaf = sc->parent_leaf;
    in.V = (const float*)dV;
    in.F = sc->F;
    in.UV = (const float*)dUV;
    in.Le = (const float*)dLe;
    in.nt = nt;
    for (int k = 0; k < 3; ++k) {
        in.lo[k] = (float)clo[k];
        const double ext = chi[k] - clo[k];
        in.scale[k] = ext > 0 ? (float)(1023.0 / ext) : 0.0f;
    }
    bo.nodes = sc->nodes;
    bo.tris = sc->tris;
    bo.tri_uv = sc->tri_uv;
    bo.emission = sc->emission;
    bo.leaf_of_prim = sc->leaf_of_prim;
    hipStream_t st = ctx->stream;
    // the whole build runs on the device: Morton sort, the hierarchy (radix tree, or PLOC
    // clustering for the SAH-quality tree), leaf records, the 4-wide collapse and the
    // tree's checks; the host reads back counts, never the tree
    uint64_t host_words[2] = {0, 0};
    const char* step = "upload";
    hipError_t e = hipMemcpyAsync(dV, m->positions, sizeof(float) * 3 * nv, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sc->F, m->triangles, sizeof(int) * 3 * nt, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dUV, m->corner_uvs, sizeof(float) * 6 * nt, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && m->emission)
        e = hipMemcpyAsync(dLe, m->emission, sizeof(float) * 3 * nt, hipMemcpyHostToDevice, st);
    Launch l{st, ctx->grid_cap};
    if (e == hipSuccess) {
        step = "init";
        launch_zero(l, (float*)in.flags, ni);
        e = hipMemsetAsync(sc->parent_int, 0xff, sizeof(int) * ni, st);   // -1: no parent (root)
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // the clock starts after the uploads
    }
    const auto t0 = std::chrono::steady_clock::now();
    if (e == hipSuccess) {
        step = "build kernels";
        e = build_bvh(st, in, bo, kind, bscr, host_words);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(sc->order, bo.order, sizeof(uint32_t) * nt, hipMemcpyDeviceToDevice, st);
    WideResult wr{};
    if (e == hipSuccess && nt > 1) {
        step = "4-wide collapse";
        // (the SAH build's leaf order lives in the scratch the collapse reuses: read the copy)
        e = build_wide(st, WideArgs{sc->nodes, sc->parent_int, sc->parent_leaf, sc->order, nt}, bscr, host_words, wr);
    }
    if (e == hipSuccess) {
        step = "synchronize";
        e = hipStreamSynchronize(st);
    }
    sc->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (e == hipErrorNotSupported) {   // the SAH build stops at a tree deeper than 64 levels
        (void)hipGetLastError();
        cleanup_tmp();
        destroy_scene();
        return fail(ctx, DPCS_E_UNSUPPORTED, "BVH deeper than 64 levels");
    }
    if (e != hipSuccess) {
        cleanup_tmp();
        hip_ok(ctx, e, (std::string("scene build (") + step + ")").c_str());
        destroy_scene();
        return DPCS_E_DEVICE;
    }
    if (wr.malformed) {
        cleanup_tmp();
        destroy_scene();
        return fail(ctx, DPCS_E_DEVICE, "BVH build produced an invalid tree");
    }
    sc->depth = nt > 1 ? wr.depth : 1;
    if (sc->depth > 64) {
        cleanup_tmp();
        destroy_scene();
        return fail(ctx, DPCS_E_UNSUPPORTED, "BVH deeper than 64 levels");
    }
    // the 4-wide BVH for the traversal kernels, when its worst-case stack fits and its byte
    // size fits the 32-bit node offsets the traversal loads with; else the binary BVH serves
    if (nt > 1 && wr.stack_bound <= MAX_STACK && sizeof(float4) * 8 * (size_t)wr.nnodes4 <= (size_t)UINT32_MAX) {
        // the dummy leaf's triangle: NaN vertices, which no ray hits
        const float qn = std::numeric_limits<float>::quiet_NaN();
        int none = -1;
        float none_f;
        std::memcpy(&none_f, &none, 4);
        const float4 dummy[3] = {make_float4(qn, qn, qn, none_f), make_float4(qn, qn, qn, 0.f),
                                 make_float4(qn, qn, qn, 0.f)};
        const size_t b4 = sizeof(float4) * 8 * (size_t)wr.nnodes4, bm = sizeof(int) * 4 * (size_t)wr.nnodes4;
        hipError_t e4 = hipMemcpy(sc->tris + 3 * (size_t)nt, dummy, sizeof(dummy), hipMemcpyHostToDevice);
        if (e4 == hipSuccess) e4 = hipMalloc((void**)&sc->nodes4, b4);
        if (e4 == hipSuccess) e4 = hipMalloc((void**)&sc->map4, bm);
        if (e4 == hipSuccess) e4 = hipMemcpyAsync(sc->nodes4, wr.nodes4, b4, hipMemcpyDeviceToDevice, st);
        if (e4 == hipSuccess) e4 = hipMemcpyAsync(sc->map4, wr.map4, bm, hipMemcpyDeviceToDevice, st);
        if (e4 == hipSuccess) e4 = hipStreamSynchronize(st);
        if (e4 != hipSuccess) {
            cleanup_tmp();
            hip_ok(ctx, e4, "scene build (4-wide BVH)");
            destroy_scene();
            return DPCS_E_DEVICE;
        }
        sc->nnodes4 = wr.nnodes4;
        sc->bytes += (int64_t)(b4 + bm);
    }
    cleanup_tmp();
    *out = sc;
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_scene_get_info(dpcs_scene s, dpcs_scene_info* out) {
    if (!s || !out) return DPCS_E_INVALID;
    std::memset(out, 0, sizeof *out);
    out->num_triangles = s->nt;
    out->num_nodes = s->nnodes;
    out->wide_nodes = s->nnodes4;
    out->max_depth = s->depth;
    out->device_bytes = s->bytes;
    out->build_ms = s->build_ms;
    for (int k = 0; k < 3; ++k) {
        out->bbox_lo[k] = s->lo[k];
        out->bbox_hi[k] = s->hi[k];
    }
    out->tmin = s->tmin;
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_scene_destroy(dpcs_scene s) {
    if (!s) return DPCS_E_INVALID;
    if (s->refs.load() > 0) return fail(s->ctx, DPCS_E_BUSY, "scene still used by queued server requests");
    dpcs_context ctx = s->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(s->nodes);
    if (s->nodes4) (void)hipFree(s->nodes4);
    (void)hipFree(s->tris);
    (void)hipFree(s->tri_uv);
    if (s->emission) (void)hipFree(s->emission);
    (void)hipFree(s->leaf_of_prim);
    for (void* q : {(void*)s->F, (void*)s->order, (void*)s->child, (void*)s->parent_int, (void*)s->parent_leaf,
                    (void*)s->map4, (void*)s->edges})
        if (q) (void)hipFree(q);
    delete s;
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_scene_refit(dpcs_context ctx, dpcs_scene s, const float* positions) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->sticky) return DPCS_E_DEVICE;
    if (!s || s->ctx != ctx) return fail(ctx, DPCS_E_INVALID, "scene is NULL or from another context");
    if (!positions) return fail(ctx, DPCS_E_INVALID, "positions is NULL");
    if (s->refs.load() > 0) return fail(ctx, DPCS_E_BUSY, "scene still used by queued server requests");
    (void)hipGetLastError();
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    dpcs_status st = DPCS_OK;
    const int ni = s->nnodes;
    int* flags = (int*)scratch(ctx, "refit.flags", sizeof(int) * ni, &st);
    if (!flags) return st;
    float* box = (float*)scratch(ctx, "refit.box", sizeof(float) * 6 * ni, &st);
    if (!box) return st;
    Launch l{ctx->stream, ctx->grid_cap};
    launch_zero(l, (float*)flags, ni);
    RefitArgs a{positions, s->F, s->order, s->child, s->parent_int, s->parent_leaf, flags, box, s->nt,
                s->nodes, s->tris, s->nodes4, s->map4, s->nodes4 ? s->nnodes4 : 0};
    if (!hip_ok(ctx, refit_bvh(ctx->stream, a), "scene refit")) return DPCS_E_DEVICE;
    s->edges_valid = false;   // vertices may have met or parted: the edge table is welded again
    ctx->err.clear();
    return DPCS_OK;
}

// ====================================================================== render
namespace dpcs {

// Per-request resident inputs of a render: E_p after the PRF and the packed maps.
bool prepare_request(dpcs_context ctx, ReqDesc& r, const dpcs_render_params* p, const char* tag, dpcs_status* st) {
    Launch l{ctx->stream, ctx->grid_cap};
    std::string a = std::string(tag) + ".Ep", b = std::string(tag) + ".tex", c = std::string(tag) + ".texb";
    float4* Ep = (float4*)scratch(ctx, a.c_str(), sizeof(float4) * (size_t)r.Wp * r.Hp, st);
    if (!Ep) return false;
    float4* tex = (float4*)scratch(ctx, b.c_str(), sizeof(float4) * (size_t)r.tw * r.th, st);
    if (!tex) return false;
    float4* texb = nullptr;
    if (p->metallic || p->normal_map) {
        texb = (float4*)scratch(ctx, c.c_str(), sizeof(float4) * (size_t)r.tw * r.th, st);
        if (!texb) return false;
    }
    launch_prf(l, r, Ep);
    launch_pack_tex(l, r, p->albedo, p->brdf == DPCS_BRDF_GGX ? p->roughness : nullptr, tex);
    if (texb) launch_pack_tex_b(l, r, p->normal_map, p->brdf == DPCS_BRDF_GGX ? p->metallic : nullptr, texb);
    r.Ep = Ep;
    r.tex4 = tex;
    r.tex4b = texb;
    return true;
}

bool side_stream(dpcs_context ctx) {
    if (ctx->side) return true;
    if (ctx->side_failed) return false;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (s) (void)hipStreamDestroy(s);
        if (a) (void)hipEventDestroy(a);
        ctx->side_failed = true;
        return false;
    }
    ctx->side = s;
    ctx->ev_shade = a;
    ctx->ev_shadow = b;
    return true;
}

int* side_spill(dpcs_context ctx, const Queues& q) {
    dpcs_status st = DPCS_OK;
    int* p = (int*)scratch(ctx, "fwd.spill2", 4 * (size_t)q.trace_blocks * TRACE_TB * SPILL, &st);
    if (!p) ctx->err.clear();   // the forward then runs on one stream
    return p;
}

void forward_wave(dpcs_context ctx, Queues& q, ReqDesc& r, uint32_t a, uint32_t b, bool finalize, int* spill2) {
    Launch l{ctx->stream, ctx->grid_cap};
    const uint32_t n = (b - a) * (uint32_t)r.spp;
    r.g_base = a * (uint32_t)r.spp;
    r.sid_base = 0;
    launch_set_count(l, q.cnt, 0, n, 1, 4);
    // the camera rays are generated by the depth-0 closest-hit and shading kernels (no
    // raygen launch); the stage record keeps the count of camera samples
    int pr = prof_begin(ctx, DPCS_STAGE_RAYGEN);
    prof_end(ctx, pr, nullptr, n);
    int cur = 0;
    // A depth's shadow rays run on the side stream (with their own spill region) while the
    // next depth's closest hit runs here, so each fills the other's tail; shading waits
    // for the previous depth's shadow rays (both add to the samples' radiance), and so
    // does the finalize.  Profiling keeps every launch on this stream.
    const bool side = spill2 && !ctx->prof_mode && (int64_t)n >= SIDE_MIN_PATHS && side_stream(ctx);
    Queues qs = q;
    qs.spill = spill2;
    const Launch ls{ctx->side, ctx->grid_cap};
    for (int d = 0; d < r.max_depth; ++d) {
        // (the closest-hit launch empties the next path queue and this depth's shadow queues)
        q.stats = prof_stats(ctx, DPCS_STAGE_TRACE);
        pr = prof_begin(ctx, DPCS_STAGE_TRACE);
        launch_trace(l, q, cur, r, nullptr, n, d == 0);
        prof_end(ctx, pr, q.cnt + cur, 0);
        if (side && d > 0) (void)hipStreamWaitEvent(ctx->stream, ctx->ev_shadow, 0);
        pr = prof_begin(ctx, DPCS_STAGE_SHADE);
        launch_shade(l, q, cur, d, r, nullptr, n, d == 0);
        prof_end(ctx, pr, q.cnt + cur, 0);
        q.stats = prof_stats(ctx, DPCS_STAGE_SHADOW);
        if (side) {
            (void)hipEventRecord(ctx->ev_shade, ctx->stream);
            (void)hipStreamWaitEvent(ctx->side, ctx->ev_shade, 0);
            for (int w = 0; w < (r.env_on ? 2 : 1); ++w) launch_shadow(ls, qs, w, r, nullptr, n, d);
            (void)hipEventRecord(ctx->ev_shadow, ctx->side);
        } else {
            for (int w = 0; w < (r.env_on ? 2 : 1); ++w) {
                pr = prof_begin(ctx, DPCS_STAGE_SHADOW);
                launch_shadow(l, q, w, r, nullptr, n, d);
                prof_end(ctx, pr, q.cnt + shadow_slot(cur, w), 0);
            }
        }
        q.stats = nullptr;
        cur ^= 1;
    }
    if (side) (void)hipStreamWaitEvent(ctx->stream, ctx->ev_shadow, 0);
    if (finalize) {
        pr = prof_begin(ctx, DPCS_STAGE_FINALIZE);
        launch_finalize(l, q, r, nullptr, 0, a, b);
        prof_end(ctx, pr, nullptr, b - a);
    }
}

void adjoint_wave(dpcs_context ctx, Queues& q, const AdjQueues& aq, ReqDesc& r, uint32_t a, uint32_t b,
                  const float* sample_L, float4* pix_dE, int* spill2) {
    Launch l{ctx->stream, ctx->grid_cap};
    const uint32_t n = (b - a) * (uint32_t)r.spp;
    r.g_base = a * (uint32_t)r.spp;
    r.sid_base = 0;
    int pr = prof_begin(ctx, DPCS_STAGE_ADJ_PIXEL);
    launch_adj_pixel(l, q, aq, r, a, b, sample_L, pix_dE);
    launch_cam_grad(l, q, aq, r, a, b);   // (no-op unless the camera-pose gradient is asked for)
    prof_end(ctx, pr, nullptr, b - a);
    int cur = 0;
    if (r.rec) {   // the forward's path records stand in for tracing (camera rays regenerated in depth 0)
        // (the replay's queue sizes rotate over their own slots: one reset for all depths)
        launch_set_count(l, q.cnt, REPLAY_CNT, n, REPLAY_CNT + 1, REPLAY_CNT + 2);
        for (int d = 0; d < r.max_depth; ++d) {
            pr = prof_begin(ctx, DPCS_STAGE_ADJ_SHADE);
            launch_adj_replay(l, q, aq, cur, d, r, nullptr, n);
            prof_end(ctx, pr, q.cnt + REPLAY_CNT + d % 3, 0);
            if ((aq.tb.rec || aq.eb.rec) && ((d + 1) % BIN_DEPTHS == 0 || d == r.max_depth - 1)) {
                pr = prof_begin(ctx, DPCS_STAGE_OTHER);
                launch_map_flush(l, aq, r);
                prof_end(ctx, pr, nullptr, 0);
            }
            cur ^= 1;
        }
        return;
    }
    launch_set_count(l, q.cnt, 0, n, 1, 4);
    launch_adj_raygen(l, q, aq, r, 0, r.g_base, n);
    // as in the forward: a depth's shadow rays on the side stream beside the next depth's
    // closest hit; the adjoint shading and the map flush (which read what they write:
    // the next paths' remaining radiance, map records) wait for them
    const bool side = spill2 && !ctx->prof_mode && (int64_t)n >= SIDE_MIN_PATHS && side_stream(ctx);
    Queues qs = q;
    qs.spill = spill2;
    const Launch ls{ctx->side, ctx->grid_cap};
    for (int d = 0; d < r.max_depth; ++d) {   // (the closest-hit launch empties the next queues)
        q.stats = prof_stats(ctx, DPCS_STAGE_TRACE);
        pr = prof_begin(ctx, DPCS_STAGE_TRACE);
        launch_trace(l, q, cur, r, nullptr, n);
        prof_end(ctx, pr, q.cnt + cur, 0);
        if (side && d > 0) (void)hipStreamWaitEvent(ctx->stream, ctx->ev_shadow, 0);
        pr = prof_begin(ctx, DPCS_STAGE_ADJ_SHADE);
        launch_adj_shade(l, q, aq, cur, d, r, nullptr, n);
        prof_end(ctx, pr, q.cnt + cur, 0);
        q.stats = prof_stats(ctx, DPCS_STAGE_ADJ_SHADOW);
        if (side) {
            (void)hipEventRecord(ctx->ev_shade, ctx->stream);
            (void)hipStreamWaitEvent(ctx->side, ctx->ev_shade, 0);
            for (int w = 0; w < (r.env_on ? 2 : 1); ++w) launch_adj_shadow(ls, qs, aq, w, cur ^ 1, r, nullptr, n);
            (void)hipEventRecord(ctx->ev_shadow, ctx->side);
        } else {
            for (int w = 0; w < (r.env_on ? 2 : 1); ++w) {
                pr = prof_begin(ctx, DPCS_STAGE_ADJ_SHADOW);
                launch_adj_shadow(l, q, aq, w, cur ^ 1, r, nullptr, n);
                prof_end(ctx, pr, q.cnt + shadow_slot(cur, w), 0);
            }
        }
        q.stats = nullptr;
        if ((aq.tb.rec || aq.eb.rec) && ((d + 1) % BIN_DEPTHS == 0 || d == r.max_depth - 1)) {
            if (side) (void)hipStreamWaitEvent(ctx->stream, ctx->ev_shadow, 0);
            pr = prof_begin(ctx, DPCS_STAGE_OTHER);
            launch_map_flush(l, aq, r);
            prof_end(ctx, pr, nullptr, 0);
        }
        cur ^= 1;
    }
    if (side) (void)hipStreamWaitEvent(ctx->stream, ctx->ev_shadow, 0);
}

}  // namespace dpcs

// The forward render (Eq. 7) in launch waves of whole pixels.  noalloc: the PRF'd
// projector image, the packed maps and the wave's queues are carved from this device's
// copy of noalloc_scratch instead of the context's pool, and the wave shrinks to fit.
static dpcs_status render_impl(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                               const float* proj_image, float* out_image, const dpcs_render_aux* aux, bool noalloc) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->sticky) return DPCS_E_DEVICE;
    if (!scene || scene->ctx != ctx) return fail(ctx, DPCS_E_INVALID, "scene is NULL or from another context");
    if (!out_image) return fail(ctx, DPCS_E_INVALID, "out_image is NULL");
    (void)hipGetLastError();
    ReqDesc r;
    std::string why;
    if (!fill_desc(ctx, r, params, scene, proj_image, &why)) return fail(ctx, DPCS_E_INVALID, why);
    r.out_image = out_image;
    if (aux) {
        r.out_linear = aux->linear;
        r.out_L = aux->sample_radiance;
        r.out_hits = aux->hit_prims;
        r.rec = aux->path_records;
        r.rec_g0 = 0;
    }
    if (r.rec && scene->nt >= (int)REC_LEAF) return fail(ctx, DPCS_E_UNSUPPORTED, "path records need < 2^30 triangles");
    const int64_t npix = (int64_t)r.Wc * r.Hc;
    int64_t cap = std::min<int64_t>(std::max<int64_t>(ctx->capacity, r.spp), npix * r.spp);
    Queues q;
    float4 *na_Ep = nullptr, *na_tex = nullptr, *na_texb = nullptr;
    if (noalloc) {
        if (!ctx->noalloc)
            return fail(ctx, DPCS_E_DEVICE, std::string("no-alloc scratch of this device unavailable: ") +
                                                hipGetErrorString((hipError_t)ctx->noalloc_err));
        const size_t ep_b = (sizeof(float4) * (size_t)r.Wp * r.Hp + 255) & ~size_t(255);
        const bool ext = params->metallic || params->normal_map;
        const size_t tex1 = (sizeof(float4) * (size_t)r.tw * r.th + 255) & ~size_t(255);
        const size_t tex_b = ext ? 2 * tex1 : tex1;
        // every path takes its queue entries and a traversal thread's spill space
        const size_t per_path = queue_bytes(1, 0) - 32 * 256 + 4 * (size_t)SPILL;
        const size_t fixed = 32 * 256 + 4 * (size_t)TRACE_TB * SPILL;
        if (ep_b + tex_b + fixed + per_path * (size_t)r.spp > NOALLOC_BYTES)
            return fail(ctx, DPCS_E_INVALID, "dpcs_render_noalloc: projector image, maps and one pixel's samples exceed "
                                             "the " + std::to_string(NOALLOC_BYTES >> 20) + " MiB no-alloc scratch");
        cap = std::min<int64_t>(cap, (int64_t)((NOALLOC_BYTES - ep_b - tex_b - fixed) / per_path));
        cap = std::max<int64_t>(r.spp, cap / r.spp * r.spp);
        const int tb = (int)((cap + TRACE_TB - 1) / TRACE_TB);
        char* base = (char*)ctx->noalloc;
        na_Ep = (float4*)base;
        na_tex = (float4*)(base + ep_b);
        na_texb = ext ? (float4*)(base + ep_b + tex1) : nullptr;
        r.Ep = na_Ep;
        r.tex4 = na_tex;
        r.tex4b = na_texb;
        if (ep_b + tex_b + queue_bytes(cap, tb) > NOALLOC_BYTES)
            return fail(ctx, DPCS_E_INVALID, "dpcs_render_noalloc: internal sizing error");
        carve_queues(base + ep_b + tex_b, cap, tb, q);
    }
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    dpcs_status st = DPCS_OK;
    const int prof_mode = ctx->prof_mode;
    if (noalloc) {
        Launch l{ctx->stream, ctx->grid_cap};
        launch_prf(l, r, na_Ep);
        launch_pack_tex(l, r, params->albedo, params->brdf == DPCS_BRDF_GGX ? params->roughness : nullptr, na_tex);
        if (na_texb)
            launch_pack_tex_b(l, r, params->normal_map, params->brdf == DPCS_BRDF_GGX ? params->metallic : nullptr,
                              na_texb);
        ctx->prof_mode = 0;   // profiling records events and pinned counts; not on this path
    } else {
        if (!prepare_request(ctx, r, params, "fwd", &st)) return st;
        if (!make_queues(ctx, "fwd.queues", cap, q, &st)) return st;
    }
    const int64_t ppw = std::max<int64_t>(1, cap / r.spp);   // whole pixels per wave
    int* spill2 = noalloc ? nullptr : side_spill(ctx, q);     // (the no-alloc path stays on one stream)
    for (int64_t a = 0; a < npix; a += ppw)
        forward_wave(ctx, q, r, (uint32_t)a, (uint32_t)std::min(npix, a + ppw), true, spill2);
    ctx->prof_mode = prof_mode;
    if (!hip_ok(ctx, hipGetLastError(), "kernel launch")) return DPCS_E_DEVICE;
    ctx->err.clear();
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_render(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                                   const float* proj_image, float* out_image, const dpcs_render_aux* aux) {
    return render_impl(ctx, scene, params, proj_image, out_image, aux, false);
}

extern "C" dpcs_status dpcs_render_noalloc(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                                           const float* proj_image, float* out_image, const dpcs_render_aux* aux) {
    return render_impl(ctx, scene, params, proj_image, out_image, aux, true);
}

extern "C" dpcs_status dpcs_render_gbuffer(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                                           float* gbuffer) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->sticky) return DPCS_E_DEVICE;
    if (!scene || scene->ctx != ctx) return fail(ctx, DPCS_E_INVALID, "scene is NULL or from another context");
    if (!gbuffer) return fail(ctx, DPCS_E_INVALID, "gbuffer is NULL");
    if (reinterpret_cast<uintptr_t>(gbuffer) % 16) return fail(ctx, DPCS_E_INVALID, "gbuffer must be 16-byte aligned");
    (void)hipGetLastError();
    ReqDesc r;
    std::string why;
    if (!fill_desc(ctx, r, params, scene, nullptr, &why, false)) return fail(ctx, DPCS_E_INVALID, why);
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    dpcs_status st = DPCS_OK;
    float4* tex = (float4*)scratch(ctx, "gbuf.tex", sizeof(float4) * (size_t)r.tw * r.th, &st);
    if (!tex) return st;
    Launch l{ctx->stream, ctx->grid_cap};
    launch_pack_tex(l, r, params->albedo, nullptr, tex);
    r.tex4 = tex;
    launch_gbuffer(l, r, gbuffer);
    if (!hip_ok(ctx, hipGetLastError(), "render_gbuffer")) return DPCS_E_DEVICE;
    ctx->err.clear();
    return DPCS_OK;
}

// ====================================================================== debug
extern "C" dpcs_status dpcs_debug_intersect(dpcs_context ctx, dpcs_scene scene, const float* rays, int64_t n,
                                            int32_t use_bvh, int32_t* prim, float* t, float* b1, float* b2) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->sticky) return DPCS_E_DEVICE;
    if (!scene || !rays || !prim || n < 0) return fail(ctx, DPCS_E_INVALID, "bad debug_intersect arguments");
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    (void)hipGetLastError();
    Launch l{ctx->stream, ctx->grid_cap};
    if (use_bvh < 0 || use_bvh > 4) return fail(ctx, DPCS_E_INVALID, "debug_intersect mode must be in 0..4");
    launch_debug_intersect(l, scene->nodes4, scene->nodes, scene->tris, scene->leaf_of_prim, scene->nt, scene->tmin,
                           rays, n, use_bvh, prim, t, b1, b2);
    return hip_ok(ctx, hipGetLastError(), "debug_intersect") ? DPCS_OK : DPCS_E_DEVICE;
}

extern "C" dpcs_status dpcs_debug_philox(dpcs_context ctx, uint64_t seed, const uint32_t* ctr, int64_t n,
                                         uint32_t* out) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!ctr || !out || n < 0) return fail(ctx, DPCS_E_INVALID, "bad debug_philox arguments");
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    (void)hipGetLastError();
    Launch l{ctx->stream, ctx->grid_cap};
    launch_debug_philox(l, seed, ctr, n, out);
    return hip_ok(ctx, hipGetLastError(), "debug_philox") ? DPCS_OK : DPCS_E_DEVICE;
}

extern "C" dpcs_status dpcs_debug_brdf(dpcs_context ctx, int32_t brdf, const double* in, int64_t n, double* out) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (n < 0 || (n > 0 && (!in || !out)) || (brdf != DPCS_BRDF_LAMBERT && brdf != DPCS_BRDF_GGX))
        return fail(ctx, DPCS_E_INVALID, "bad debug_brdf arguments");
    if (n > (int64_t(1) << 31)) return fail(ctx, DPCS_E_INVALID, "debug_brdf: too many rows");
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    (void)hipGetLastError();
    Launch l{ctx->stream, ctx->grid_cap};
    launch_debug_brdf(l, brdf, in, n, out);
    return hip_ok(ctx, hipGetLastError(), "debug_brdf") ? DPCS_OK : DPCS_E_DEVICE;
}

// ====================================================================== profiling
extern "C" dpcs_status dpcs_context_set_profiling(dpcs_context ctx, int32_t mode) {
    if (!ctx || mode < 0 || mode > 2) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    (void)hipStreamSynchronize(ctx->stream);
    ctx->prof.clear();
    ctx->ev_used = 0;
    ctx->pinned_used = 0;
    if (mode && !ctx->pinned) {
        ctx->pinned_cap = 1 << 16;
        if (hipHostMalloc((void**)&ctx->pinned, sizeof(uint32_t) * ctx->pinned_cap) != hipSuccess) {
            (void)hipGetLastError();
            ctx->pinned = nullptr;
            ctx->pinned_cap = 0;
        }
    }
    if (mode >= 2 && !ctx->dstats) {
        if (hipMalloc((void**)&ctx->dstats, sizeof(unsigned long long) * 2 * DPCS_NUM_STAGES) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, DPCS_E_OOM, "profiling counters");
        }
    }
    if (ctx->dstats) (void)hipMemset(ctx->dstats, 0, sizeof(unsigned long long) * 2 * DPCS_NUM_STAGES);
    ctx->prof_mode = mode;
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_context_get_profile(dpcs_context ctx, dpcs_profile* out) {
    if (!ctx || !out) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    if (!hip_ok(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize")) return DPCS_E_DEVICE;
    std::memset(out, 0, sizeof *out);
    for (const auto& r : ctx->prof) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        out->launches[r.stage] += 1;
        out->ms[r.stage] += ms;
        out->items[r.stage] += r.slot >= 0 ? (int64_t)ctx->pinned[r.slot] : r.host_count;
    }
    if (ctx->dstats) {
        unsigned long long h[2 * DPCS_NUM_STAGES];
        (void)hipMemcpy(h, ctx->dstats, sizeof h, hipMemcpyDeviceToHost);
        for (int k = 0; k < DPCS_NUM_STAGES; ++k) {
            out->nodes[k] = (int64_t)h[2 * k];
            out->tris[k] = (int64_t)h[2 * k + 1];
        }
        (void)hipMemset(ctx->dstats, 0, sizeof h);
    }
    ctx->prof.clear();
    ctx->ev_used = 0;
    ctx->pinned_used = 0;
    return DPCS_OK;
}
