// runtime.hpp -- host-side state behind the C ABI (context, scratch pool, scenes).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dpcs.h"
#include "kernels.hpp"

struct dpcs_context_s {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t scratch_limit = 0;
    size_t scratch_bytes = 0;
    int64_t capacity = int64_t(1) << 22;   // paths per launch wave
    std::string err;
    bool sticky = false;
    std::map<std::string, std::pair<void*, size_t>> pool;
    std::recursive_mutex mu;               // serialises calls from several host threads
    int grid_cap = 4096;
    // profiling (dpcs_context_set_profiling)
    struct ProfRec {
        int stage;
        hipEvent_t a, b;
        int slot;            // pinned count slot, -1: host count below
        int64_t host_count;
    };
    int prof_mode = 0;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    uint32_t* pinned = nullptr;            // queue-size snapshots
    int pinned_cap = 0, pinned_used = 0;
    unsigned long long* dstats = nullptr;  // device [DPCS_NUM_STAGES][2]
    void* noalloc = nullptr;               // this device's copy of the no-alloc scratch array
    int noalloc_err = 0;                   // hipError_t of its address lookup
    // second stream (default priority) for a depth's shadow rays beside the next depth's
    // closest hit, and the two events that order them (made on first use)
    hipStream_t side = nullptr;
    hipEvent_t ev_shade = nullptr, ev_shadow = nullptr;
    bool side_failed = false;
};

struct dpcs_scene_s {
    dpcs_context ctx = nullptr;
    float4* nodes = nullptr;
    float4* nodes4 = nullptr;              // 4-wide BVH, or null
    float4* tris = nullptr;
    float4* tri_uv = nullptr;
    float4* emission = nullptr;
    int* leaf_of_prim = nullptr;
    // topology kept for dpcs_scene_refit: triangles, leaf order, binary children and
    // parents, and the binary node (>= 0) or leaf (~l) behind every 4-wide child slot
    int* F = nullptr;
    uint32_t* order = nullptr;
    int* child = nullptr;
    int* parent_int = nullptr;
    int* parent_leaf = nullptr;
    int* map4 = nullptr;
    int nv = 0;
    int nt = 0, nnodes = 0, nnodes4 = 0, depth = 0;
    float tmin = 0.0f;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int64_t bytes = 0;
    double build_ms = 0.0;
    // edge table of the camera-pose gradient's boundary part (built on first use, again
    // after a refit): per welded edge (leaf0, leaf1, corners, faces)
    int4* edges = nullptr;
    int64_t n_edges = 0;
    bool edges_valid = false;
    std::atomic<int> refs{0};              // requests of a server that still use the scene
};

namespace dpcs {

// sets ctx->err and returns s
dpcs_status fail(dpcs_context ctx, dpcs_status s, const std::string& msg);
// checks a HIP status; on error marks the context sticky-failed
bool hip_ok(dpcs_context ctx, hipError_t e, const char* what);
// named scratch buffer of at least `bytes` (grows; never shrinks)
void* scratch(dpcs_context ctx, const char* name, size_t bytes, dpcs_status* st);
// fills a request descriptor from validated params; false + message on invalid input
// (need_proj false: the projector image is not read and may be NULL)
bool fill_desc(dpcs_context ctx, ReqDesc& r, const dpcs_render_params* p, dpcs_scene sc, const float* proj_image,
               std::string* why, bool need_proj = true);

// profiling hooks around one stage launch (no-ops when profiling is off)
int prof_begin(dpcs_context ctx, int stage);
void prof_end(dpcs_context ctx, int rec, const uint32_t* dev_count, int64_t host_count);
unsigned long long* prof_stats(dpcs_context ctx, int stage);

// path queues for `cap` paths carved from one scratch buffer (prefix selects the buffer)
bool make_queues(dpcs_context ctx, const char* name, int64_t cap, Queues& q, dpcs_status* st);
// bytes of the queues of `cap` paths with a traversal grid capped at trace_blocks
// workgroups, and their layout from base (256-byte aligned)
size_t queue_bytes(int64_t cap, int trace_blocks);
void carve_queues(char* base, int64_t cap, int trace_blocks, Queues& q);
// ext: also the pending buffers of the metallic / normal-map replay
bool make_adj_queues(dpcs_context ctx, const char* name, int64_t cap, AdjQueues& aq, dpcs_status* st,
                     bool ext = false);
void make_map_bins(dpcs_context ctx, ZeroList& zl, MapBins& mb, const char* name, int W, int H, int C, int RS,
                   int64_t cap);

// PRF'd projector irradiance and packed maps of one request in scratch (tag selects the buffers)
bool prepare_request(dpcs_context ctx, ReqDesc& r, const dpcs_render_params* p, const char* tag, dpcs_status* st);
// one launch wave of the forward path over pixels [a, b) (whole pixels); per-sample
// radiance lands in q.L; finalize writes the request's outputs
// spill2: a second traversal spill region like q.spill (null: every launch on the
// context's stream, one after the other)
void forward_wave(dpcs_context ctx, Queues& q, ReqDesc& r, uint32_t a, uint32_t b, bool finalize,
                  int* spill2 = nullptr);
// the second spill region of forward_wave for q (null when unavailable: then the
// forward runs on one stream)
int* side_spill(dpcs_context ctx, const Queues& q);
// the context's side stream and its two events, made on first use (false: run on one stream)
bool side_stream(dpcs_context ctx);
// one launch wave of the path-replay adjoint over pixels [a, b) (q.L holds the samples
// unless sample_L is given)
void adjoint_wave(dpcs_context ctx, Queues& q, const AdjQueues& aq, ReqDesc& r, uint32_t a, uint32_t b,
                  const float* sample_L, float4* pix_dE = nullptr, int* spill2 = nullptr);
// the boundary part of the camera-pose gradient at the images of mesh edges, added into
// dst[0..11] (R row-major, t); pix_dE: per-pixel cotangent of the clipped pixel means;
// K the camera intrinsics; q's paths are reused (at most q.cap / 2 edge points per wave)
dpcs_status camera_edge_term(dpcs_context ctx, dpcs_scene sc, const ReqDesc& r, const Queues& q, double density,
                             const double K[9], const float4* pix_dE, float* dst);

}  // namespace dpcs
