// kernels.hpp -- host-side entry points of the device kernels (one process, one device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace dpcs {

// ------------------------------------------------------------------ BVH build
struct BvhInputs {
    const float* V;          // device vertices
    const int* F;            // device triangles
    const float* UV;         // device corner uvs
    const float* Le;         // device emission or null
    int nt;
    float lo[3], scale[3];   // centroid box origin and 1023 / extent
    uint32_t* keys[2];
    uint32_t* vals[2];
    uint32_t* hist;          // 256 * ntiles
    int* child;              // 2 * (nt - 1)
    int* parent_int;         // nt - 1
    int* parent_leaf;        // nt
    int* flags;              // nt - 1, zeroed
    float* node_box;         // 6 * (nt - 1)
};
struct BvhOutputs {
    float4* nodes;           // 4 * max(nt - 1, 1)
    float4* tris;            // 3 * nt
    float4* tri_uv;          // 2 * nt
    float4* emission;        // nt or null
    int* leaf_of_prim;       // nt
    const uint32_t* order;   // leaf -> original triangle (points into keys/vals scratch)
};
// The binary hierarchy with its bounds, then the leaf records.  LBVH: the radix tree over
// the Morton-sorted codes; PLOC: clustering over the Morton order (scratch of
// ploc_scratch_bytes); SAH: top-down binned SAH (scratch of sah_scratch_bytes).  PLOC and
// SAH read one count per round into host_word[0..1].  child / parent_int / parent_leaf
// receive the topology (parent_int must hold -1 everywhere beforehand); out.order points
// into in.vals (LBVH, PLOC) or into the scratch (SAH).  SAH returns hipErrorNotSupported
// for a tree deeper than 64 levels.
enum class BvhBuild { LBVH, PLOC, SAH };
hipError_t build_bvh(hipStream_t st, const BvhInputs& in, BvhOutputs& out, BvhBuild kind = BvhBuild::LBVH,
                     void* scratch = nullptr, uint64_t* host_word = nullptr);
size_t ploc_scratch_bytes(int nt);
hipError_t build_ploc(hipStream_t st, const BvhInputs& in, const uint32_t* order, void* scratch, uint64_t* host_word,
                      float4* nodes);
size_t sah_scratch_bytes(int nt);
hipError_t build_sah(hipStream_t st, const BvhInputs& in, void* scratch, uint64_t* host_word, float4* nodes,
                     const uint32_t** order_out);
// the 4-wide BVH of a binary one (nt >= 2) and the tree's checks, in scratch of
// wide_scratch_bytes(nt): result nodes4 (8 float4 per node) and map4 (4 ints per node)
// point into the scratch; the host reads one count per level into host_words (>= 2)
struct WideArgs {
    const float4* nodes;
    const int* parent_int;
    const int* parent_leaf;
    const uint32_t* order;
    int nt;
};
struct WideResult {
    float4* nodes4;
    int* map4;
    int nnodes4, depth4;   // 4-wide nodes and levels
    int stack_bound;       // most stack entries a traversal holds
    int depth;             // binary depth (internal nodes on the longest root-to-leaf path)
    bool malformed;        // a leaf reached other than once, a parent chain off the root, or
                           // a leaf order that is not a permutation
};
size_t wide_scratch_bytes(int nt);
hipError_t build_wide(hipStream_t st, const WideArgs& a, void* scratch, uint64_t* host_words, WideResult& res);
// leaf-ordered triangle / UV / emission records for a leaf order built elsewhere
hipError_t build_leaf_records(hipStream_t st, const BvhInputs& in, const uint32_t* order, BvhOutputs& out);
// new vertex positions on a fixed topology: the binary node boxes bottom-up (flags: ni
// zeroed ints, node_box: 6 ni floats of scratch), the leaf records' vertices, and the
// 4-wide nodes' child boxes from map4 (4 per node: binary node, ~leaf, or INT_MIN empty)
struct RefitArgs {
    const float* V;
    const int* F;
    const uint32_t* order;
    const int* child;
    const int* parent_int;
    const int* parent_leaf;
    int* flags;
    float* node_box;
    int nt;
    float4* nodes;
    float4* tris;
    float4* nodes4;
    const int* map4;
    int nnodes4;
};
hipError_t refit_bvh(hipStream_t st, const RefitArgs& a);

// ------------------------------------------------------------------ path queues
// Structure-of-arrays queues in HBM.  Path state is FP64 position/direction (PathO,
// PathD, 32 B each) plus FP32 throughput; shadow rays only need a visibility
// decision and are FP32 (16-byte float4 fields: a wave64 touches 1 KiB per field).
struct Queues {
    PathO* po[2];      // path ray origin, slot, triangle left
    PathD* pd[2];      // path ray direction, global sample index g
    float4* pb[2];     // path throughput beta (rgb, -)
    int* hit;          // leaf-order triangle hit by the current queue (-1: escaped)
    float4* so[2];     // shadow ray origin (w: slot); [0] projector, [1] environment
    float4* sd[2];     // shadow direction (w: triangle the ray leaves)
    float4* sc[2];     // shadow contribution (w: batch sample index)
    float* st[2];      // shadow tmax
    float4* L;         // per batch sample radiance (rgb, -)
    uint32_t* cnt;     // [0], [1] path queue sizes, [4..6] the replay's path queue sizes (by
                       // depth mod 3), [8..11] shadow queue sizes (shadow_slot)
    int64_t cap;       // path capacity
    unsigned long long* stats;   // null, or [0] nodes visited, [1] triangles tested (profiling)
    int* spill;        // traversal stack overflow: SPILL ints per thread of a capped grid
    int trace_blocks;  // workgroups the spill region covers: the traversal grid cap
};

constexpr int SHORT_STACK = 8;                 // LDS stack entries per thread
constexpr int SPILL = 64 - SHORT_STACK;        // overflow entries per thread
constexpr int TRACE_TB = 128;                  // threads per workgroup of the traversal kernels
// traversal kernels are compiled for 8 waves per SIMD (at most 64 VGPRs): the loop is
// latency-bound enough that occupancy pays more than the odd spilled register costs
#define TRAVERSAL_OCCUPANCY __attribute__((amdgpu_waves_per_eu(8, 8)))
// except the forward's shadow rays: with the staged tree top their any-hit loop spills a
// few registers at 64 VGPRs; at 7 waves (71 VGPRs, no spill) they run ~3 % faster
#define SHADOW_OCCUPANCY __attribute__((amdgpu_waves_per_eu(7, 7)))
// and the re-tracing replay's shadow rays, whose gradient bookkeeping after the query
// spilled ~150 bytes per lane at 64 VGPRs: at 4 waves (105 VGPRs) nothing spills and
// the re-tracing step is ~1.5 % faster
#define ADJ_SHADOW_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4, 4)))
// Traversal grids are capped at `rounds` x grid_cap x 128 threads (grid_cap x 128 threads
// is one resident round at 8 waves per SIMD); the spill region holds SPILL ints for every
// thread of that grid.  Several rounds let workgroups that finish early be replaced
// while others still trace long paths (4 rounds: traversal -7 %), at 224 B of spill
// space per thread (never more threads than paths of a wave in the request loop, whose
// queues count against its memory budget).
constexpr int TRACE_ROUNDS = 4;
inline int trace_grid_cap(int grid_cap, int rounds) {
    const int g = grid_cap * 128 / TRACE_TB * rounds;
    return g > 0 ? g : 1;
}
inline size_t spill_ints(int grid_cap, int rounds) { return (size_t)trace_grid_cap(grid_cap, rounds) * TRACE_TB * SPILL; }

// Binned accumulation of the cotangent of one texel map (BRDF maps or E_p): the replay
// writes one record per (vertex, map) -- bilinear base texel and offsets plus the C
// cotangent values -- instead of 4 x C global atomics; a flush groups the records by
// T x T texel tile (counting sort), accumulates every tile in LDS and adds the tiles
// into the map with plain stores.
constexpr int MAP_MAX_BINS = 4096;
constexpr int MAP_MAX_T = 16;   // tile side 8 or 16: maps up to 1024 x 1024 are binned
constexpr int BIN_DEPTHS = 4;   // replay depths between flushes (record capacity follows)
constexpr int ACC_CHUNK = 4096; // records per workgroup of the accumulation; the stage holds
                                // ceil(cap / ACC_CHUNK) + nb blocks of (T + 1)^2 x C floats
constexpr int ACC_TB = 1024;    // threads per workgroup of the accumulation
constexpr int BIN_CHUNK = 16384;// records per workgroup of the histogram and the placement
constexpr int BIN_TB = 1024;    // their threads per workgroup: 16 waves share one LDS
                                // histogram, so the few chunks of a flush still fill the chip
constexpr int BIN_U = 4;        // records a thread of the placement loads at once
static_assert(BIN_CHUNK % (BIN_TB * BIN_U) == 0, "placement chunking");
constexpr long long STAGE_NAN = -0x7fffffffffffffffll - 1;   // INT64_MIN
struct MapBins {
    float* rec;          // records of rs floats (null: binning off, the replay scatters directly)
    float* sorted;       // the same records grouped by tile
    long long* stage;    // per (chunk, tile) pair (T + 1)^2 x C exact fixed-point sums (tile plus one
                         // halo row/column); STAGE_NAN marks a chunk with a non-finite value
    uint32_t* count;     // records appended since the last flush (may exceed cap)
    uint32_t* bins;      // counts[nb], offsets[nb + 1], fixed-point exponent E, (unused)[nb - 1],
                         // largest |value| (float bits)
    uint32_t* rowbase;   // per (BIN_CHUNK chunk, tile): where the chunk's records start in the tile
    int64_t cap;         // record capacity
    int W, H, T, nbx, nby, nb;
};

// adjoint additions (see adjoint.hip)
struct alignas(16) PendX {   // per channel c: albedo, roughness, specular, metallic, normal map (xyz)
    float a[3], r[3], s[3], m[3], n[9], pad[3];
};
struct AdjQueues {
    float4* rl[2];     // remaining radiance L_r of the path (rgb, -), follows the path queue
    float4* delta;     // per batch sample cotangent of its radiance (rgb, -)
    double2* sproj[2]; // shadow: projector pixel position (pu, pv) of the vertex
    double2* suv[2];   // shadow: texture coordinate (u, v) of the vertex (FP64: 1k+ maps)
    float4* sg[2];     // shadow: E_p cotangent weight per channel (w: -)
    float4* sa[2];     // shadow: albedo cotangent rgb (w: roughness cotangent)
    float* ss[2];      // shadow: specular cotangent
    float4* pn[2];     // replay: pending next-event cotangents of the previous vertex (albedo rgb, roughness)
    float* pns[2];     // replay: pending next-event specular cotangent
    double2* puv[2];   // pending bounce: texture coordinate (u, v) of the previous vertex
    float2* pend[2];   // pending bounce: (dr, dsp) cotangent scale of the previous vertex
    float4* penda[2];  // pending bounce: albedo cotangent scale rgb
    // with the metallic and normal maps (replay only): the pending bounce's derivative
    // coefficients (d(f_c c)/d theta) / (f_c c) for albedo, roughness, specular, metallic
    // and the normal map's stored values (21 floats, PendX) and the pending next-event
    // cotangents of metallic and the normal map (float4)
    struct PendX* px[2];
    float4* pnx[2];
    MapBins tb;        // BRDF-map cotangent records (C = 5, 8 floats per record; C = 9, 12 floats
                       // with the metallic and normal maps)
    MapBins eb;        // E_p cotangent records (C = 3, 6 floats per record)
};

constexpr int REPLAY_CNT = 4;   // first of the replay's three queue-size slots in Queues::cnt
// The shadow queues' sizes alternate by depth parity: shading at depth d appends to
// q.cnt[shadow_slot(d & 1, which)] (every depth loop starts with cur = 0, so d & 1 = cur),
// so the closest-hit launch of depth d + 1, which empties the slots shading at d + 1
// appends to, leaves intact the sizes that depth d's shadow launch reads (the two may
// run at the same time on two streams).
constexpr int SHADOW_CNT = 8;
// Launch waves of fewer paths keep their shadow rays on the main stream: their launches
// take a few microseconds, less than the two cross-stream waits per depth cost.
constexpr int64_t SIDE_MIN_PATHS = int64_t(1) << 17;
constexpr int64_t LOOP_SIDE_MIN_PATHS = int64_t(1) << 21;   // the same for the request loop's waves
__host__ __device__ constexpr int shadow_slot(int parity, int which) { return SHADOW_CNT + 2 * parity + which; }
struct Launch {
    hipStream_t st;
    int grid_cap;      // upper bound on workgroups of grid-stride kernels
};

// forward kernels; `uni` is the request descriptor when every path of the launch
// belongs to one request (table == null), else descriptors are read from `table`.
void launch_prf(const Launch& l, const ReqDesc& r, float4* Ep);
void launch_pack_tex(const Launch& l, const ReqDesc& r, const float* albedo, const float* rough, float4* tex4);
void launch_pack_tex_b(const Launch& l, const ReqDesc& r, const float* nmap, const float* metal, float4* tex4b);
void launch_set_count(const Launch& l, uint32_t* cnt, int idx, uint32_t value, int zero_from, int zero_to);
void launch_raygen(const Launch& l, const Queues& q, const ReqDesc& r, const ReqDesc* table, int slot,
                   uint32_t g0, uint32_t n, bool adjoint, const AdjQueues* aq);
// cam (one request, no table): the queue is the request's camera rays, generated by the
// closest-hit and shading kernels themselves (no raygen launch, no path state read)
void launch_trace(const Launch& l, const Queues& q, int cur, const ReqDesc& uni, const ReqDesc* table,
                  int64_t n_upper, bool cam = false);
void launch_shade(const Launch& l, const Queues& q, int cur, int depth, const ReqDesc& uni, const ReqDesc* table,
                  int64_t n_upper, bool cam = false);
// depth: the bounce the shadow rays leave from (for the path records); one_tree (with a
// table): every ray is on the tree of `uni` (several requests of one scene)
void launch_shadow(const Launch& l, const Queues& q, int which, const ReqDesc& uni, const ReqDesc* table,
                   int64_t n_upper, int depth, bool one_tree = false);
void launch_finalize(const Launch& l, const Queues& q, const ReqDesc& r, const ReqDesc* table, int slot,
                     uint32_t p0, uint32_t p1);
void launch_set_desc(const Launch& l, ReqDesc* table, int slot, const ReqDesc& r);

// adjoint kernels
// floats of the scalar-partials buffer (ReqDesc::d_part) for waves of up to
// pixels_per_wave pixels and a projector of proj_pixels pixels
size_t partial_floats(int64_t pixels_per_wave, int64_t proj_pixels);
// pix_dE (optional): per-pixel cotangent of the clipped pixel mean (rgb, -), whole image
void launch_adj_pixel(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, uint32_t p0,
                      uint32_t p1, const float* sample_L, float4* pix_dE = nullptr);
void launch_adj_raygen(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, int slot, uint32_t g0,
                       uint32_t n);
void launch_adj_shade(const Launch& l, const Queues& q, const AdjQueues& aq, int cur, int depth, const ReqDesc& uni,
                      const ReqDesc* table, int64_t n_upper);
void launch_adj_shadow(const Launch& l, const Queues& q, const AdjQueues& aq, int which, int nxt, const ReqDesc& uni,
                       const ReqDesc* table, int64_t n_upper);
// replay of one bounce from the path records (no tracing): shade, next-event gradients
// for the recorded visibilities, bounce
void launch_adj_replay(const Launch& l, const Queues& q, const AdjQueues& aq, int cur, int depth, const ReqDesc& uni,
                       const ReqDesc* table, int64_t n_upper);
// adds the binned records of tb / eb into r.d_tex / r.dEp and empties the bins
void launch_map_flush(const Launch& l, const AdjQueues& aq, const ReqDesc& r);
// tile side and bin count for a W x H map (false: too many tiles, bin nothing)
bool map_tiling(int W, int H, int& T, int& nbx, int& nby);
// PRF backward, map de-interleave and scalar gradients; acc: 20 floats (see adjoint.hip)
// camera-pose gradient of a wave's camera samples (after launch_adj_pixel, with path
// records): per-workgroup partials into r.d_cam_part (cam_partial_floats of the wave's
// samples), summed in a fixed order into r.d_acc[20..32)
size_t cam_partial_floats(int64_t samples_per_wave);
void launch_cam_grad(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, uint32_t p0, uint32_t p1);
// dst[k] += the sum of nb partials part[b * stride + k], k < nv, in a fixed order
void launch_sum_partials(const Launch& l, const float* part, int nb, int stride, int nv, float* dst);
void launch_adj_finish(const Launch& l, const ReqDesc& r, float* d_proj, float* d_albedo, float* d_rough,
                       float* d_spec, float* d_scalars, float* acc, float* d_metal = nullptr,
                       float* d_nmap = nullptr);
void launch_zero(const Launch& l, float* p, int64_t n);
// Float buffers cleared together by one launch on l's stream: add() collects them (a
// full list is cleared at once and started again), launch() clears what is held.
constexpr int ZERO_LIST_MAX = 8;
struct ZeroArgs {
    float* p[ZERO_LIST_MAX];
    int64_t n[ZERO_LIST_MAX];
};
struct ZeroList {
    explicit ZeroList(const Launch& l) : l(l) {}
    void add(float* ptr, int64_t count);
    void launch();
    Launch l;
    ZeroArgs a{};
    int k = 0;
};

// debug
void launch_debug_intersect(const Launch& l, const float4* nodes4, const float4* nodes, const float4* tris,
                            const int* leaf_of_prim, int nt, float tmin, const float* rays, int64_t n, int mode,
                            int32_t* prim, float* t, float* b1, float* b2);
void launch_debug_brdf(const Launch& l, int kind, const double* in, int64_t n, double* out);
// guide features through the pixel centres (out: Wc x Hc x 8 floats, 16-byte aligned)
void launch_gbuffer(const Launch& l, const ReqDesc& r, float* out);
void launch_debug_philox(const Launch& l, uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out);

}  // namespace dpcs
