// bvh_sah.hip -- device construction of the binary BVH by binned surface-area heuristic,
// top down and breadth first (one level of tasks per round of launches).
//
// A task is a range [a, b) of the leaf order holding >= 2 triangles, with the box of
// their centroids.  Its triangles are binned by centroid into SAH_BINS bins along every
// axis with a non-zero centroid extent, and the split minimising
// area(left) x count(left) + area(right) x count(right) is taken (ties to the lower axis
// and bin).  A task whose centroids coincide is split at the middle of its range.  The
// range is then partitioned stably (left side first, order kept), and the task's node is
// written with both child boxes; children of >= 2 triangles become the next level's tasks,
// single triangles are leaves (leaf l is triangle order[l]).
//
// Work is cut into chunks of SAH_CHUNK triangles, one workgroup each.  A task of one chunk
// is binned, split and partitioned inside its workgroup (LDS only); a larger task merges
// its chunks' bins with global atomics, is split by one thread, and is partitioned by its
// chunks through a staging copy.  Node ids are handed out breadth first by prefix sums, so
// the tree does not depend on scheduling.  Boxes are accumulated as order-preserving
// integer images of the floats (exact min / max).
#include <algorithm>
#include <cfloat>
#include <climits>

#include "kernels.hpp"
#include "prefix.hpp"

namespace dpcs {

namespace {

constexpr int SAH_BINS = 32;
constexpr int SAH_CHUNK = 1024;
constexpr int TB = SCAN_TB;   // every kernel here but the block-sum scan
constexpr int PER = SAH_CHUNK / TB;
constexpr int BIN_INTS = 7;   // count, lo.xyz, hi.xyz
constexpr int LARGE_BIN_INTS = 3 * SAH_BINS * BIN_INTS;

struct SahTask {
    int a, b, node;
    int c0;       // first chunk of the task in this level's chunk list
    int cb[6];    // centroid box (lo.xyz, hi.xyz), order-preserving integers
    int large;    // index among this level's multi-chunk tasks, or -1
    int pad;
};
struct SahRes {
    int axis, split;   // axis -1: coincident centroids, split at the middle of the range
    int nleft;
    int box[2][12];    // per child: box lo.xyz hi.xyz, centroid box lo.xyz hi.xyz (integers)
    int pad;
};

__device__ __forceinline__ int fenc(float f) {
    const int b = __float_as_int(f);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float fdec(int i) { return __int_as_float(i ^ ((i >> 31) & 0x7fffffff)); }

__device__ __forceinline__ void box_init(int* b, int n6) {
    for (int k = 0; k < n6; ++k) {
        b[6 * k + 0] = b[6 * k + 1] = b[6 * k + 2] = fenc(FLT_MAX);
        b[6 * k + 3] = b[6 * k + 4] = b[6 * k + 5] = fenc(-FLT_MAX);
    }
}

__device__ __forceinline__ double enc_area(const int* b) {
    const double dx = fmax(0.0, (double)fdec(b[3]) - fdec(b[0])), dy = fmax(0.0, (double)fdec(b[4]) - fdec(b[1])),
                 dz = fmax(0.0, (double)fdec(b[5]) - fdec(b[2]));
    return dx * dy + dy * dz + dz * dx;
}

// the bin of a centroid coordinate: floor((c - lo) * SAH_BINS / extent), clamped
__device__ __forceinline__ int sah_bin(float c, float lo, double sc) {
    return max(0, min(SAH_BINS - 1, (int)(((double)c - (double)lo) * sc)));
}

struct Tri {
    float lo[3], hi[3], c[3];
};
__device__ __forceinline__ Tri load_tri(const float4* __restrict__ tb, uint32_t p) {
    const float4 a = tb[3 * (size_t)p], b = tb[3 * (size_t)p + 1], c = tb[3 * (size_t)p + 2];
    return Tri{{a.x, a.y, a.z}, {b.x, b.y, b.z}, {c.x, c.y, c.z}};
}

// left side of the task's split?
__device__ __forceinline__ bool goes_left(const SahTask& t, const SahRes& r, const Tri& x, int i) {
    if (r.axis < 0) return i < t.a + (t.b - t.a) / 2;
    const float lo = fdec(t.cb[r.axis]), hi = fdec(t.cb[3 + r.axis]);
    const double sc = SAH_BINS / ((double)hi - lo);
    return sah_bin(x.c[r.axis], lo, sc) < r.split;
}

// best split along one axis of binned counts / boxes (bins[axis][bin][7]): cost -1 when
// the axis has no centroid extent or no split leaves both sides non-empty; split is the
// first bin of the right side, the first of equal costs wins
__device__ void sah_sweep_axis(const int* bins, const int* cb, int ax, double* cost_out, int* split_out) {
    *cost_out = -1.0;
    *split_out = 0;
    if (!((double)fdec(cb[3 + ax]) - fdec(cb[ax]) > 0.0)) return;
    const int* B = bins + ax * SAH_BINS * BIN_INTS;
    double suf_area[SAH_BINS];
    int suf_n[SAH_BINS];
    int acc[6];
    box_init(acc, 1);
    int an = 0;
    for (int s = SAH_BINS - 1; s >= 0; --s) {
        const int* q = B + s * BIN_INTS;
        an += q[0];
        for (int k = 0; k < 3; ++k) {
            acc[k] = min(acc[k], q[1 + k]);
            acc[3 + k] = max(acc[3 + k], q[4 + k]);
        }
        suf_area[s] = enc_area(acc);
        suf_n[s] = an;
    }
    box_init(acc, 1);
    int pn = 0;
    double best = -1.0;
    for (int s = 1; s < SAH_BINS; ++s) {
        const int* q = B + (s - 1) * BIN_INTS;
        pn += q[0];
        for (int k = 0; k < 3; ++k) {
            acc[k] = min(acc[k], q[1 + k]);
            acc[3 + k] = max(acc[3 + k], q[4 + k]);
        }
        if (pn == 0 || suf_n[s] == 0) continue;
        const double cost = enc_area(acc) * pn + suf_area[s] * suf_n[s];
        if (best < 0.0 || cost < best) {
            best = cost;
            *split_out = s;
        }
    }
    *cost_out = best;
}

// the best of the three axes (the lower axis on equal cost); axis -1: none splits
__device__ __forceinline__ void sah_pick(const double cost[3], const int split[3], int* axis, int* sp) {
    *axis = -1;
    *sp = 0;
    double best = -1.0;
    for (int ax = 0; ax < 3; ++ax)
        if (cost[ax] >= 0.0 && (best < 0.0 || cost[ax] < best)) {
            best = cost[ax];
            *axis = ax;
            *sp = split[ax];
        }
}

}  // namespace

// per triangle: box and centroid (3 float4), the identity order, and the root task's
// centroid box (workgroup reduction, then global atomics)
__global__ void __launch_bounds__(TB) k_sah_init(const float* __restrict__ V, const int* __restrict__ F, int nt,
                                                 float4* __restrict__ tb, uint32_t* __restrict__ ord,
                                                 SahTask* __restrict__ root) {
    __shared__ int cb[6];
    if (threadIdx.x == 0) box_init(cb, 1);
    __syncthreads();
    const int p = blockIdx.x * TB + threadIdx.x;
    if (p < nt) {
        const int a = F[3 * p], b = F[3 * p + 1], c = F[3 * p + 2];
        float lo[3], hi[3], ce[3];
        for (int k = 0; k < 3; ++k) {
            const float x = V[3 * a + k], y = V[3 * b + k], z = V[3 * c + k];
            lo[k] = fminf(x, fminf(y, z));
            hi[k] = fmaxf(x, fmaxf(y, z));
            ce[k] = (x + y + z) * (1.0f / 3.0f);   // the centroid as the Morton codes take it
            atomicMin(&cb[k], fenc(ce[k]));
            atomicMax(&cb[3 + k], fenc(ce[k]));
        }
        tb[3 * (size_t)p] = make_float4(lo[0], lo[1], lo[2], 0.f);
        tb[3 * (size_t)p + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
        tb[3 * (size_t)p + 2] = make_float4(ce[0], ce[1], ce[2], 0.f);
        ord[p] = (uint32_t)p;
    }
    __syncthreads();
    if (threadIdx.x < 3) atomicMin(&root->cb[threadIdx.x], cb[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&root->cb[threadIdx.x], cb[threadIdx.x]);
}

__global__ void k_sah_root(SahTask* __restrict__ root, int nt) {
    root->a = 0;
    root->b = nt;
    root->node = 0;
    root->c0 = 0;
    root->large = -1;
    root->pad = 0;
    box_init(root->cb, 1);
}

// chunks (low) and multi-chunk tasks (high) per task, summed per workgroup
__global__ void __launch_bounds__(TB) k_sah_plan_count(const SahTask* __restrict__ tasks, int T,
                                                       uint64_t* __restrict__ sums) {
    __shared__ uint64_t ws[TB / 64];
    const int t = blockIdx.x * TB + threadIdx.x;
    uint64_t v = 0;
    if (t < T) {
        const int n = tasks[t].b - tasks[t].a, nc = (n + SAH_CHUNK - 1) / SAH_CHUNK;
        v = (uint64_t)nc | ((uint64_t)(nc > 1) << 32);
    }
    uint64_t tot;
    block_exclusive(v, ws, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// the chunk list (task, first index), the multi-chunk tasks' list, cleared bins and
// results
__global__ void __launch_bounds__(TB) k_sah_plan_write(SahTask* __restrict__ tasks, int T, const uint64_t* __restrict__ sums,
                                                       int2* __restrict__ chunks, int* __restrict__ large_task,
                                                       int* __restrict__ large_bins, SahRes* __restrict__ res) {
    __shared__ uint64_t ws[TB / 64];
    const int t = blockIdx.x * TB + threadIdx.x;
    int nc = 0;
    uint64_t v = 0;
    if (t < T) {
        const int n = tasks[t].b - tasks[t].a;
        nc = (n + SAH_CHUNK - 1) / SAH_CHUNK;
        v = (uint64_t)nc | ((uint64_t)(nc > 1) << 32);
    }
    uint64_t tot;
    const uint64_t pre = sums[blockIdx.x] + block_exclusive(v, ws, &tot);
    if (t >= T) return;
    SahTask& k = tasks[t];
    const int c0 = (int)(uint32_t)pre, li = (int)(pre >> 32);
    k.c0 = c0;
    k.large = nc > 1 ? li : -1;
    for (int c = 0; c < nc; ++c) chunks[c0 + c] = make_int2(t, k.a + c * SAH_CHUNK);
    SahRes& r = res[t];
    r.axis = -1;
    r.split = 0;
    r.nleft = 0;
    box_init(&r.box[0][0], 4);
    if (nc > 1) {
        large_task[li] = t;
        int* B = large_bins + (size_t)li * LARGE_BIN_INTS;
        for (int q = 0; q < 3 * SAH_BINS; ++q) {
            B[q * BIN_INTS] = 0;
            box_init(B + q * BIN_INTS + 1, 1);
        }
    }
}

// binning of one chunk; a task of one chunk is also split and partitioned here
__global__ void __launch_bounds__(TB) k_sah_bin(const float4* __restrict__ tb, uint32_t* __restrict__ ord,
                                                const SahTask* __restrict__ tasks, const int2* __restrict__ chunks,
                                                const uint64_t* __restrict__ counts, int* __restrict__ large_bins,
                                                SahRes* __restrict__ res) {
    __shared__ int bins[3 * SAH_BINS * BIN_INTS];
    __shared__ int cbox[2][12];
    __shared__ uint32_t part[SAH_CHUNK];
    __shared__ uint64_t ws[TB / 64];
    __shared__ int dec[2];
    __shared__ double acost[3];
    __shared__ int asplit[3];
    const int c = blockIdx.x;
    if (c >= (int)(uint32_t)counts[0]) return;
    const int2 ch = chunks[c];
    const SahTask t = tasks[ch.x];
    const int s = ch.y, e = min(s + SAH_CHUNK, t.b);
    for (int q = threadIdx.x; q < 3 * SAH_BINS; q += TB) {
        bins[q * BIN_INTS] = 0;
        box_init(bins + q * BIN_INTS + 1, 1);
    }
    if (threadIdx.x == 0) box_init(&cbox[0][0], 4);
    float lo[3];
    double sc[3];
    for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = fdec(t.cb[ax]);
        const double ext = (double)fdec(t.cb[3 + ax]) - lo[ax];
        sc[ax] = ext > 0.0 ? SAH_BINS / ext : 0.0;
    }
    __syncthreads();
    // PER consecutive triangles per thread (the partition below keeps their order)
    uint32_t p[PER];
    for (int k = 0; k < PER; ++k) {
        const int i = s + PER * threadIdx.x + k;
        p[k] = i < e ? ord[i] : UINT32_MAX;
        if (i >= e) continue;
        const Tri x = load_tri(tb, p[k]);
        for (int ax = 0; ax < 3; ++ax) {
            if (!(sc[ax] > 0.0)) continue;
            int* q = bins + (ax * SAH_BINS + sah_bin(x.c[ax], lo[ax], sc[ax])) * BIN_INTS;
            atomicAdd(q, 1);
            for (int j = 0; j < 3; ++j) {
                atomicMin(q + 1 + j, fenc(x.lo[j]));
                atomicMax(q + 4 + j, fenc(x.hi[j]));
            }
        }
    }
    __syncthreads();
    if (t.large >= 0) {   // merge into the task's bins
        int* B = large_bins + (size_t)t.large * LARGE_BIN_INTS;
        for (int q = threadIdx.x; q < 3 * SAH_BINS; q += TB) {
            const int* b = bins + q * BIN_INTS;
            if (b[0] == 0) continue;
            atomicAdd(B + q * BIN_INTS, b[0]);
            for (int j = 0; j < 3; ++j) {
                atomicMin(B + q * BIN_INTS + 1 + j, b[1 + j]);
                atomicMax(B + q * BIN_INTS + 4 + j, b[4 + j]);
            }
        }
        return;
    }
    if (threadIdx.x < 3) sah_sweep_axis(bins, t.cb, threadIdx.x, &acost[threadIdx.x], &asplit[threadIdx.x]);
    __syncthreads();
    if (threadIdx.x == 0) sah_pick(acost, asplit, &dec[0], &dec[1]);
    __syncthreads();
    SahRes r;
    r.axis = dec[0];
    r.split = dec[1];
    int nl = 0;
    bool left[PER];
    for (int k = 0; k < PER; ++k) {
        const int i = s + PER * threadIdx.x + k;
        left[k] = false;
        if (i >= e) continue;
        const Tri x = load_tri(tb, p[k]);
        left[k] = goes_left(t, r, x, i);
        nl += left[k];
        int* cbx = cbox[left[k] ? 0 : 1];
        for (int j = 0; j < 3; ++j) {
            atomicMin(cbx + j, fenc(x.lo[j]));
            atomicMax(cbx + 3 + j, fenc(x.hi[j]));
            atomicMin(cbx + 6 + j, fenc(x.c[j]));
            atomicMax(cbx + 9 + j, fenc(x.c[j]));
        }
    }
    uint64_t tot;
    const int lpre = (int)block_exclusive((uint64_t)nl, ws, &tot);
    const int nleft = (int)tot;
    int li = lpre;
    for (int k = 0; k < PER; ++k) {
        const int i = s + PER * threadIdx.x + k;
        if (i >= e) continue;
        const int rel = i - s;
        const int pos = left[k] ? li++ : nleft + (rel - li);
        part[pos] = p[k];
    }
    __syncthreads();
    for (int i = s + threadIdx.x; i < e; i += TB) ord[i] = part[i - s];
    if (threadIdx.x == 0) {
        SahRes& o = res[ch.x];
        o.axis = r.axis;
        o.split = r.split;
        o.nleft = nleft;
        for (int j = 0; j < 12; ++j) {
            o.box[0][j] = cbox[0][j];
            o.box[1][j] = cbox[1][j];
        }
    }
}

// the split of every multi-chunk task from its merged bins
__global__ void k_sah_split_large(const SahTask* __restrict__ tasks, const int* __restrict__ large_task,
                                  const uint64_t* __restrict__ counts, const int* __restrict__ large_bins,
                                  SahRes* __restrict__ res) {
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= (int)(counts[0] >> 32)) return;
    const int t = large_task[li];
    double cost[3];
    int sp[3], axis, split;
    for (int ax = 0; ax < 3; ++ax) sah_sweep_axis(large_bins + (size_t)li * LARGE_BIN_INTS, tasks[t].cb, ax, &cost[ax], &sp[ax]);
    sah_pick(cost, sp, &axis, &split);
    res[t].axis = axis;
    res[t].split = split;
}

// multi-chunk tasks: left count of every chunk, and the children's boxes
__global__ void __launch_bounds__(TB) k_sah_part_count(const float4* __restrict__ tb, const uint32_t* __restrict__ ord,
                                                       const SahTask* __restrict__ tasks, const int2* __restrict__ chunks,
                                                       const uint64_t* __restrict__ counts, int* __restrict__ chunk_left,
                                                       SahRes* __restrict__ res) {
    __shared__ int cbox[2][12];
    __shared__ int nl;
    const int c = blockIdx.x;
    if (c >= (int)(uint32_t)counts[0]) return;
    const int2 ch = chunks[c];
    const SahTask t = tasks[ch.x];
    if (t.large < 0) return;
    const SahRes r = res[ch.x];
    if (threadIdx.x == 0) {
        box_init(&cbox[0][0], 4);
        nl = 0;
    }
    __syncthreads();
    const int s = ch.y, e = min(s + SAH_CHUNK, t.b);
    int my = 0;
    for (int i = s + threadIdx.x; i < e; i += TB) {
        const Tri x = load_tri(tb, ord[i]);
        const bool l = goes_left(t, r, x, i);
        my += l;
        int* cbx = cbox[l ? 0 : 1];
        for (int j = 0; j < 3; ++j) {
            atomicMin(cbx + j, fenc(x.lo[j]));
            atomicMax(cbx + 3 + j, fenc(x.hi[j]));
            atomicMin(cbx + 6 + j, fenc(x.c[j]));
            atomicMax(cbx + 9 + j, fenc(x.c[j]));
        }
    }
    atomicAdd(&nl, my);
    __syncthreads();
    SahRes& o = res[ch.x];
    if (threadIdx.x < 24) {
        const int k = threadIdx.x / 12, j = threadIdx.x % 12;
        if ((j % 6) < 3) atomicMin(&o.box[k][j], cbox[k][j]);
        else atomicMax(&o.box[k][j], cbox[k][j]);
    }
    if (threadIdx.x == 0) {
        chunk_left[c] = nl;
        atomicAdd(&o.nleft, nl);
    }
}

// multi-chunk tasks: stable partition into the staging order
__global__ void __launch_bounds__(TB) k_sah_part_scatter(const float4* __restrict__ tb, const uint32_t* __restrict__ ord,
                                                         const SahTask* __restrict__ tasks, const int2* __restrict__ chunks,
                                                         const uint64_t* __restrict__ counts,
                                                         const int* __restrict__ chunk_left, const SahRes* __restrict__ res,
                                                         uint32_t* __restrict__ staging) {
    __shared__ uint64_t ws[TB / 64];
    const int c = blockIdx.x;
    if (c >= (int)(uint32_t)counts[0]) return;
    const int2 ch = chunks[c];
    const SahTask t = tasks[ch.x];
    if (t.large < 0) return;
    const SahRes r = res[ch.x];
    int before = 0;   // left triangles of the task's earlier chunks
    for (int q = t.c0; q < c; ++q) before += chunk_left[q];
    const int s = ch.y, e = min(s + SAH_CHUNK, t.b);
    uint32_t p[PER];
    bool left[PER];
    int nl = 0;
    for (int k = 0; k < PER; ++k) {
        const int i = s + PER * threadIdx.x + k;
        left[k] = false;
        p[k] = 0;
        if (i >= e) continue;
        p[k] = ord[i];
        left[k] = goes_left(t, r, load_tri(tb, p[k]), i);
        nl += left[k];
    }
    uint64_t tot;
    int li = before + (int)block_exclusive((uint64_t)nl, ws, &tot);
    for (int k = 0; k < PER; ++k) {
        const int i = s + PER * threadIdx.x + k;
        if (i >= e) continue;
        const int rel = i - t.a;   // index within the task
        const int pos = left[k] ? t.a + li++ : t.a + r.nleft + (rel - li);
        if (pos >= t.a && pos < t.b) staging[pos] = p[k];
    }
}

__global__ void __launch_bounds__(TB) k_sah_copy_back(const SahTask* __restrict__ tasks, const int2* __restrict__ chunks,
                                                      const uint64_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ staging, uint32_t* __restrict__ ord) {
    const int c = blockIdx.x;
    if (c >= (int)(uint32_t)counts[0]) return;
    const int2 ch = chunks[c];
    const SahTask t = tasks[ch.x];
    if (t.large < 0) return;
    const int s = ch.y, e = min(s + SAH_CHUNK, t.b);
    for (int i = s + threadIdx.x; i < e; i += TB) ord[i] = staging[i];
}

__device__ __forceinline__ int internal_children(const SahTask& t, const SahRes& r) {
    const int nl = r.nleft, nr = (t.b - t.a) - r.nleft;
    return (nl > 1) + (nr > 1);
}

__global__ void __launch_bounds__(TB) k_sah_emit_count(const SahTask* __restrict__ tasks, int T,
                                                       const SahRes* __restrict__ res, uint64_t* __restrict__ sums) {
    __shared__ uint64_t ws[TB / 64];
    const int t = blockIdx.x * TB + threadIdx.x;
    const uint64_t v = t < T ? (uint64_t)internal_children(tasks[t], res[t]) : 0;
    uint64_t tot;
    block_exclusive(v, ws, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// the level's nodes (child boxes and references, parents) and the next level's tasks
__global__ void __launch_bounds__(TB) k_sah_emit(const SahTask* __restrict__ tasks, int T, const SahRes* __restrict__ res,
                                                 const uint64_t* __restrict__ sums, int next_id, int nt, int tcap,
                                                 float4* __restrict__ nodes, int* __restrict__ child,
                                                 int* __restrict__ parent_int, int* __restrict__ parent_leaf,
                                                 SahTask* __restrict__ next, int* __restrict__ bad) {
    __shared__ uint64_t ws[TB / 64];
    const int t = blockIdx.x * TB + threadIdx.x;
    SahTask k{};
    SahRes r{};
    int ni = 0;
    if (t < T) {
        k = tasks[t];
        r = res[t];
        ni = internal_children(k, r);
    }
    uint64_t tot;
    int slot = (int)(sums[blockIdx.x] + block_exclusive((uint64_t)ni, ws, &tot));
    if (t >= T) return;
    const int mid = k.a + r.nleft;
    if (r.nleft < 1 || mid >= k.b || k.node < 0 || k.node >= nt - 1) {   // never: both sides hold a triangle
        atomicExch(bad, 1);
        return;
    }
    const int lo_[2] = {k.a, mid}, hi_[2] = {mid, k.b};
    int ref[2];
    for (int j = 0; j < 2; ++j) {
        if (hi_[j] - lo_[j] == 1) {
            ref[j] = ~lo_[j];
            parent_leaf[lo_[j]] = k.node;
        } else {
            const int id = next_id + slot;
            if (id >= nt - 1 || slot >= tcap) {
                atomicExch(bad, 1);
                return;
            }
            ref[j] = id;
            parent_int[id] = k.node;
            SahTask& n = next[slot];
            n.a = lo_[j];
            n.b = hi_[j];
            n.node = id;
            n.c0 = 0;
            n.large = -1;
            n.pad = 0;
            for (int q = 0; q < 6; ++q) n.cb[q] = r.box[j][6 + q];
            ++slot;
        }
    }
    float b[2][6];
    for (int j = 0; j < 2; ++j)
        for (int q = 0; q < 6; ++q) b[j][q] = fdec(r.box[j][q]);
    nodes[4 * (size_t)k.node] = make_float4(b[0][0], b[0][1], b[0][2], b[0][3]);
    nodes[4 * (size_t)k.node + 1] = make_float4(b[0][4], b[0][5], b[1][0], b[1][1]);
    nodes[4 * (size_t)k.node + 2] = make_float4(b[1][2], b[1][3], b[1][4], b[1][5]);
    nodes[4 * (size_t)k.node + 3] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), 0.f, 0.f);
    child[2 * (size_t)k.node] = ref[0];
    child[2 * (size_t)k.node + 1] = ref[1];
}

static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline size_t r256(size_t b) { return (b + 255) & ~size_t(255); }

namespace {
struct SahLayout {
    size_t tb, ord, staging, tasks, res, chunks, chunk_left, large_task, large_bins, sums, words, total;
    int tcap, ccap, lcap;
    explicit SahLayout(int nt) {
        const size_t n = (size_t)nt;
        tcap = nt / 2 + 1;
        ccap = tcap + nt / SAH_CHUNK + 1;
        lcap = nt / (SAH_CHUNK + 1) + 1;
        size_t o = 0;
        auto put = [&](size_t b) {
            const size_t at = o;
            o += r256(b);
            return at;
        };
        tb = put(48 * n);
        ord = put(4 * n);
        staging = put(4 * n);
        tasks = put(2 * sizeof(SahTask) * (size_t)tcap);
        res = put(sizeof(SahRes) * (size_t)tcap);
        chunks = put(8 * (size_t)ccap);
        chunk_left = put(4 * (size_t)ccap);
        large_task = put(4 * (size_t)lcap);
        large_bins = put(4 * (size_t)LARGE_BIN_INTS * lcap);
        sums = put(8 * ((size_t)tcap / TB + 1));
        words = put(64);
        total = o;
    }
};
}  // namespace

size_t sah_scratch_bytes(int nt) { return SahLayout(nt).total; }

hipError_t build_sah(hipStream_t st, const BvhInputs& in, void* scratch, uint64_t* host_word, float4* nodes,
                     const uint32_t** order_out) {
    const int nt = in.nt;
    if (nt < 2) return hipErrorInvalidValue;
    const SahLayout L(nt);
    char* base = (char*)scratch;
    float4* tb = (float4*)(base + L.tb);
    uint32_t* ord = (uint32_t*)(base + L.ord);
    uint32_t* staging = (uint32_t*)(base + L.staging);
    SahTask* tasks[2] = {(SahTask*)(base + L.tasks), (SahTask*)(base + L.tasks) + L.tcap};
    SahRes* res = (SahRes*)(base + L.res);
    int2* chunks = (int2*)(base + L.chunks);
    int* chunk_left = (int*)(base + L.chunk_left);
    int* large_task = (int*)(base + L.large_task);
    int* large_bins = (int*)(base + L.large_bins);
    uint64_t* sums = (uint64_t*)(base + L.sums);
    uint64_t* words = (uint64_t*)(base + L.words);   // [0] chunks | large << 32, [1] next tasks, [2] bad flag
    int* bad = (int*)(words + 2);
    *order_out = ord;
    hipLaunchKernelGGL(k_sah_root, dim3(1), dim3(1), 0, st, tasks[0], nt);
    hipLaunchKernelGGL(k_sah_init, dim3(grid_of(nt, TB)), dim3(TB), 0, st, in.V, in.F, nt, tb, ord, tasks[0]);
    hipError_t e = hipMemsetAsync(words, 0, 64, st);
    if (e != hipSuccess) return e;
    int T = 1, next_id = 1, cur = 0;
    for (int level = 1; T > 0; ++level) {
        // binary depth is capped at 64 levels for the traversal's stack; a deeper SAH tree is
        // refused rather than built
        if (level > 64) return hipErrorNotSupported;
        const unsigned nbT = grid_of(T, TB);
        const unsigned cub = (unsigned)std::min<int64_t>((int64_t)T + nt / SAH_CHUNK + 1, L.ccap);
        const unsigned lub = (unsigned)std::min(T, L.lcap);
        hipLaunchKernelGGL(k_sah_plan_count, dim3(nbT), dim3(TB), 0, st, tasks[cur], T, sums);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, sums, (int)nbT, words);
        hipLaunchKernelGGL(k_sah_plan_write, dim3(nbT), dim3(TB), 0, st, tasks[cur], T, sums, chunks, large_task,
                           large_bins, res);
        hipLaunchKernelGGL(k_sah_bin, dim3(cub), dim3(TB), 0, st, tb, ord, tasks[cur], chunks, words, large_bins, res);
        hipLaunchKernelGGL(k_sah_split_large, dim3(grid_of(lub, 64)), dim3(64), 0, st, tasks[cur], large_task, words,
                           large_bins, res);
        hipLaunchKernelGGL(k_sah_part_count, dim3(cub), dim3(TB), 0, st, tb, ord, tasks[cur], chunks, words, chunk_left,
                           res);
        hipLaunchKernelGGL(k_sah_part_scatter, dim3(cub), dim3(TB), 0, st, tb, ord, tasks[cur], chunks, words,
                           chunk_left, res, staging);
        hipLaunchKernelGGL(k_sah_copy_back, dim3(cub), dim3(TB), 0, st, tasks[cur], chunks, words, staging, ord);
        hipLaunchKernelGGL(k_sah_emit_count, dim3(nbT), dim3(TB), 0, st, tasks[cur], T, res, sums);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, sums, (int)nbT, words + 1);
        hipLaunchKernelGGL(k_sah_emit, dim3(nbT), dim3(TB), 0, st, tasks[cur], T, res, sums, next_id, nt, L.tcap, nodes,
                           in.child, in.parent_int, in.parent_leaf, tasks[cur ^ 1], bad);
        e = hipMemcpyAsync(host_word, words + 1, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        const int tn = (int)host_word[0];
        if ((int)host_word[1] != 0 || tn > L.tcap || next_id + tn > nt - 1) return hipErrorUnknown;
        next_id += tn;
        T = tn;
        cur ^= 1;
    }
    return next_id == nt - 1 ? hipGetLastError() : hipErrorUnknown;
}

}  // namespace dpcs
