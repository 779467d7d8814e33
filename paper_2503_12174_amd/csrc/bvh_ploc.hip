// bvh_ploc.hip -- device construction of an SAH-quality binary BVH by parallel
// locally-ordered clustering (Meister & Bittner, IEEE TVCG 2018), the device collapse of
// a binary BVH into the 4-wide tree the renderer traverses, and the device checks of a
// built tree.  The host reads back one 8-byte count per clustering round and per
// collapsed level, never the tree.
//
// Clustering: the triangles in Morton order start as one cluster each.  Every round, each
// cluster finds the neighbour within PLOC_R places of it in the current order whose union
// box has the least surface area (ties go to the pair of smaller indices); mutual nearest
// neighbours merge into a new internal node, and the survivors are compacted in order.
// The pair with the globally least cost is chosen from both sides, so every round merges.
// Internal node ids are handed out from nt - 2 downward by a prefix sum over the merging
// pairs: the last merge -- the root -- is node 0 and the ids do not depend on scheduling.
//
// Collapse: breadth first, one level per launch; each 4-wide node takes a binary node's
// two children and keeps opening the internal child with the largest surface area (the
// first such child on a tie) until it holds four.  The next level is numbered by a prefix
// sum over this level's nodes in order, so the numbering is breadth first and the top of
// the tree is the leading block of nodes (what a traversal workgroup stages in LDS).  The
// pass also records the binary node or leaf behind every slot (for refits), the worst
// traversal stack on any root-to-node path, and how often each leaf is reached.
#include <climits>
#include <cstring>

#include "kernels.hpp"
#include "prefix.hpp"

namespace dpcs {

constexpr int PLOC_R = 16;   // search radius in the Morton order
constexpr int TB = SCAN_TB;  // workgroup size of every kernel here except the block-sum scan

// ---------------------------------------------------------------- clustering
__device__ __forceinline__ float union_area(float4 alo, float4 ahi, float4 blo, float4 bhi) {
    const float dx = fmaxf(ahi.x, bhi.x) - fminf(alo.x, blo.x);
    const float dy = fmaxf(ahi.y, bhi.y) - fminf(alo.y, blo.y);
    const float dz = fmaxf(ahi.z, bhi.z) - fminf(alo.z, blo.z);
    return dx * dy + dy * dz + dz * dx;
}

// one cluster per leaf (leaf l is triangle order[l]); lo.w holds the cluster's reference,
// here the leaf ~l
__global__ void k_ploc_init(const float* __restrict__ V, const int* __restrict__ F, const uint32_t* __restrict__ order,
                            int n, float4* __restrict__ lo, float4* __restrict__ hi) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const uint32_t p = order[l];
    float b[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (p < (uint32_t)n) {
        const int a = F[3 * p], c = F[3 * p + 1], e = F[3 * p + 2];
        for (int k = 0; k < 3; ++k) {
            const float x = V[3 * a + k], y = V[3 * c + k], z = V[3 * e + k];
            b[k] = fminf(x, fminf(y, z));
            b[3 + k] = fmaxf(x, fmaxf(y, z));
        }
    }
    lo[l] = make_float4(b[0], b[1], b[2], __int_as_float(~l));
    hi[l] = make_float4(b[3], b[4], b[5], 0.f);
}

// nearest neighbour of every cluster within PLOC_R places (the window staged in LDS).
// Pairs are ranked by (cost, distance in the order, odd lower index, lower index) -- a
// strict order on pairs, the same seen from both clusters -- so the globally least pair is
// mutual and every round merges.  Among equal costs the tie rule pairs a run of identical
// clusters as (0,1), (2,3), ..., halving the run each round instead of peeling it one
// cluster at a time.
__global__ void __launch_bounds__(TB) k_ploc_nn(const float4* __restrict__ lo, const float4* __restrict__ hi, int m,
                                                int* __restrict__ nn) {
    __shared__ float4 slo[TB + 2 * PLOC_R], shi[TB + 2 * PLOC_R];
    const int base = blockIdx.x * TB;
    for (int k = threadIdx.x; k < TB + 2 * PLOC_R; k += TB) {
        const int g = base - PLOC_R + k;
        if (g >= 0 && g < m) {
            slo[k] = lo[g];
            shi[k] = hi[g];
        }
    }
    __syncthreads();
    const int i = base + threadIdx.x;
    if (i >= m) return;
    const int si = threadIdx.x + PLOC_R;
    const float4 alo = slo[si], ahi = shi[si];
    float best = 0.0f;
    int bj = -1;
    for (int d = -PLOC_R; d <= PLOC_R; ++d) {
        const int j = i + d;
        if (d == 0 || j < 0 || j >= m) continue;
        const float a = union_area(alo, ahi, slo[si + d], shi[si + d]);
        bool take = bj < 0 || a < best;
        if (!take && a == best) {
            const int dj = abs(d), db = abs(bj - i);
            const int p0 = min(i, j), q0 = min(i, bj);
            take = dj < db || (dj == db && ((p0 & 1) < (q0 & 1) || ((p0 & 1) == (q0 & 1) && p0 < q0)));
        }
        if (take) {
            best = a;
            bj = j;
        }
    }
    nn[i] = bj;
}

// (merges, survivors) of cluster i packed low / high: the lower index of a mutual pair
// merges, the higher one is absorbed
__device__ __forceinline__ uint64_t ploc_flags(const int* __restrict__ nn, int m, int i, int* partner) {
    const int j = nn[i];
    const bool mutual = j >= 0 && j < m && nn[j] == i;
    *partner = mutual ? j : -1;
    if (mutual && j < i) return 0;
    return (mutual ? 1ull : 0ull) | (1ull << 32);
}

__global__ void __launch_bounds__(TB) k_ploc_count(const int* __restrict__ nn, int m, uint64_t* __restrict__ sums) {
    __shared__ uint64_t ws[TB / 64];
    const int i = blockIdx.x * TB + threadIdx.x;
    int j;
    const uint64_t v = i < m ? ploc_flags(nn, m, i, &j) : 0;
    uint64_t tot;
    block_exclusive(v, ws, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// the merging pairs' internal nodes (id = top - merges before), their children and
// parents, and the compacted cluster list of the next round
__global__ void __launch_bounds__(TB) k_ploc_merge(const float4* __restrict__ lo, const float4* __restrict__ hi,
                                                   const int* __restrict__ nn, int m, const uint64_t* __restrict__ sums,
                                                   int top, int nt, float4* __restrict__ nodes, int* __restrict__ child,
                                                   int* __restrict__ parent_int, int* __restrict__ parent_leaf,
                                                   float4* __restrict__ lo2, float4* __restrict__ hi2) {
    __shared__ uint64_t ws[TB / 64];
    const int i = blockIdx.x * TB + threadIdx.x;
    int j = -1;
    const uint64_t v = i < m ? ploc_flags(nn, m, i, &j) : 0;
    uint64_t tot;
    const uint64_t pre = sums[blockIdx.x] + block_exclusive(v, ws, &tot);
    if (i >= m || v == 0) return;   // out of range, or absorbed by its partner
    float4 nlo = lo[i], nhi = hi[i];
    if (j >= 0) {
        const int id = top - (int)(uint32_t)pre;
        if (id < 0 || id >= nt - 1) return;   // never for a consistent prefix sum
        const float4 blo = lo[j], bhi = hi[j];
        const int ra = __float_as_int(nlo.w), rb = __float_as_int(blo.w);
        nodes[4 * id] = make_float4(nlo.x, nlo.y, nlo.z, nhi.x);
        nodes[4 * id + 1] = make_float4(nhi.y, nhi.z, blo.x, blo.y);
        nodes[4 * id + 2] = make_float4(blo.z, bhi.x, bhi.y, bhi.z);
        nodes[4 * id + 3] = make_float4(__int_as_float(ra), __int_as_float(rb), 0.0f, 0.0f);
        child[2 * id] = ra;
        child[2 * id + 1] = rb;
        for (const int r : {ra, rb}) {
            if (r < 0 && ~r < nt) parent_leaf[~r] = id;
            else if (r >= 0 && r < nt - 1) parent_int[r] = id;
        }
        nlo = make_float4(fminf(nlo.x, blo.x), fminf(nlo.y, blo.y), fminf(nlo.z, blo.z), __int_as_float(id));
        nhi = make_float4(fmaxf(nhi.x, bhi.x), fmaxf(nhi.y, bhi.y), fmaxf(nhi.z, bhi.z), 0.0f);
    }
    const uint32_t pos = (uint32_t)(pre >> 32);
    if (pos < (uint32_t)m) {
        lo2[pos] = nlo;
        hi2[pos] = nhi;
    }
}

static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline size_t r256(size_t b) { return (b + 255) & ~size_t(255); }

size_t ploc_scratch_bytes(int nt) {
    const size_t n = (size_t)nt;
    return 4 * r256(16 * n) + r256(4 * n) + r256(8 * (n / TB + 1)) + 256;
}

hipError_t build_ploc(hipStream_t st, const BvhInputs& in, const uint32_t* order, void* scratch, uint64_t* host_word,
                      float4* nodes) {
    const int n = in.nt;
    if (n < 2) return hipErrorInvalidValue;
    char* s = (char*)scratch;
    auto take = [&](size_t b) {
        char* p = s;
        s += r256(b);
        return (void*)p;
    };
    float4* lo[2] = {(float4*)take(16 * (size_t)n), (float4*)take(16 * (size_t)n)};
    float4* hi[2] = {(float4*)take(16 * (size_t)n), (float4*)take(16 * (size_t)n)};
    int* nn = (int*)take(4 * (size_t)n);
    uint64_t* sums = (uint64_t*)take(8 * ((size_t)n / TB + 1));
    uint64_t* total = (uint64_t*)take(8);
    hipLaunchKernelGGL(k_ploc_init, dim3(grid_of(n, TB)), dim3(TB), 0, st, in.V, in.F, order, n, lo[0], hi[0]);
    int m = n, cur = 0, top = n - 2;
    while (m > 1) {
        const unsigned nb = grid_of(m, TB);
        hipLaunchKernelGGL(k_ploc_nn, dim3(nb), dim3(TB), 0, st, lo[cur], hi[cur], m, nn);
        hipLaunchKernelGGL(k_ploc_count, dim3(nb), dim3(TB), 0, st, nn, m, sums);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, sums, (int)nb, total);
        hipLaunchKernelGGL(k_ploc_merge, dim3(nb), dim3(TB), 0, st, lo[cur], hi[cur], nn, m, sums, top, n, nodes,
                           in.child, in.parent_int, in.parent_leaf, lo[cur ^ 1], hi[cur ^ 1]);
        hipError_t e = hipMemcpyAsync(host_word, total, sizeof(uint64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        const int merges = (int)(uint32_t)*host_word, survivors = (int)(*host_word >> 32);
        // every round merges at least the globally least pair; anything else is a broken
        // build (non-finite boxes), reported rather than looped on
        if (merges < 1 || survivors != m - merges || merges > top + 1) return hipErrorUnknown;
        top -= merges;
        m = survivors;
        cur ^= 1;
    }
    return top == -1 ? hipGetLastError() : hipErrorUnknown;
}

// ---------------------------------------------------------------- checks
// stats: [0] worst 4-wide stack, [1] malformed tree flag, [2] binary depth, [3] unused
__global__ void k_tree_depth(const int* __restrict__ parent_int, const int* __restrict__ parent_leaf, int nt,
                             int* __restrict__ stats) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nt) return;
    int node = parent_leaf[l], d = 1;
    while (node > 0 && node < nt - 1 && d <= 4096) {
        node = parent_int[node];
        ++d;
    }
    if (node != 0) atomicExch(&stats[1], 1);   // the parent chain does not end at the root
    atomicMax(&stats[2], d);
}

__global__ void k_count_refs(const uint32_t* __restrict__ order, int nt, int* __restrict__ seen) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nt && order[l] < (uint32_t)nt) atomicAdd(&seen[order[l]], 1);
}

// every counter exactly one, else the malformed flag
__global__ void k_check_once(const int* __restrict__ seen, int n, int* __restrict__ stats) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n && seen[l] != 1) atomicExch(&stats[1], 1);
}

// ---------------------------------------------------------------- 4-wide collapse
struct Kid {
    int ref;     // binary node (>= 0) or ~leaf
    float b[6];  // lo.xyz, hi.xyz
};

__device__ __forceinline__ Kid bin_kid(const float4* __restrict__ nodes, int node, int k) {
    const float4* p = nodes + 4 * (size_t)node;
    Kid c;
    if (k == 0) {
        const float4 n0 = p[0], n1 = p[1];
        c.b[0] = n0.x; c.b[1] = n0.y; c.b[2] = n0.z; c.b[3] = n0.w; c.b[4] = n1.x; c.b[5] = n1.y;
        c.ref = __float_as_int(p[3].x);
    } else {
        const float4 n1 = p[1], n2 = p[2];
        c.b[0] = n1.z; c.b[1] = n1.w; c.b[2] = n2.x; c.b[3] = n2.y; c.b[4] = n2.z; c.b[5] = n2.w;
        c.ref = __float_as_int(p[3].y);
    }
    return c;
}

__device__ __forceinline__ double kid_area(const Kid& c) {
    const double dx = (double)c.b[3] - c.b[0], dy = (double)c.b[4] - c.b[1], dz = (double)c.b[5] - c.b[2];
    return dx * dy + dy * dz + dz * dx;
}

// the up to four children of the 4-wide node over binary node b; returns how many
__device__ int pick_kids(const float4* __restrict__ nodes, int ni, int b, Kid k[4]) {
    if (b < 0 || b >= ni) return 0;
    k[0] = bin_kid(nodes, b, 0);
    k[1] = bin_kid(nodes, b, 1);
    int cnt = 2;
    while (cnt < 4) {
        int best = -1;
        double ba = -1.0;
        for (int j = 0; j < cnt; ++j)
            if (k[j].ref >= 0 && k[j].ref < ni && kid_area(k[j]) > ba) {
                ba = kid_area(k[j]);
                best = j;
            }
        if (best < 0) break;
        const int c = k[best].ref;
        for (int j = best; j + 1 < cnt; ++j) k[j] = k[j + 1];   // remove it, keeping the order
        k[cnt - 1] = bin_kid(nodes, c, 0);                       // and append its two children
        k[cnt] = bin_kid(nodes, c, 1);
        ++cnt;
    }
    return cnt;
}

__device__ __forceinline__ int internal_kids(const Kid k[4], int cnt) {
    int c = 0;
    for (int j = 0; j < 4; ++j) c += (j < cnt && k[j].ref >= 0) ? 1 : 0;
    return c;
}

__global__ void k_collapse_root(int* __restrict__ bin, int* __restrict__ acc, int* __restrict__ stats) {
    bin[0] = 0;
    acc[0] = 0;
    for (int k = 0; k < 4; ++k) stats[k] = 0;
}

__global__ void __launch_bounds__(TB) k_collapse_count(const float4* __restrict__ nodes, int ni, const int* __restrict__ bin,
                                                       int m, uint64_t* __restrict__ sums) {
    __shared__ uint64_t ws[TB / 64];
    const int e = blockIdx.x * TB + threadIdx.x;
    uint64_t v = 0;
    if (e < m) {
        Kid k[4];
        v = (uint64_t)internal_kids(k, pick_kids(nodes, ni, bin[e], k));
    }
    uint64_t tot;
    block_exclusive(v, ws, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// 4-wide node base + e over binary node bin[e]; its internal children become the next
// level's entries base + m + prefix, carrying the stack depth reached at this node
__global__ void __launch_bounds__(TB) k_collapse_write(const float4* __restrict__ nodes, int ni, const int* __restrict__ bin,
                                                       const int* __restrict__ acc, int m, const uint64_t* __restrict__ sums,
                                                       int base, int cap4, int nt, float4* __restrict__ nodes4,
                                                       int* __restrict__ map4, int* __restrict__ nbin,
                                                       int* __restrict__ nacc, int* __restrict__ stats,
                                                       int* __restrict__ leaf_seen) {
    __shared__ uint64_t ws[TB / 64];
    const int e = blockIdx.x * TB + threadIdx.x;
    Kid k[4];
    int cnt = 0, internal = 0;
    if (e < m) {
        cnt = pick_kids(nodes, ni, bin[e], k);
        internal = internal_kids(k, cnt);
    }
    uint64_t tot;
    int slot = (int)(sums[blockIdx.x] + block_exclusive((uint64_t)internal, ws, &tot));
    if (e >= m) return;
    const int w = base + e;
    if (cnt < 2 || w >= cap4) {   // never for a well-formed tree
        atomicExch(&stats[1], 1);
        return;
    }
    const int a = acc[e] + max(internal - 1, 0);   // stack entries held below this node
    atomicMax(&stats[0], a);
    const int next_base = base + m;
    float box[6][4];
    int refs[4];
    for (int j = 0; j < 4; ++j) {
        if (j >= cnt) {   // empty slot: inverted box far away (never entered), dummy leaf nt
            for (int q = 0; q < 3; ++q) {
                box[q][j] = 1e30f;
                box[q + 3][j] = -1e30f;
            }
            refs[j] = ~nt;
            map4[4 * (size_t)w + j] = INT_MIN;
            continue;
        }
        for (int q = 0; q < 6; ++q) box[q][j] = k[j].b[q];
        const int r = k[j].ref;
        map4[4 * (size_t)w + j] = r;
        if (r >= 0) {
            refs[j] = next_base + slot;
            if (refs[j] >= cap4 || r >= ni) {
                atomicExch(&stats[1], 1);
                refs[j] = ~nt;
            } else {
                nbin[slot] = r;
                nacc[slot] = a;
            }
            ++slot;
        } else {
            refs[j] = r;
            if (~r < nt) atomicAdd(&leaf_seen[~r], 1);
            else atomicExch(&stats[1], 1);
        }
    }
    float4* o = nodes4 + 8 * (size_t)w;
    for (int q = 0; q < 6; ++q) o[q] = make_float4(box[q][0], box[q][1], box[q][2], box[q][3]);
    o[6] = make_float4(__int_as_float(refs[0]), __int_as_float(refs[1]), __int_as_float(refs[2]),
                       __int_as_float(refs[3]));
    o[7] = make_float4(0.f, 0.f, 0.f, 0.f);
}

size_t wide_scratch_bytes(int nt) {
    const size_t ni = (size_t)(nt > 1 ? nt - 1 : 1), n = (size_t)nt;
    return 4 * r256(4 * ni) + r256(8 * (ni / TB + 1)) + 256 + 2 * r256(4 * n) + r256(128 * ni) + r256(16 * ni);
}

hipError_t build_wide(hipStream_t st, const WideArgs& a, void* scratch, uint64_t* host_words, WideResult& res) {
    const int nt = a.nt, ni = nt - 1, cap4 = ni;
    res = WideResult{};
    if (nt < 2) return hipErrorInvalidValue;
    char* s = (char*)scratch;
    auto take = [&](size_t b) {
        char* p = s;
        s += r256(b);
        return (void*)p;
    };
    int* bin[2] = {(int*)take(4 * (size_t)ni), (int*)take(4 * (size_t)ni)};
    int* acc[2] = {(int*)take(4 * (size_t)ni), (int*)take(4 * (size_t)ni)};
    uint64_t* sums = (uint64_t*)take(8 * ((size_t)ni / TB + 1));
    uint64_t* total = (uint64_t*)take(256);
    int* stats = (int*)(total + 1);
    int* leaf_seen = (int*)take(4 * (size_t)nt);
    int* prim_seen = (int*)take(4 * (size_t)nt);
    res.nodes4 = (float4*)take(128 * (size_t)ni);
    res.map4 = (int*)take(16 * (size_t)ni);
    hipError_t e = hipMemsetAsync(leaf_seen, 0, 4 * (size_t)nt, st);
    if (e == hipSuccess) e = hipMemsetAsync(prim_seen, 0, 4 * (size_t)nt, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_collapse_root, dim3(1), dim3(1), 0, st, bin[0], acc[0], stats);
    // the binary tree: every parent chain ends at the root, the leaf order is a permutation
    hipLaunchKernelGGL(k_tree_depth, dim3(grid_of(nt, TB)), dim3(TB), 0, st, a.parent_int, a.parent_leaf, nt, stats);
    hipLaunchKernelGGL(k_count_refs, dim3(grid_of(nt, TB)), dim3(TB), 0, st, a.order, nt, prim_seen);
    hipLaunchKernelGGL(k_check_once, dim3(grid_of(nt, TB)), dim3(TB), 0, st, prim_seen, nt, stats);
    int m = 1, base = 0, cur = 0, levels = 0;
    while (m > 0) {
        // the 4-wide nodes stand for distinct binary nodes, and a tree no deeper than 4096
        // has no more 4-wide levels than that
        if (base + m > cap4 || ++levels > 4096) return hipErrorUnknown;
        const unsigned nb = grid_of(m, TB);
        hipLaunchKernelGGL(k_collapse_count, dim3(nb), dim3(TB), 0, st, a.nodes, ni, bin[cur], m, sums);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, sums, (int)nb, total);
        hipLaunchKernelGGL(k_collapse_write, dim3(nb), dim3(TB), 0, st, a.nodes, ni, bin[cur], acc[cur], m, sums, base,
                           cap4, nt, res.nodes4, res.map4, bin[cur ^ 1], acc[cur ^ 1], stats, leaf_seen);
        e = hipMemcpyAsync(host_words, total, sizeof(uint64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        base += m;
        m = (int)(uint32_t)host_words[0];
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_check_once, dim3(grid_of(nt, TB)), dim3(TB), 0, st, leaf_seen, nt, stats);
    e = hipMemcpyAsync(host_words, stats, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    int hs[4];
    std::memcpy(hs, host_words, sizeof hs);
    res.nnodes4 = base;
    res.depth4 = levels;
    res.stack_bound = hs[0];
    res.malformed = hs[1] != 0;
    res.depth = hs[2];
    return hipGetLastError();
}

}  // namespace dpcs
