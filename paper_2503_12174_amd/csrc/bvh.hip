// bvh.hip -- GPU construction of the binary BVH over a triangle mesh.
//
//  1. Morton code (30 bits) of every triangle centroid in the centroid bounding box.
//  2. Stable LSD radix sort of (code, triangle) pairs, 8-bit digits: per-tile digit
//     histograms, one exclusive scan, and a scatter that ranks equal digits inside a
//     tile with wave64 ballots (match mask from 8 ballots, rank = popcount below).
//  3. Binary radix tree over the sorted codes (Karras, HPG 2012): one thread per
//     internal node finds its key range and split; equal codes split by index.
//  4. Bounds bottom-up: a thread per leaf climbs; the second thread to reach a node
//     (atomic arrival counter) writes the node's two child boxes and continues.
//  5. Leaf-ordered 48-byte triangle records and UV / emission records.
#include <climits>

#include "kernels.hpp"

namespace dpcs {

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(const float* __restrict__ V, const int* __restrict__ F, int nt, float lx, float ly, float lz,
                         float sx, float sy, float sz, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nt) return;
    const int a = F[3 * p], b = F[3 * p + 1], c = F[3 * p + 2];
    const float cx = (V[3 * a] + V[3 * b] + V[3 * c]) * (1.0f / 3.0f);
    const float cy = (V[3 * a + 1] + V[3 * b + 1] + V[3 * c + 1]) * (1.0f / 3.0f);
    const float cz = (V[3 * a + 2] + V[3 * b + 2] + V[3 * c + 2]) * (1.0f / 3.0f);
    const float qx = fminf(fmaxf((cx - lx) * sx, 0.0f), 1023.0f);
    const float qy = fminf(fmaxf((cy - ly) * sy, 0.0f), 1023.0f);
    const float qz = fminf(fmaxf((cz - lz) * sz, 0.0f), 1023.0f);
    keys[p] = (spread10((uint32_t)qx) << 2) | (spread10((uint32_t)qy) << 1) | spread10((uint32_t)qz);
    vals[p] = (uint32_t)p;
}

// ---------------------------------------------------------------- radix sort
constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 4;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;

__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                            uint32_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int tile = blockIdx.x;
    for (int k = 0; k < SORT_ROUNDS; ++k) {
        const int i = tile * SORT_TILE + k * SORT_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + tile] = h[threadIdx.x];   // digit-major
}

// exclusive scan of n entries in place, one workgroup of 1024 threads
__global__ void __launch_bounds__(1024) k_scan_exclusive(uint32_t* __restrict__ data, int n) {
    __shared__ uint32_t part[1024];
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per;
    const int e = min(b + per, n);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += data[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // Hillis-Steele inclusive scan of the partials
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int i = b; i < e; ++i) {
        const uint32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               int n, int shift, const uint32_t* __restrict__ offsets,
                                                               int ntiles) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[SORT_THREADS / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tile = blockIdx.x;
    base[tid] = offsets[tid * ntiles + tile];
    for (int w = 0; w < SORT_THREADS / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int k = 0; k < SORT_ROUNDS; ++k) {
        const int i = tile * SORT_TILE + k * SORT_THREADS + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const unsigned long long m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            if (pos < (uint32_t)n) {   // always true for a consistent histogram
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < SORT_THREADS / 64; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        base[tid] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- hierarchy
__device__ __forceinline__ int common_prefix(const uint32_t* __restrict__ codes, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint32_t a = codes[i], b = codes[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

__global__ void k_hierarchy(const uint32_t* __restrict__ codes, int n, int* __restrict__ child,
                            int* __restrict__ parent_int, int* __restrict__ parent_leaf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int dir = common_prefix(codes, n, i, i + 1) - common_prefix(codes, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = common_prefix(codes, n, i, i - dir);
    int lmax = 2;
    while (common_prefix(codes, n, i, i + lmax * dir) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (common_prefix(codes, n, i, i + (l + t) * dir) > dmin) l += t;
    const int j = i + l * dir;
    const int dnode = common_prefix(codes, n, i, j);
    int s = 0;
    for (int div = 2;; div <<= 1) {
        const int t = (l + div - 1) / div;
        if (common_prefix(codes, n, i, i + (s + t) * dir) > dnode) s += t;
        if (t <= 1) break;
    }
    const int split = i + s * dir + min(dir, 0);
    const int lo = min(i, j), hi = max(i, j);
    const int left = lo == split ? ~split : split;
    const int right = hi == split + 1 ? ~(split + 1) : split + 1;
    child[2 * i] = left;
    child[2 * i + 1] = right;
    if (left < 0) parent_leaf[~left] = i; else parent_int[left] = i;
    if (right < 0) parent_leaf[~right] = i; else parent_int[right] = i;
}

__device__ __forceinline__ void tri_box(const float* __restrict__ V, const int* __restrict__ F, int p, float* b) {
    const int a = F[3 * p], c = F[3 * p + 1], e = F[3 * p + 2];
    for (int k = 0; k < 3; ++k) {
        const float x = V[3 * a + k], y = V[3 * c + k], z = V[3 * e + k];
        b[k] = fminf(x, fminf(y, z));
        b[3 + k] = fmaxf(x, fmaxf(y, z));
    }
}

__global__ void k_bounds(const float* __restrict__ V, const int* __restrict__ F, const uint32_t* __restrict__ order,
                         int n, const int* __restrict__ child, const int* __restrict__ parent_int,
                         const int* __restrict__ parent_leaf, int* __restrict__ flags, float* node_box,
                         float4* __restrict__ nodes) {
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= n) return;
    int node = parent_leaf[leaf];
    // a valid radix tree has depth < 64 + 32; the bound only guards against a malformed one
    for (int step = 0; step < 128; ++step) {
        if (node < 0 || node >= n - 1) return;
        __threadfence();
        if (atomicAdd(&flags[node], 1) == 0) return;   // the sibling's thread finishes this node
        __threadfence();
        float bx[2][6];
        int ch[2] = {child[2 * node], child[2 * node + 1]};
        for (int k = 0; k < 2; ++k) {
            if (ch[k] < -n || ch[k] >= n - 1) return;
            if (ch[k] < 0) {
                const uint32_t p = order[~ch[k]];
                if (p >= (uint32_t)n) return;
                tri_box(V, F, (int)p, bx[k]);
            } else {
                const volatile float* src = node_box + 6 * ch[k];
                for (int q = 0; q < 6; ++q) bx[k][q] = src[q];
            }
        }
        nodes[4 * node] = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
        nodes[4 * node + 1] = make_float4(bx[0][4], bx[0][5], bx[1][0], bx[1][1]);
        nodes[4 * node + 2] = make_float4(bx[1][2], bx[1][3], bx[1][4], bx[1][5]);
        nodes[4 * node + 3] = make_float4(__int_as_float(ch[0]), __int_as_float(ch[1]), 0.0f, 0.0f);
        volatile float* dst = node_box + 6 * node;
        for (int q = 0; q < 3; ++q) {
            dst[q] = fminf(bx[0][q], bx[1][q]);
            dst[3 + q] = fmaxf(bx[0][3 + q], bx[1][3 + q]);
        }
        if (node == 0) return;
        node = parent_int[node];
    }
}

// single-triangle scene: one node whose two children are the same leaf
__global__ void k_single_node(const float* __restrict__ V, const int* __restrict__ F, float4* __restrict__ nodes) {
    float b[6];
    tri_box(V, F, 0, b);
    nodes[0] = make_float4(b[0], b[1], b[2], b[3]);
    nodes[1] = make_float4(b[4], b[5], b[0], b[1]);
    nodes[2] = make_float4(b[2], b[3], b[4], b[5]);
    nodes[3] = make_float4(__int_as_float(~0), __int_as_float(~0), 0.0f, 0.0f);
}

__global__ void k_leaf_records(const float* __restrict__ V, const int* __restrict__ F, const float* __restrict__ UV,
                               const float* __restrict__ Le, const uint32_t* __restrict__ order, int n,
                               float4* __restrict__ tris, float4* __restrict__ tri_uv, float4* __restrict__ em,
                               int* __restrict__ leaf_of_prim) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    if (order[l] >= (uint32_t)n) return;
    const int p = (int)order[l];
    const int a = F[3 * p], b = F[3 * p + 1], c = F[3 * p + 2];
    tris[3 * l] = make_float4(V[3 * a], V[3 * a + 1], V[3 * a + 2], __int_as_float(p));
    tris[3 * l + 1] = make_float4(V[3 * b], V[3 * b + 1], V[3 * b + 2], 0.0f);
    tris[3 * l + 2] = make_float4(V[3 * c], V[3 * c + 1], V[3 * c + 2], 0.0f);
    const float* uv = UV + 6 * (size_t)p;
    tri_uv[2 * l] = make_float4(uv[0], uv[1], uv[2], uv[3]);
    tri_uv[2 * l + 1] = make_float4(uv[4], uv[5], 0.0f, 0.0f);
    if (em) em[l] = make_float4(Le[3 * p], Le[3 * p + 1], Le[3 * p + 2], 0.0f);
    leaf_of_prim[p] = l;
}

// the leaf records' vertices at new positions (original index bits in v0.w kept)
__global__ void k_refit_tris(const float* __restrict__ V, const int* __restrict__ F, const uint32_t* __restrict__ order,
                             int n, float4* __restrict__ tris) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n || order[l] >= (uint32_t)n) return;
    const int p = (int)order[l];
    const int a = F[3 * p], b = F[3 * p + 1], c = F[3 * p + 2];
    tris[3 * l] = make_float4(V[3 * a], V[3 * a + 1], V[3 * a + 2], __int_as_float(p));
    tris[3 * l + 1] = make_float4(V[3 * b], V[3 * b + 1], V[3 * b + 2], 0.0f);
    tris[3 * l + 2] = make_float4(V[3 * c], V[3 * c + 1], V[3 * c + 2], 0.0f);
}

// one thread per 4-wide child slot: the box of the binary node behind it (the union of
// the two child boxes that node stores) or of its leaf triangle; empty slots keep
// their inverted box
__global__ void k_refit_wide(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                             const int* __restrict__ map4, int nnodes4, int nt, float4* __restrict__ nodes4) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * nnodes4) return;
    const int w = k >> 2, j = k & 3;
    const int ref = map4[k];
    if (ref == INT_MIN) return;
    float b[6];
    if (ref >= 0) {
        if (ref >= nt - 1) return;
        const float4 n0 = nodes[4 * ref], n1 = nodes[4 * ref + 1], n2 = nodes[4 * ref + 2];
        const float c0[6] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y}, c1[6] = {n1.z, n1.w, n2.x, n2.y, n2.z, n2.w};
        for (int q = 0; q < 3; ++q) {
            b[q] = fminf(c0[q], c1[q]);
            b[3 + q] = fmaxf(c0[3 + q], c1[3 + q]);
        }
    } else {
        const int l = ~ref;
        if (l >= nt) return;
        const float4 a = tris[3 * l], c = tris[3 * l + 1], e = tris[3 * l + 2];
        const float x[3] = {a.x, c.x, e.x}, y[3] = {a.y, c.y, e.y}, z[3] = {a.z, c.z, e.z};
        b[0] = fminf(x[0], fminf(x[1], x[2]));
        b[1] = fminf(y[0], fminf(y[1], y[2]));
        b[2] = fminf(z[0], fminf(z[1], z[2]));
        b[3] = fmaxf(x[0], fmaxf(x[1], x[2]));
        b[4] = fmaxf(y[0], fmaxf(y[1], y[2]));
        b[5] = fmaxf(z[0], fmaxf(z[1], z[2]));
    }
    float* o = reinterpret_cast<float*>(nodes4 + 8 * (size_t)w);
    for (int a = 0; a < 6; ++a) o[4 * a + j] = b[a];
}

// ---------------------------------------------------------------- host side
static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t build_leaf_records(hipStream_t st, const BvhInputs& in, const uint32_t* order, BvhOutputs& out) {
    const int n = in.nt;
    out.order = order;
    hipLaunchKernelGGL(k_leaf_records, dim3(grid_of(n, 256)), dim3(256), 0, st, in.V, in.F, in.UV, in.Le, order, n,
                       out.tris, out.tri_uv, out.emission, out.leaf_of_prim);
    return hipGetLastError();
}

hipError_t refit_bvh(hipStream_t st, const RefitArgs& a) {
    const int n = a.nt;
    if (n == 1) {
        hipLaunchKernelGGL(k_single_node, dim3(1), dim3(1), 0, st, a.V, a.F, a.nodes);
    } else {
        hipLaunchKernelGGL(k_bounds, dim3(grid_of(n, 256)), dim3(256), 0, st, a.V, a.F, a.order, n, a.child,
                           a.parent_int, a.parent_leaf, a.flags, a.node_box, a.nodes);
    }
    hipLaunchKernelGGL(k_refit_tris, dim3(grid_of(n, 256)), dim3(256), 0, st, a.V, a.F, a.order, n, a.tris);
    if (a.nodes4 && a.nnodes4 > 0)
        hipLaunchKernelGGL(k_refit_wide, dim3(grid_of(4 * (int64_t)a.nnodes4, 256)), dim3(256), 0, st, a.nodes, a.tris,
                           a.map4, a.nnodes4, n, a.nodes4);
    return hipGetLastError();
}

hipError_t build_bvh(hipStream_t st, const BvhInputs& in, BvhOutputs& out, BvhBuild kind, void* scratch,
                     uint64_t* host_word) {
    const int n = in.nt;
    if (kind == BvhBuild::SAH && n > 1) {
        const uint32_t* order = nullptr;
        const hipError_t e = build_sah(st, in, scratch, host_word, out.nodes, &order);
        if (e != hipSuccess) return e;
        out.order = order;
        return build_leaf_records(st, in, order, out);
    }
    const int ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    hipLaunchKernelGGL(k_morton, dim3(grid_of(n, 256)), dim3(256), 0, st, in.V, in.F, n, in.lo[0], in.lo[1],
                       in.lo[2], in.scale[0], in.scale[1], in.scale[2], in.keys[0], in.vals[0]);
    int cur = 0;
    for (int shift = 0; shift < 30; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(SORT_THREADS), 0, st, in.keys[cur], n, shift, in.hist,
                           ntiles);
        hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, st, in.hist, 256 * ntiles);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(SORT_THREADS), 0, st, in.keys[cur], in.vals[cur],
                           in.keys[cur ^ 1], in.vals[cur ^ 1], n, shift, in.hist, ntiles);
        cur ^= 1;
    }
    const uint32_t* codes = in.keys[cur];
    const uint32_t* order = in.vals[cur];
    out.order = order;
    if (n == 1) {
        hipLaunchKernelGGL(k_single_node, dim3(1), dim3(1), 0, st, in.V, in.F, out.nodes);
    } else if (kind == BvhBuild::PLOC) {
        const hipError_t e = build_ploc(st, in, order, scratch, host_word, out.nodes);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_hierarchy, dim3(grid_of(n - 1, 256)), dim3(256), 0, st, codes, n, in.child,
                           in.parent_int, in.parent_leaf);
        hipLaunchKernelGGL(k_bounds, dim3(grid_of(n, 256)), dim3(256), 0, st, in.V, in.F, order, n, in.child,
                           in.parent_int, in.parent_leaf, in.flags, in.node_box, out.nodes);
    }
    hipLaunchKernelGGL(k_leaf_records, dim3(grid_of(n, 256)), dim3(256), 0, st, in.V, in.F, in.UV, in.Le, order, n,
                       out.tris, out.tri_uv, out.emission, out.leaf_of_prim);
    return hipGetLastError();
}

}  // namespace dpcs
