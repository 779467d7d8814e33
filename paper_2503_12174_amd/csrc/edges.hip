// edges.hip -- the camera-pose gradient's boundary part (Sec. 3.2: R_c and t_c are in
// theta and refined with it).
//
// A pixel is the integral of the sample radiance over its unit square of image
// coordinates x = (K X)_{1,2} / (K X)_3, X = R_c P + t_c (the uniform jitter of the camera
// samples, Eq. 6).  Where the radiance jumps along a curve of the image, moving the camera
// moves the curve: d I_p / d theta gains the line integral of (f- - f+) (n . dx/dtheta)
// over the curve's part inside the pixel, n the unit normal toward the f+ side.  The curves
// are the images of the mesh edges across which the first surface seen changes
// discontinuously -- vertices of triangles at one position being one vertex, faces of no
// area left out --: edges of
// one face or of three or more, edges whose faces are not coplanar (creases, and every
// silhouette), coplanar faces folded onto one side, texture-coordinate and emission seams.
// Shadow and projector-frustum boundaries on the surfaces are not among them.
//
// Each taken edge, clipped to w >= tmin in front of the camera and to the image, gets
// n_e = ceil(density * l_e) stratified points (l_e its image length in pixels): point k at
// (k + u) / n_e along the clipped segment, weight l_e / n_e.  f-, f+ are the sample
// radiances (clipped like the forward's samples) of two full paths through x -/+ EDGE_EPS n
// that share the point's random numbers; the forward's own wavefront kernels trace them.
// Points are numbered over the edges in order of (lower, higher welded vertex index); point
// k draws from counter (k, 0, block, 0) under the key seed ^ EDGE_KEY, u being the first
// uniform of block 0.  The speed of the edge point P (fixed on the mesh) in the image is
// dx/dR_ij = c_i P_j, dx/dt_i = c_i with c_i = (K_{.i} - x K_{3i}) / w.
//
// The edge table is built on the host from the device's triangle records on first use
// (sorting 3 T (vertex, vertex, face) keys) and again after a refit.
#include <algorithm>
#include <cmath>
#include <vector>

#include "prefix.hpp"
#include "runtime.hpp"
#include "shade.hpp"

namespace dpcs {

constexpr double EDGE_EPS = 1e-2;                        // side points, pixels from the edge
constexpr uint64_t EDGE_KEY = 0x9E3779B97F4A7C15ull;     // XORed into the seed of edge paths
constexpr int EDGE_GRAD_TB = 128;

struct EdgeArgs {
    const int4* edges;     // (leaf0, leaf1, corners a0 | b0 << 2 | a1 << 4 | b1 << 6, faces)
    int64_t n_edges;
    uint32_t* cnt;         // points per edge
    uint64_t* off;         // exclusive prefix of cnt
    uint64_t* bsum;        // per-workgroup totals of the count pass, then their prefix
    uint64_t* total;
    double K[9];
    double density;
    uint64_t k0;           // this wave's first point
    uint32_t m;            // points in this wave
    uint32_t seed_lo, seed_hi;   // the edge paths' key
    const float4* pix_dE;  // per-pixel cotangent of the clipped pixel mean (rgb, -)
    float* part;           // per-workgroup partials of the 12 pose entries
};

__device__ __forceinline__ D3 corner_pos(const ReqDesc& r, int leaf, int k) {
    const float4 v = r.tris[3 * leaf + k];
    return d3(v.x, v.y, v.z);
}
__device__ __forceinline__ float2 corner_uv(const ReqDesc& r, int leaf, int k) {
    const float4 a = r.tri_uv[2 * leaf], b = r.tri_uv[2 * leaf + 1];
    return k == 0 ? make_float2(a.x, a.y) : k == 1 ? make_float2(a.z, a.w) : make_float2(b.x, b.y);
}

// the edge's end points, and whether the first surface seen jumps across its image
__device__ bool edge_taken(const ReqDesc& r, int4 e, D3& A, D3& B) {
    const int a0 = e.z & 3, b0 = (e.z >> 2) & 3, a1 = (e.z >> 4) & 3, b1 = (e.z >> 6) & 3;
    A = corner_pos(r, e.x, a0);
    B = corner_pos(r, e.x, b0);
    if (e.w != 2) return true;
    const D3 C0 = corner_pos(r, e.x, 3 - a0 - b0), C1 = corner_pos(r, e.y, 3 - a1 - b1);
    const D3 n0 = normalize(cross(B - A, C0 - A)), n1 = normalize(cross(B - A, C1 - A));
    const D3 x = cross(n0, n1);
    if (sqrt(dot(x, x)) > 1e-9) return true;
    if (dot(C0 - A, C1 - A) - dot(C0 - A, B - A) * dot(C1 - A, B - A) / dot(B - A, B - A) > 0) return true;
    const float2 ua0 = corner_uv(r, e.x, a0), ua1 = corner_uv(r, e.y, a1);
    const float2 ub0 = corner_uv(r, e.x, b0), ub1 = corner_uv(r, e.y, b1);
    if (ua0.x != ua1.x || ua0.y != ua1.y || ub0.x != ub1.x || ub0.y != ub1.y) return true;
    if (r.emission) {
        const float4 l0 = r.emission[e.x], l1 = r.emission[e.y];
        if (l0.x != l1.x || l0.y != l1.y || l0.z != l1.z) return true;
    }
    return false;
}

__device__ __forceinline__ D3 homog(const ReqDesc& r, const double* K, D3 P) {
    return mat3(K, mat3(r.cam_R, P) + d3(r.cam_t[0], r.cam_t[1], r.cam_t[2]));
}

// the edge's image clipped to w >= tmin and to the image: 3D ends A1, B1 with depths wA,
// wB, image segment a + lambda d kept for lambda in [l0, l1]
struct EdgeGeo {
    D3 A1, B1;
    double wA, wB, ax, ay, dx, dy, l0, l1, len;
};

__device__ bool edge_clip(const ReqDesc& r, const double* K, D3 A, D3 B, EdgeGeo& g) {
    const D3 hA = homog(r, K, A), hB = homog(r, K, B);
    const double wmin = r.tmin;
    double s0 = 0.0, s1 = 1.0;
    if (hA.z < wmin && hB.z < wmin) return false;
    if (hA.z < wmin) s0 = (wmin - hA.z) / (hB.z - hA.z);
    if (hB.z < wmin) s1 = (wmin - hA.z) / (hB.z - hA.z);
    g.A1 = A + (B - A) * s0;
    g.B1 = A + (B - A) * s1;
    const D3 gA = hA + (hB - hA) * s0, gB = hA + (hB - hA) * s1;
    g.wA = gA.z;
    g.wB = gB.z;
    g.ax = gA.x / gA.z;
    g.ay = gA.y / gA.z;
    g.dx = gB.x / gB.z - g.ax;
    g.dy = gB.y / gB.z - g.ay;
    const double p[4] = {-g.dx, g.dx, -g.dy, g.dy};
    const double q[4] = {g.ax, (double)r.Wc - g.ax, g.ay, (double)r.Hc - g.ay};
    double l0 = 0.0, l1 = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (p[k] == 0.0) {
            if (q[k] < 0.0) return false;
        } else {
            const double t = q[k] / p[k];
            if (p[k] < 0.0) l0 = fmax(l0, t);
            else l1 = fmin(l1, t);
        }
    }
    if (!(l0 < l1)) return false;
    g.l0 = l0;
    g.l1 = l1;
    g.len = (l1 - l0) * sqrt(g.dx * g.dx + g.dy * g.dy);
    return g.len > 0.0;
}

// one thread per edge: its point count, and the workgroup-local exclusive prefix
__global__ void __launch_bounds__(SCAN_TB) k_edge_count(ReqDesc r, EdgeArgs a) {
    __shared__ uint64_t wsum[SCAN_TB / 64];
    const int64_t e = (int64_t)blockIdx.x * SCAN_TB + threadIdx.x;
    uint64_t n = 0;
    if (e < a.n_edges) {
        D3 A, B;
        EdgeGeo g;
        if (edge_taken(r, a.edges[e], A, B) && edge_clip(r, a.K, A, B, g)) n = (uint64_t)ceil(a.density * g.len);
    }
    uint64_t tot;
    const uint64_t loc = block_exclusive(n, wsum, &tot);
    if (e < a.n_edges) {
        a.cnt[e] = (uint32_t)n;
        a.off[e] = loc;
    }
    if (threadIdx.x == 0) a.bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_TB) k_edge_offsets(EdgeArgs a) {
    const int64_t e = (int64_t)blockIdx.x * SCAN_TB + threadIdx.x;
    if (e < a.n_edges) a.off[e] += a.bsum[blockIdx.x];
}

// point k of the wave: its edge, image position, unit normal, 3D point and weight
struct EdgePoint {
    double x, y, nx, ny, w;
    D3 P;
};

__device__ bool edge_point(const ReqDesc& r, const EdgeArgs& a, uint64_t k, EdgePoint& pt) {
    // the last edge whose offset is <= k (edges without points share their successor's)
    int64_t lo = 0, hi = a.n_edges - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (a.off[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t n = a.cnt[lo];
    const uint64_t kk = k - a.off[lo];
    D3 A, B;
    EdgeGeo g;
    if (n == 0 || kk >= n || !edge_taken(r, a.edges[lo], A, B) || !edge_clip(r, a.K, A, B, g)) return false;
    const U4 x = philox4x32_10((uint32_t)k, 0u, 0u, 0u, a.seed_lo, a.seed_hi);
    const double lam = g.l0 + (g.l1 - g.l0) * ((double)kk + u24(x.x)) / (double)n;
    pt.x = g.ax + lam * g.dx;
    pt.y = g.ay + lam * g.dy;
    const double el = sqrt(g.dx * g.dx + g.dy * g.dy);
    pt.nx = -g.dy / el;
    pt.ny = g.dx / el;
    const double mu = lam * g.wA / (lam * g.wA + (1.0 - lam) * g.wB);
    pt.P = g.A1 + (g.B1 - g.A1) * mu;
    pt.w = g.len / (double)n;
    return true;
}

// camera rays through the points' side positions (side 0: x - eps n, 1: x + eps n)
__global__ void k_edge_raygen(Queues q, ReqDesc r, EdgeArgs a, int side) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m) return;
    const uint64_t k = a.k0 + i;
    EdgePoint pt;
    D3 dir = d3(0.0, 0.0, 1.0);
    if (edge_point(r, a, k, pt)) {
        const double s = side ? EDGE_EPS : -EDGE_EPS;
        dir = normalize(mat3(r.cam_M, d3(pt.x + s * pt.nx, pt.y + s * pt.ny, 1.0)));
    }
    q.po[0][i] = PathO{r.cam_o[0], r.cam_o[1], r.cam_o[2], 0, -1};
    q.pd[0][i] = PathD{dir.x, dir.y, dir.z, (uint32_t)k, 0u};
    q.pb[0][i] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    q.L[i + (side ? a.m : 0u)] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// jump x normal speed x weight of every point, per-workgroup partial sums of the 12 entries
__global__ void __launch_bounds__(EDGE_GRAD_TB) k_edge_grad(Queues q, ReqDesc r, EdgeArgs a) {
    double acc[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[j] = 0.0;
    const uint32_t i = blockIdx.x * EDGE_GRAD_TB + threadIdx.x;
    EdgePoint pt;
    if (i < a.m && edge_point(r, a, a.k0 + i, pt)) {
        const int pi = min(max((int)floor(pt.x), 0), r.Wc - 1), pj = min(max((int)floor(pt.y), 0), r.Hc - 1);
        const float4 g = a.pix_dE[(size_t)pj * r.Wc + pi];
        const float4 Lm = q.L[i], Lp = q.L[a.m + i];
        float fm[3] = {Lm.x, Lm.y, Lm.z}, fp[3] = {Lp.x, Lp.y, Lp.z};
        if (r.clip) {
            const float thr = clip_threshold(r);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (fm[c] > thr) fm[c] = thr;
                if (fp[c] > thr) fp[c] = thr;
            }
        }
        const double J = ((double)g.x * ((double)fm[0] - fp[0]) + (double)g.y * ((double)fm[1] - fp[1]) +
                          (double)g.z * ((double)fm[2] - fp[2])) * pt.w;
        const D3 h = homog(r, a.K, pt.P);
        const double Pj[3] = {pt.P.x, pt.P.y, pt.P.z};
#pragma unroll
        for (int ri = 0; ri < 3; ++ri) {
            const double cx = (a.K[ri] - pt.x * a.K[6 + ri]) / h.z, cy = (a.K[3 + ri] - pt.y * a.K[6 + ri]) / h.z;
            const double s = J * (pt.nx * cx + pt.ny * cy);
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[3 * ri + j] = s * Pj[j];
            acc[9 + ri] = s;
        }
    }
    __shared__ double red[12][EDGE_GRAD_TB / 64];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        double v = acc[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0) red[j][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        double v = 0.0;
        for (int w = 0; w < EDGE_GRAD_TB / 64; ++w) v += red[threadIdx.x][w];
        a.part[12 * (size_t)blockIdx.x + threadIdx.x] = (float)v;
    }
}

// ---------------------------------------------------------------- host
namespace {

// the welded edge table from the device's triangle records
bool build_edges(dpcs_context ctx, dpcs_scene sc, dpcs_status* st) {
    const int nt = sc->nt;
    std::vector<int32_t> F(3 * (size_t)nt), leaf(nt);
    std::vector<float4> tris(3 * (size_t)nt);
    if (!hip_ok(ctx, hipMemcpyAsync(F.data(), sc->F, sizeof(int32_t) * F.size(), hipMemcpyDeviceToHost, ctx->stream),
                "edge table: indices") ||
        !hip_ok(ctx, hipMemcpyAsync(leaf.data(), sc->leaf_of_prim, sizeof(int32_t) * nt, hipMemcpyDeviceToHost,
                                    ctx->stream), "edge table: leaf order") ||
        !hip_ok(ctx, hipMemcpyAsync(tris.data(), sc->tris, sizeof(float4) * tris.size(), hipMemcpyDeviceToHost,
                                    ctx->stream), "edge table: triangles") ||
        !hip_ok(ctx, hipStreamSynchronize(ctx->stream), "edge table")) {
        *st = DPCS_E_DEVICE;
        return false;
    }
    // positions of the vertices the triangles use (their records were written from them)
    const int nv = sc->nv;
    std::vector<float> pos(3 * (size_t)nv, 0.0f);
    std::vector<char> used(nv, 0);
    for (int f = 0; f < nt; ++f)
        for (int k = 0; k < 3; ++k) {
            const int v = F[3 * (size_t)f + k];
            const float4 p = tris[3 * (size_t)leaf[f] + k];
            used[v] = 1;
            pos[3 * (size_t)v] = p.x;
            pos[3 * (size_t)v + 1] = p.y;
            pos[3 * (size_t)v + 2] = p.z;
        }
    // weld: the lowest used index at each position
    std::vector<int32_t> ids, canon(nv);
    for (int v = 0; v < nv; ++v) {
        canon[v] = v;
        if (used[v]) ids.push_back(v);
    }
    auto pless = [&](int32_t i, int32_t j) {
        for (int k = 0; k < 3; ++k) {
            const float a = pos[3 * (size_t)i + k], b = pos[3 * (size_t)j + k];
            if (a != b) return a < b;
        }
        return i < j;
    };
    std::sort(ids.begin(), ids.end(), pless);
    for (size_t i = 1; i < ids.size(); ++i) {
        const float* p = &pos[3 * (size_t)ids[i]];
        const float* q = &pos[3 * (size_t)ids[i - 1]];
        if (p[0] == q[0] && p[1] == q[1] && p[2] == q[2]) canon[ids[i]] = canon[ids[i - 1]];
    }
    // (lower, higher, face) per triangle side, sorted; runs are the edges
    struct Key {
        int32_t a, b, f;
    };
    // faces of no area are never seen and bound nothing (the cross product of float
    // differences is exact in double, so the test is exact)
    std::vector<Key> key;
    key.reserve(3 * (size_t)nt);
    for (int f = 0; f < nt; ++f) {
        const float4* t = &tris[3 * (size_t)leaf[f]];
        const double ax = (double)t[1].x - t[0].x, ay = (double)t[1].y - t[0].y, az = (double)t[1].z - t[0].z;
        const double bx = (double)t[2].x - t[0].x, by = (double)t[2].y - t[0].y, bz = (double)t[2].z - t[0].z;
        if (ay * bz - az * by == 0.0 && az * bx - ax * bz == 0.0 && ax * by - ay * bx == 0.0) continue;
        for (int k = 0; k < 3; ++k) {
            const int32_t u = canon[F[3 * (size_t)f + k]], v = canon[F[3 * (size_t)f + (k + 1) % 3]];
            key.push_back(Key{std::min(u, v), std::max(u, v), f});
        }
    }
    std::sort(key.begin(), key.end(), [](const Key& x, const Key& y) {
        return x.a != y.a ? x.a < y.a : x.b != y.b ? x.b < y.b : x.f < y.f;
    });
    auto corner = [&](int f, int32_t v) {
        for (int k = 0; k < 3; ++k)
            if (canon[F[3 * (size_t)f + k]] == v) return k;
        return 0;
    };
    std::vector<int4> E;
    E.reserve(key.size() / 2 + 1);
    for (size_t i = 0; i < key.size();) {
        size_t j = i;
        while (j < key.size() && key[j].a == key[i].a && key[j].b == key[i].b) ++j;
        const int f0 = key[i].f, nf = (int)(j - i);
        const int f1 = nf > 1 ? key[i + 1].f : f0;
        const int cs = corner(f0, key[i].a) | corner(f0, key[i].b) << 2 | corner(f1, key[i].a) << 4 |
                       corner(f1, key[i].b) << 6;
        E.push_back(make_int4(leaf[f0], nf > 1 ? leaf[f1] : -1, cs, nf));
        i = j;
    }
    if (sc->edges) (void)hipFree(sc->edges);
    sc->edges = nullptr;
    sc->n_edges = (int64_t)E.size();
    if (hipMalloc((void**)&sc->edges, sizeof(int4) * std::max<size_t>(E.size(), 1)) != hipSuccess) {
        (void)hipGetLastError();
        *st = fail(ctx, DPCS_E_OOM, "edge table");
        return false;
    }
    if (!hip_ok(ctx, hipMemcpy(sc->edges, E.data(), sizeof(int4) * E.size(), hipMemcpyHostToDevice), "edge table")) {
        *st = DPCS_E_DEVICE;
        return false;
    }
    sc->edges_valid = true;
    return true;
}

}  // namespace

dpcs_status camera_edge_term(dpcs_context ctx, dpcs_scene sc, const ReqDesc& r, const Queues& q, double density,
                             const double K[9], const float4* pix_dE, float* dst) {
    dpcs_status st = DPCS_OK;
    if (!sc->edges_valid && !build_edges(ctx, sc, &st)) return st;
    if (sc->n_edges == 0) return DPCS_OK;
    Launch l{ctx->stream, ctx->grid_cap};
    const int64_t ne = sc->n_edges;
    const int nb = (int)((ne + SCAN_TB - 1) / SCAN_TB);
    EdgeArgs a{};
    a.edges = sc->edges;
    a.n_edges = ne;
    a.cnt = (uint32_t*)scratch(ctx, "edge.cnt", sizeof(uint32_t) * ne, &st);
    a.off = (uint64_t*)scratch(ctx, "edge.off", sizeof(uint64_t) * ne, &st);
    a.bsum = (uint64_t*)scratch(ctx, "edge.bsum", sizeof(uint64_t) * (nb + 1), &st);
    if (!a.cnt || !a.off || !a.bsum) return st;
    a.total = a.bsum + nb;
    for (int k = 0; k < 9; ++k) a.K[k] = K[k];
    a.density = density;
    const uint64_t key = ((uint64_t)r.seed_hi << 32 | r.seed_lo) ^ EDGE_KEY;
    a.seed_lo = (uint32_t)key;
    a.seed_hi = (uint32_t)(key >> 32);
    a.pix_dE = pix_dE;
    hipLaunchKernelGGL(k_edge_count, dim3(nb), dim3(SCAN_TB), 0, l.st, r, a);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, l.st, a.bsum, nb, a.total);
    hipLaunchKernelGGL(k_edge_offsets, dim3(nb), dim3(SCAN_TB), 0, l.st, a);
    uint64_t total = 0;
    if (!hip_ok(ctx, hipMemcpyAsync(&total, a.total, sizeof(uint64_t), hipMemcpyDeviceToHost, l.st), "edge count") ||
        !hip_ok(ctx, hipStreamSynchronize(l.st), "edge count"))
        return DPCS_E_DEVICE;
    if (total >= (uint64_t(1) << 32))
        return fail(ctx, DPCS_E_UNSUPPORTED, "camera edge samples exceed 2^32 (lower camera_edge_density)");
    // the edge paths of a wave: both sides' radiance in one queue of 2 m paths; the VJP's
    // queues when they hold every point, else queues sized for them
    Queues qe = q;
    const int64_t want = (int64_t)std::min<uint64_t>(2 * total, (uint64_t)std::max<int64_t>(ctx->capacity, 2));
    if (want > q.cap && !make_queues(ctx, "edge.queues", want, qe, &st)) return st;
    const int64_t m_max = qe.cap / 2;
    const int64_t nbg_max = (m_max + EDGE_GRAD_TB - 1) / EDGE_GRAD_TB;
    a.part = (float*)scratch(ctx, "edge.partials", sizeof(float) * 12 * nbg_max, &st);
    if (!a.part) return st;
    // as in the forward: a depth's shadow rays on the side stream beside the next depth's
    // closest hit, shading and the gradient kernel waiting for them
    int* spill2 = ctx->prof_mode ? nullptr : side_spill(ctx, qe);
    const bool sidestream = spill2 && std::min<int64_t>(m_max, (int64_t)total) >= SIDE_MIN_PATHS && side_stream(ctx);
    Queues qs = qe;
    qs.spill = spill2;
    const Launch ls{ctx->side, ctx->grid_cap};
    for (uint64_t k0 = 0; k0 < total; k0 += (uint64_t)m_max) {
        const uint32_t m = (uint32_t)std::min<uint64_t>((uint64_t)m_max, total - k0);
        a.k0 = k0;
        a.m = m;
        for (int side = 0; side < 2; ++side) {
            // the edge paths: one sample per path, their own key, results at [side m, side m + m)
            ReqDesc re = r;
            re.seed_lo = a.seed_lo;
            re.seed_hi = a.seed_hi;
            re.sample_offset = 0;
            re.spp = 1;
            re.g_base = (uint32_t)k0;
            re.sid_base = side ? m : 0u;
            re.rec = nullptr;
            re.out_hits = nullptr;
            re.out_L = nullptr;
            re.out_image = nullptr;
            re.out_linear = nullptr;
            re.d_cam_part = nullptr;
            launch_set_count(l, qe.cnt, 0, m, 1, 4);
            hipLaunchKernelGGL(k_edge_raygen, dim3((m + 255) / 256), dim3(256), 0, l.st, qe, re, a, side);
            int cur = 0;
            for (int d = 0; d < re.max_depth; ++d) {
                launch_trace(l, qe, cur, re, nullptr, m);   // (empties the queues shading appends to)
                if (sidestream && d > 0) (void)hipStreamWaitEvent(l.st, ctx->ev_shadow, 0);
                launch_shade(l, qe, cur, d, re, nullptr, m);
                if (sidestream) {
                    (void)hipEventRecord(ctx->ev_shade, l.st);
                    (void)hipStreamWaitEvent(ctx->side, ctx->ev_shade, 0);
                    for (int w = 0; w < (re.env_on ? 2 : 1); ++w) launch_shadow(ls, qs, w, re, nullptr, m, d);
                    (void)hipEventRecord(ctx->ev_shadow, ctx->side);
                } else {
                    for (int w = 0; w < (re.env_on ? 2 : 1); ++w) launch_shadow(l, qe, w, re, nullptr, m, d);
                }
                cur ^= 1;
            }
            if (sidestream) (void)hipStreamWaitEvent(l.st, ctx->ev_shadow, 0);
        }
        const unsigned nbg = (m + EDGE_GRAD_TB - 1) / EDGE_GRAD_TB;
        hipLaunchKernelGGL(k_edge_grad, dim3(nbg), dim3(EDGE_GRAD_TB), 0, l.st, qe, r, a);
        launch_sum_partials(l, a.part, (int)nbg, 12, 12, dst);
    }
    if (hipGetLastError() != hipSuccess) return fail(ctx, DPCS_E_DEVICE, "camera edge term launch failed");
    return DPCS_OK;
}

}  // namespace dpcs
