// shade.hpp -- per-vertex shading steps shared by the forward kernels and the
// path-replay adjoint (the replay must reproduce the forward path exactly, so both
// call these same routines).
#pragma once

#include "common.hpp"
#include "trace.hpp"

namespace dpcs {

template <bool UNI>
__device__ __forceinline__ const ReqDesc& sel(const ReqDesc& uni, const ReqDesc* __restrict__ table, int slot) {
    return UNI ? uni : table[slot];
}

// wave-aggregated append: one atomic per wave64, lane order preserved
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return 0u;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// workgroup-aggregated append to NQ queues: one atomic per queue per workgroup
// (instead of one per wave), lane order preserved within each wave.  Every thread of
// the workgroup (NT threads) must call it, with its predicates; idx[q] is the slot of
// a thread whose pred[q] holds.
template <int NQ, int NT = BLOCK>
__device__ __forceinline__ void block_append(const bool* pred, uint32_t* const* counter, uint32_t* idx) {
    constexpr int NW = NT / 64;
    __shared__ uint32_t wcount[NQ][NW];
    __shared__ uint32_t wbase[NQ][NW];
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long m[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        m[q] = __ballot(pred[q]);
        if (lane == 0) wcount[q][wv] = (uint32_t)__popcll(m[q]);
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int q = threadIdx.x;
        uint32_t total = 0;
        for (int w = 0; w < NW; ++w) total += wcount[q][w];
        uint32_t run = total ? atomicAdd(counter[q], total) : 0u;
        for (int w = 0; w < NW; ++w) {
            wbase[q][w] = run;
            run += wcount[q][w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) idx[q] = wbase[q][wv] + (uint32_t)__popcll(m[q] & below);
}

// block_append whose entries of one workgroup are grouped by a key in [0, NK) (key
// order, then wave and lane order): rays appended with their direction octant as key
// leave the workgroup as runs of like-signed directions, so the waves that trace them
// next take more similar paths through the BVH.  Still one atomic per queue.
template <int NQ, int NK, int NT = BLOCK>
__device__ __forceinline__ void block_append_keyed(const bool* pred, const int* key, uint32_t* const* counter,
                                                   uint32_t* idx) {
    constexpr int NW = NT / 64;
    __shared__ uint32_t wcount[NQ][NK][NW];
    __shared__ uint32_t wbase[NQ][NK][NW];
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long mine[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        mine[q] = 0ull;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const unsigned long long m = __ballot(pred[q] && key[q] == k);
            if (lane == 0) wcount[q][k][wv] = (uint32_t)__popcll(m);
            if (key[q] == k) mine[q] = m;
        }
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int q = threadIdx.x;
        uint32_t total = 0;
        for (int k = 0; k < NK; ++k)
            for (int w = 0; w < NW; ++w) total += wcount[q][k][w];
        uint32_t run = total ? atomicAdd(counter[q], total) : 0u;
        for (int k = 0; k < NK; ++k)
            for (int w = 0; w < NW; ++w) {
                wbase[q][k][w] = run;
                run += wcount[q][k][w];
            }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) idx[q] = wbase[q][key[q]][wv] + (uint32_t)__popcll(mine[q] & below);
}

// octant of a direction (sign bits of x, y, z)
__device__ __forceinline__ int octant(double x, double y, double z) {
    return (x < 0.0 ? 1 : 0) | (y < 0.0 ? 2 : 0) | (z < 0.0 ? 4 : 0);
}

// camera ray of global sample g (pixel = g / spp, sample = g % spp), Eq. 6 inverted
__device__ __forceinline__ D3 camera_dir(const ReqDesc& r, uint32_t g) {
    const uint32_t pixel = g / (uint32_t)r.spp, s = g - pixel * (uint32_t)r.spp;
    const U4 x = philox4x32_10(pixel, s + r.sample_offset, 0u, 0u, r.seed_lo, r.seed_hi);
    const double px = (double)(pixel % (uint32_t)r.Wc) + u24(x.x);
    const double py = (double)(pixel / (uint32_t)r.Wc) + u24(x.y);
    return normalize(mat3(r.cam_M, d3(px, py, 1.0)));
}

struct Surf {
    D3 x, n, wo;
    double u, v;     // texture coordinates
    int prim;
    Bilin tb;
    D3 alb;
    double rough, spec;
};

// The normal map's shading frame and the metallic value at a hit (requests with tex4b):
// T along dP/du of the triangle's texture parameterisation, orthogonal to the two-sided
// geometric normal n (the Duff et al. basis when the parameterisation is degenerate),
// B = n x T; the map value v decodes to t = 2 v - 1 and ns = (t_x T + t_y B + t_z n) / |t|
// (n itself when t = 0).  th = t / |t|, tlen = |t| for the chain rule back to v.
struct Shading {
    D3 ns, T, B, th;
    double tlen, metal;
};
__device__ __forceinline__ Shading shading(const ReqDesc& r, int leaf, const Surf& s) {
    Shading h;
    V3 f0, f1, f2;
    int prim;
    load_tri(r.tris, leaf, f0, f1, f2, prim);
    const D3 e1 = to_d(f1) - to_d(f0), e2 = to_d(f2) - to_d(f0);
    const float4 ua = r.tri_uv[2 * leaf], ub = r.tri_uv[2 * leaf + 1];
    const double du1 = (double)ua.z - ua.x, dv1 = (double)ua.w - ua.y;
    const double du2 = (double)ub.x - ua.x, dv2 = (double)ub.y - ua.y;
    const double det = du1 * dv2 - du2 * dv1;
    D3 t = d3(0., 0., 0.);
    if (det != 0.0) {
        const D3 dpdu = (e1 * dv2 - e2 * dv1) * (1.0 / det);
        t = dpdu - s.n * dot(s.n, dpdu);
    }
    const double tl = sqrt(dot(t, t));
    if (tl > 0.0) {
        h.T = t * (1.0 / tl);
    } else {   // first axis of the Duff et al. basis of n
        const double sg = copysign(1.0, s.n.z);
        const double a = -1.0 / (sg + s.n.z);
        h.T = d3(1.0 + sg * s.n.x * s.n.x * a, sg * s.n.x * s.n.y * a, -sg * s.n.x);
    }
    h.B = cross(s.n, h.T);
    const D4 m = fetch4(r.tex4b, s.tb);
    h.metal = r.brdf ? m.w : 0.0;
    const D3 tv = d3(2.0 * m.x - 1.0, 2.0 * m.y - 1.0, 2.0 * m.z - 1.0);
    h.tlen = sqrt(dot(tv, tv));
    if (h.tlen > 0.0) {
        h.th = tv * (1.0 / h.tlen);
        h.ns = h.T * h.th.x + h.B * h.th.y + s.n * h.th.z;
    } else {
        h.th = d3(0., 0., 1.);
        h.ns = s.n;
    }
    return h;
}
// cotangent of the stored map value v from a cotangent g of ns: ns = F t / |t|, t = 2 v - 1
__device__ __forceinline__ D3 nmap_cotangent(const Shading& h, const D3& n, D3 g) {
    if (!(h.tlen > 0.0)) return d3(0., 0., 0.);
    const D3 gl = d3(dot(h.T, g), dot(h.B, g), dot(n, g));
    const D3 gt = (gl - h.th * dot(h.th, gl)) * (1.0 / h.tlen);
    return gt * 2.0;
}

// Hit attributes of the ray (o, d) on the leaf the FP32 traversal found: barycentrics
// re-solved in FP64 (Cramer's rule on o + t d = v0 + b1 e1 + b2 e2), flat two-sided
// normal facing the incoming ray, bilinear BRDF maps at the interpolated UV.
// the surface at a hit without its maps: point, two-sided normal, texture coordinates
// and the bilinear corners of the maps (surface_maps reads them)
__device__ __forceinline__ Surf surface_geo(const ReqDesc& r, int leaf, D3 o, D3 d) {
    Surf s;
    V3 f0, f1, f2;
    load_tri(r.tris, leaf, f0, f1, f2, s.prim);
    // the corner texture coordinates load with the vertices (both need only the leaf): read
    // after the barycentrics, they cost a second trip to memory
    const float4 ua = r.tri_uv[2 * leaf], ub = r.tri_uv[2 * leaf + 1];
    const D3 v0 = to_d(f0), v1 = to_d(f1), v2 = to_d(f2);
    const D3 e1 = v1 - v0, e2 = v2 - v0;
    const D3 p = cross(d, e2);
    const double det = dot(e1, p);
    double b1 = 1.0 / 3.0, b2 = 1.0 / 3.0;
    if (det != 0.0) {
        const double inv = 1.0 / det;
        const D3 tv = o - v0;
        b1 = dot(tv, p) * inv;
        b2 = dot(d, cross(tv, e1)) * inv;
    }
    const double b0 = 1.0 - b1 - b2;
    s.x = v0 * b0 + v1 * b1 + v2 * b2;
    D3 n = normalize(cross(e1, e2));
    s.wo = -d;
    if (dot(n, s.wo) < 0.0) n = -n;
    s.n = n;
    s.u = b0 * ua.x + b1 * ua.z + b2 * ub.x;
    s.v = b0 * ua.y + b1 * ua.w + b2 * ub.y;
    s.tb = bilinear(s.u * r.tw - 0.5, s.v * r.th - 0.5, r.tw, r.th);
    return s;
}
__device__ __forceinline__ void surface_maps(const ReqDesc& r, Surf& s) {
    const D4 t4 = fetch4(r.tex4, s.tb);
    s.alb = d3(t4.x, t4.y, t4.z);
    s.rough = t4.w;
    s.spec = r.brdf ? fetch1(r.spec, s.tb) : 0.0;
}
__device__ __forceinline__ Surf surface(const ReqDesc& r, int leaf, D3 o, D3 d) {
    Surf s = surface_geo(r, leaf, o, d);
    surface_maps(r, s);
    return s;
}

// projector next-event estimation geometry (Eq. 2, 6); false outside the frustum or
// when the projector is behind the surface
struct ProjNee {
    D3 wp;
    double dist, geom;   // (1/cos^3 alpha) cos theta / d^2
    double g0;           // 1 / (cos^3 alpha d^2): geom without the cosine
    double pu, pv;
    Bilin pb;
};
__device__ __forceinline__ bool projector_nee(const ReqDesc& r, const Surf& s, ProjNee& p) {
    const D3 xp = mat3(r.prj_R, s.x) + d3(r.prj_t[0], r.prj_t[1], r.prj_t[2]);
    if (!(xp.z > 0.0)) return false;
    const double iz = 1.0 / xp.z;
    p.pu = (r.prj_K[0] * xp.x + r.prj_K[1] * xp.y + r.prj_K[2] * xp.z) * iz;
    p.pv = (r.prj_K[3] * xp.x + r.prj_K[4] * xp.y + r.prj_K[5] * xp.z) * iz;
    if (!(p.pu >= 0.0 && p.pu < (double)r.Wp && p.pv >= 0.0 && p.pv < (double)r.Hp)) return false;
    const D3 tow = d3(r.prj_o[0], r.prj_o[1], r.prj_o[2]) - s.x;
    p.dist = sqrt(dot(tow, tow));
    p.wp = tow * (1.0 / p.dist);
    const double cp = dot(s.n, p.wp);
    if (!(cp > 0.0)) return false;
    const double ca = xp.z / sqrt(dot(xp, xp));
    p.geom = cp / (ca * ca * ca * p.dist * p.dist);
    p.g0 = 1.0 / (ca * ca * ca * p.dist * p.dist);
    p.pb = bilinear(p.pu - 0.5, p.pv - 0.5, r.Wp, r.Hp);
    return true;
}

__device__ __forceinline__ U4 vertex_rng(const ReqDesc& r, uint32_t g, uint32_t block) {
    const uint32_t pixel = g / (uint32_t)r.spp, s = g - pixel * (uint32_t)r.spp;
    return philox4x32_10(pixel, s + r.sample_offset, block, 0u, r.seed_lo, r.seed_hi);
}

}  // namespace dpcs
