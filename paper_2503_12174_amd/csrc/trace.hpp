// trace.hpp -- ray queries on the device BVH.
//
// BVH2 node (64 B, 4 x float4): both children's boxes inline so one node fetch
// tests two boxes.
//   n0 = (lo0.x, lo0.y, lo0.z, hi0.x)  n1 = (hi0.y, hi0.z, lo1.x, lo1.y)
//   n2 = (lo1.z, hi1.x, hi1.y, hi1.z)  n3 = (child0, child1, -, -) as int bits
// BVH4 node (128 B, one cache line, 8 x float4): the four children's boxes as
// structure of arrays, lo.x[4], lo.y[4], lo.z[4], hi.x[4], hi.y[4], hi.z[4], then the
// four child references and 16 unused bytes.
// child >= 0: internal node index; child < 0: leaf ~child (one triangle, leaf order).
// An unused slot of a BVH4 node holds an inverted box far from the scene, which the
// 4-wide box test never enters, and the dummy leaf nt (one record past the mesh's
// triangles, NaN vertices), which no ray hits, so the loop needs no test for them.
// Triangle record (48 B): v0 (w = original triangle index bits), v1, v2.
//
// Closest hit: smallest t in (tmin, tmax); equal t -> smaller original triangle
// index, so the result equals a brute-force scan in the same arithmetic.  Box tests
// are widened by a few ulps so no triangle a brute-force scan would accept is culled.
#pragma once

#include "common.hpp"

namespace dpcs {

// watertight ray / triangle test (Woop, Benthin, Wald, JCGT 2013)
struct WtRay {
    V3 o;
    uint32_t k;          // axis permutation kx | ky << 2 | kz << 4
    float Sx, Sy, Sz;
};

__device__ __forceinline__ WtRay wt_setup(V3 o, V3 d) {
    WtRay r;
    r.o = o;
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    const float dz = comp(d, kz);
    if (dz < 0.0f) {
        const int tmp = kx;
        kx = ky;
        ky = tmp;
    }
    r.k = (uint32_t)kx | (uint32_t)ky << 2 | (uint32_t)kz << 4;
    // the shear need not be correctly rounded, only the same for every triangle a ray
    // meets (watertightness), so the hardware reciprocal (within 1 ulp) stands in for the
    // multi-instruction IEEE division; |dz| >= 1/sqrt(3) for a unit direction
    r.Sz = __builtin_amdgcn_rcpf(dz);
    r.Sx = comp(d, kx) * r.Sz;
    r.Sy = comp(d, ky) * r.Sz;
    return r;
}

// returns false on a miss; on a hit t and the barycentrics (b1 of v1, b2 of v2)
__device__ __forceinline__ bool wt_intersect(const WtRay& r, V3 v0, V3 v1, V3 v2, float& t, float& b1, float& b2) {
    const int kx = (int)(r.k & 3u), ky = (int)((r.k >> 2) & 3u), kz = (int)(r.k >> 4);
    const V3 A = v0 - r.o, B = v1 - r.o, C = v2 - r.o;
    const float Akz = comp(A, kz), Bkz = comp(B, kz), Ckz = comp(C, kz);
    const float Ax = comp(A, kx) - r.Sx * Akz, Ay = comp(A, ky) - r.Sy * Akz;
    const float Bx = comp(B, kx) - r.Sx * Bkz, By = comp(B, ky) - r.Sy * Bkz;
    const float Cx = comp(C, kx) - r.Sx * Ckz, Cy = comp(C, ky) - r.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {  // edge case: decide in double
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = U + V + W;
    if (det == 0.0f) return false;
    const float T = U * (r.Sz * Akz) + V * (r.Sz * Bkz) + W * (r.Sz * Ckz);
    const float inv = 1.0f / det;
    t = T * inv;
    b1 = V * inv;
    b2 = W * inv;
    return true;
}

// The traversal loops decide hits with this cheaper form of the same test: no
// barycentrics, and t = (Sz T') * rcp(det) with T' = U Akz + V Bkz + W Ckz (the hardware
// reciprocal, not the correctly rounded quotient).  Every query -- BVH or brute force --
// decides with it and then recomputes the reported t and barycentrics of its winner with
// wt_intersect, so all of them agree bit for bit.
__device__ __forceinline__ bool wt_hit(const WtRay& r, V3 v0, V3 v1, V3 v2, float& t) {
    const int kx = (int)(r.k & 3u), ky = (int)((r.k >> 2) & 3u), kz = (int)(r.k >> 4);
    const V3 A = v0 - r.o, B = v1 - r.o, C = v2 - r.o;
    const float Akz = comp(A, kz), Bkz = comp(B, kz), Ckz = comp(C, kz);
    const float Ax = comp(A, kx) - r.Sx * Akz, Ay = comp(A, ky) - r.Sy * Akz;
    const float Bx = comp(B, kx) - r.Sx * Bkz, By = comp(B, ky) - r.Sy * Bkz;
    const float Cx = comp(C, kx) - r.Sx * Ckz, Cy = comp(C, ky) - r.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {  // edge case: decide in double
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = U + V + W;
    if (det == 0.0f) return false;
    const float T = U * Akz + V * Bkz + W * Ckz;
    t = (T * r.Sz) * __builtin_amdgcn_rcpf(det);
    return true;
}

struct Hit {
    float t;
    int leaf;   // leaf-order triangle index, -1 on a miss
    int prim;   // original triangle index
    float b1, b2;
};

struct BoxRay {
    V3 o, inv;
};
// (hardware reciprocals, within 1 ulp: the 4e-6 widening of every slab covers it)
__device__ __forceinline__ BoxRay box_setup(V3 o, V3 d) {
    return BoxRay{o, v3(__builtin_amdgcn_rcpf(d.x), __builtin_amdgcn_rcpf(d.y), __builtin_amdgcn_rcpf(d.z))};
}

// conservative entry distance of the ray into [lo, hi]; returns +inf when missed
__device__ __forceinline__ float box_enter(const BoxRay& r, float lx, float ly, float lz, float hx, float hy, float hz,
                                           float tmin, float tmax) {
    const float tx0 = (lx - r.o.x) * r.inv.x, tx1 = (hx - r.o.x) * r.inv.x;
    const float ty0 = (ly - r.o.y) * r.inv.y, ty1 = (hy - r.o.y) * r.inv.y;
    const float tz0 = (lz - r.o.z) * r.inv.z, tz1 = (hz - r.o.z) * r.inv.z;
    float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
    float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
    // widen by 4e-6 relative (a few ulps of every operation above)
    tn = tn - fabsf(tn) * 4e-6f;
    tf = tf + fabsf(tf) * 4e-6f;
    tn = fmaxf(tn, tmin);
    tf = fminf(tf, tmax);
    return tn <= tf ? tn : __builtin_inff();
}

__device__ __forceinline__ void load_tri(const float4* __restrict__ tris, int leaf, V3& v0, V3& v1, V3& v2, int& prim) {
    const float4 a = tris[3 * leaf], b = tris[3 * leaf + 1], c = tris[3 * leaf + 2];
    v0 = xyz(a);
    v1 = xyz(b);
    v2 = xyz(c);
    prim = __float_as_int(a.w);
}

// Traversal stack of internal node indices: the first SHORT entries live in LDS, entry
// k of lane `lane` at stack[k * TBK + lane] (consecutive lanes on consecutive banks),
// plus one more LDS entry per lane (k = SHORT) that the 4-wide push writes candidates
// it does not keep to;
// deeper entries -- rare with near-child-first order -- go to the workgroup's region of
// global memory with the same interleaving, spill[(k - SHORT) * TBK + lane].  Both
// bases are uniform, so a lane holds only its index.  The host only launches on trees
// whose stack bound is <= 64, so at most 64 entries are ever live.
//
// Node and triangle visit counters for the profiler's counting pass; the timed
// kernels use Visits<false>, which keeps no registers.
template <bool ON>
struct Visits {
    uint32_t nodes = 0, tris = 0;
    __device__ __forceinline__ void node() { ++nodes; }
    __device__ __forceinline__ void tri() { ++tris; }
};
template <>
struct Visits<false> {
    static constexpr uint32_t nodes = 0, tris = 0;
    __device__ __forceinline__ void node() {}
    __device__ __forceinline__ void tri() {}
};

template <bool ANY, int SHORT, int TBK, class VIS>
__device__ __forceinline__ bool traverse(const float4* __restrict__ nodes, const float4* __restrict__ tris, V3 o, V3 d,
                                         float tmin, float tmax, int skip, Hit& h, int* stack, int* spill, int lane,
                                         VIS& vis) {
    const BoxRay br = box_setup(o, d);
    const WtRay wr = wt_setup(o, d);
    float best_t = tmax;
    int best_prim = 0x7fffffff, best_leaf = -1;
    int sp = 0;
    int node = 0;
    while (node >= 0) {   // the only exit (see traverse4)
        vis.node();
        const float4 n0 = nodes[4 * node], n1 = nodes[4 * node + 1], n2 = nodes[4 * node + 2];
        const int4 n3 = *reinterpret_cast<const int4*>(&nodes[4 * node + 3]);
        float t0 = box_enter(br, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tmin, best_t);
        float t1 = box_enter(br, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tmin, best_t);
        const int c0 = n3.x, c1 = n3.y;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int c = k == 0 ? c0 : c1;
            const float tc = k == 0 ? t0 : t1;
            if (c < 0 && tc < __builtin_inff()) {
                const int leaf = ~c;
                V3 v0, v1, v2;
                int prim;
                vis.tri();
                load_tri(tris, leaf, v0, v1, v2, prim);
                float t;
                const bool hit = wt_hit(wr, v0, v1, v2, t);   // the skip test after it (one load)
                if (hit & (prim != skip) & (t > tmin) &&
                    (t < best_t || (t == best_t && best_leaf >= 0 && prim < best_prim))) {
                    best_t = t;
                    best_prim = prim;
                    best_leaf = leaf;
                }
            }
        }
        // a missed box reports +inf, which must not pass while best_t is still +inf
        const bool h0 = c0 >= 0 && t0 < __builtin_inff() && t0 <= best_t;
        const bool h1 = c1 >= 0 && t1 < __builtin_inff() && t1 <= best_t;
        if (ANY && best_leaf >= 0) {   // any hit ends the query
            node = -1;
        } else if (h0 && h1) {
            const bool first0 = t0 <= t1;
            const int far = first0 ? c1 : c0;
            if (sp < SHORT) stack[sp * TBK + lane] = far;
            else if constexpr (SHORT < MAX_STACK) {
                if (sp < MAX_STACK) spill[(sp - SHORT) * TBK + lane] = far;
            }
            sp = sp < MAX_STACK ? sp + 1 : sp;   // depth <= 64 is checked on the host
            node = first0 ? c0 : c1;
        } else if (h0) {
            node = c0;
        } else if (h1) {
            node = c1;
        } else if (sp > 0) {
            --sp;
            node = stack[min(sp, SHORT - 1) * TBK + lane];
            if constexpr (SHORT < MAX_STACK)
                if (sp >= SHORT) node = spill[(sp - SHORT) * TBK + lane];
        } else {
            node = -1;
        }
    }
    float bb1 = 0.f, bb2 = 0.f;
    if (best_leaf >= 0) {   // reported t and barycentrics: the exact test on the winner
        V3 v0, v1, v2;
        int prim;
        load_tri(tris, best_leaf, v0, v1, v2, prim);
        wt_intersect(wr, v0, v1, v2, best_t, bb1, bb2);
    }
    h.t = best_t;
    h.leaf = best_leaf;
    h.prim = best_leaf >= 0 ? best_prim : -1;
    h.b1 = bb1;
    h.b2 = bb2;
    return best_leaf >= 0;
}

// compare-exchange on (key, ref) pairs, smaller key first
__device__ __forceinline__ void cmpx(float& ka, int& ra, float& kb, int& rb) {
    if (kb < ka) {
        const float k = ka;
        ka = kb;
        kb = k;
        const int r = ra;
        ra = rb;
        rb = r;
    }
}

// Ray constants of the 4-wide box tests.  Per axis, the sign of the direction says
// which of a child's two planes the ray meets first, so a node load fetches the near
// and the far coordinates directly (byte offsets below) and each slab takes one FMA,
// plane * (1 / d) + off, with no min/max per axis.  off is -o / d rounded outward:
// down by at least the rounding error of o / d for near planes, up for far planes.
// With that, a slab value can only err by the relative rounding of 1 / d and of the
// FMA, which the relative widening in the test covers; it needs no absolute term
// that would grow for near-axis-parallel rays.  Degenerate axes (d = 0) give NaN or
// infinite slab values, which the min/max below drop or keep in the conservative
// direction.  The relative widening multiplies (t x (1 -+ 4e-6)) rather than adding
// a multiple of |t|, so infinite slab values stay infinite instead of turning NaN,
// and an inverted box (lo = +1e30, hi = -1e30: every near plane ahead of every far
// plane) is always missed.
struct Box4Ray {
    float ix, iy, iz;             // 1 / d
    float anx, any, anz;          // near-plane offsets
    float afx, afy, afz;          // far-plane offsets
    uint32_t onx, ony, onz;       // byte offset of the near coordinate float4 in a node
};
// the far coordinate float4 of each axis sits at the near one's offset XOR these
// (x: 0 <-> 48, y: 16 <-> 64, z: 32 <-> 80)
constexpr uint32_t FAR_X = 48u, FAR_Y = 80u, FAR_Z = 112u;

__device__ __forceinline__ Box4Ray box4_setup(V3 o, V3 d) {
    Box4Ray r;
    // hardware reciprocals (within 1 ulp, +-inf for a zero component like 1 / d)
    r.ix = __builtin_amdgcn_rcpf(d.x);
    r.iy = __builtin_amdgcn_rcpf(d.y);
    r.iz = __builtin_amdgcn_rcpf(d.z);
    // |fl(o rcp(d)) - o / d| <= (2^-23 + 2^-24) |fl(o rcp(d))| (1 + 2^-23); 2^-21 also
    // covers the rounding of the two sums below
    const float px = o.x * r.ix, py = o.y * r.iy, pz = o.z * r.iz;
    const float ex = fabsf(px) * 0x1p-21f, ey = fabsf(py) * 0x1p-21f, ez = fabsf(pz) * 0x1p-21f;
    r.anx = -px - ex;
    r.any = -py - ey;
    r.anz = -pz - ez;
    r.afx = -px + ex;
    r.afy = -py + ey;
    r.afz = -pz + ez;
    // node float4s: 0 lo.x, 1 lo.y, 2 lo.z, 3 hi.x, 4 hi.y, 5 hi.z
    const bool sx = __builtin_signbit(r.ix), sy = __builtin_signbit(r.iy), sz = __builtin_signbit(r.iz);
    r.onx = sx ? 48u : 0u;
    r.ony = sy ? 64u : 16u;
    r.onz = sz ? 80u : 32u;
    return r;
}

// entry distance of the ray into a child box of a node (near / far planes as loaded),
// widened by 4e-6 relative like box_enter; NaN where missed, so a single test
// `t <= bound` both checks the hit and the bound.  (A negative entry or exit is
// scaled the wrong way, which the clamp to tmin > 0 makes irrelevant.)
__device__ __forceinline__ float box4_enter(const Box4Ray& r, float nx, float ny, float nz, float fx, float fy,
                                            float fz, float tmin, float tmax) {
    float tn = fmaxf(fmaxf(fmaf(nx, r.ix, r.anx), fmaf(ny, r.iy, r.any)), fmaf(nz, r.iz, r.anz));
    float tf = fminf(fminf(fmaf(fx, r.ix, r.afx), fmaf(fy, r.iy, r.afy)), fmaf(fz, r.iz, r.afz));
    tn = fmaxf(tn * (1.0f - 4e-6f), tmin);
    tf = fminf(tf * (1.0f + 4e-6f), tmax);
    return tn <= tf ? tn : __builtin_nanf("");
}

// The top of the 4-wide tree in LDS: the collapse numbers nodes breadth first, so nodes
// [0, n) are its top levels; a workgroup copies them once and every ray that passes them
// reads LDS instead of L2.  bytes = 128 n (0: nothing staged).  (The scene only keeps a
// 4-wide tree whose worst-case stack fits MAX_STACK.)
struct TopNodes {
    const float4* lds;
    uint32_t bytes;
};


// all threads of the workgroup call it (it ends with a barrier); n <= TOP_NODES
template <int TBK>
__device__ __forceinline__ TopNodes stage_top(float4* lds, const float4* __restrict__ nodes4, int n) {
    for (int k = threadIdx.x; k < 8 * n; k += TBK) lds[k] = nodes4[k];
    __syncthreads();
    return TopNodes{lds, 128u * (uint32_t)n};
}

// One 4-wide query's state: the ray constants, the best hit so far, the stack depth and
// the next node (-1: the query has ended).
struct Trav4 {
    Box4Ray br;
    WtRay wr;
    float tmin, best_t;
    int skip, best_leaf, sp, node;
};

__device__ __forceinline__ void trav4_start(Trav4& s, V3 o, V3 d, float tmin, float tmax, int skip) {
    s.br = box4_setup(o, d);
    s.wr = wt_setup(o, d);
    s.tmin = tmin;
    s.best_t = tmax;
    s.skip = skip;
    s.best_leaf = -1;
    s.sp = 0;
    s.node = 0;
}

// One node of the query (s.node >= 0): its four box tests, the leaf children hit tested
// at once, the internal children still in range visited nearest first (the others
// pushed, farthest first); s.node becomes the next node, or -1 when the query ends.
template <bool ANY, int SHORT, int TBK, class VIS>
__device__ __forceinline__ void trav4_visit(Trav4& s, const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                            int* stack, int* spill, int lane, VIS& vis, TopNodes top) {
    vis.node();
    // 32-bit byte offsets from the tree's base (the build keeps 128 x nodes < 2^32), so
    // each load is base + one 32-bit register
    const uint32_t nb = (uint32_t)s.node * 128u;
    const uint32_t ax = nb | s.br.onx, ay = nb | s.br.ony, az = nb | s.br.onz;
    float4 nx, ny, nz, fx, fy, fz;
    int4 cr;
    // the empty asm ends the LDS branch differently from the global one: otherwise the
    // compiler sinks the two sets of loads into one generic (flat) load of a selected
    // address, which is slower for the global case
    if (nb < top.bytes) {   // staged top levels: same byte offsets from the LDS copy
        const char* lb = reinterpret_cast<const char*>(top.lds);
        nx = *reinterpret_cast<const float4*>(lb + ax);
        ny = *reinterpret_cast<const float4*>(lb + ay);
        nz = *reinterpret_cast<const float4*>(lb + az);
        fx = *reinterpret_cast<const float4*>(lb + (ax ^ FAR_X));
        fy = *reinterpret_cast<const float4*>(lb + (ay ^ FAR_Y));
        fz = *reinterpret_cast<const float4*>(lb + (az ^ FAR_Z));
        cr = *reinterpret_cast<const int4*>(lb + (nb + 96u));
        asm volatile("");
    } else {
        const char* base = reinterpret_cast<const char*>(nodes);
        nx = *reinterpret_cast<const float4*>(base + ax);
        ny = *reinterpret_cast<const float4*>(base + ay);
        nz = *reinterpret_cast<const float4*>(base + az);
        fx = *reinterpret_cast<const float4*>(base + (ax ^ FAR_X));
        fy = *reinterpret_cast<const float4*>(base + (ay ^ FAR_Y));
        fz = *reinterpret_cast<const float4*>(base + (az ^ FAR_Z));
        cr = *reinterpret_cast<const int4*>(base + (nb + 96u));
    }
    const int cc[4] = {cr.x, cr.y, cr.z, cr.w};
    float tc[4];
    tc[0] = box4_enter(s.br, nx.x, ny.x, nz.x, fx.x, fy.x, fz.x, s.tmin, s.best_t);
    tc[1] = box4_enter(s.br, nx.y, ny.y, nz.y, fx.y, fy.y, fz.y, s.tmin, s.best_t);
    tc[2] = box4_enter(s.br, nx.z, ny.z, nz.z, fx.z, fy.z, fz.z, s.tmin, s.best_t);
    tc[3] = box4_enter(s.br, nx.w, ny.w, nz.w, fx.w, fy.w, fz.w, s.tmin, s.best_t);
    // Leaf children whose box is hit, tested one per pass; the wave runs as many passes
    // as its busiest lane needs.
    uint32_t lm = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (cc[k] < 0 && tc[k] <= s.best_t) lm |= 1u << k;
    auto test_leaf = [&](int leaf) {
        V3 v0, v1, v2;
        int prim;
        vis.tri();
        load_tri(tris, leaf, v0, v1, v2, prim);
        float t;
        // the triangle left is rejected after the test, not before it: checked first, the
        // prim id was loaded alone and the vertices only after the compare (two dependent
        // round trips to memory per test)
        const bool hit = wt_hit(s.wr, v0, v1, v2, t);
        if (!hit | !(t > s.tmin) | (prim == s.skip)) return;
        bool take = t < s.best_t;
        if constexpr (!ANY) {
            // equal t: the smaller original index wins (the current best's index is read
            // back from its record, so no register holds it)
            if (!take && t == s.best_t && s.best_leaf >= 0) take = prim < __float_as_int(tris[3 * s.best_leaf].w);
        }
        if (take) {
            s.best_t = t;
            s.best_leaf = leaf;
        }
    };
    {
        // the lane's hit leaves compacted: pass j runs when some lane has more than j of
        // them (fewer passes than one per slot any lane uses)
        const int nl = __popc(lm);
        uint32_t m = lm;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < nl) {
                const int k = __builtin_ctz(m);
                m &= m - 1u;
                test_leaf(~(k == 0 ? cc[0] : (k == 1 ? cc[1] : (k == 2 ? cc[2] : cc[3]))));
            }
    }
    // internal children still in range (a missed box reports NaN; one entered only at
    // +inf is dropped like a miss)
    float key[4];
    int ref[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = cc[k] >= 0 && tc[k] <= s.best_t;
        key[k] = in ? tc[k] : __builtin_inff();
        ref[k] = cc[k];
    }
    cmpx(key[0], ref[0], key[1], ref[1]);
    cmpx(key[2], ref[2], key[3], ref[3]);
    cmpx(key[0], ref[0], key[2], ref[2]);
    cmpx(key[1], ref[1], key[3], ref[3]);
    cmpx(key[1], ref[1], key[2], ref[2]);
    if (ANY && s.best_leaf >= 0) {   // any hit ends the query
        s.node = -1;
    } else if (key[0] < __builtin_inff()) {
        s.node = ref[0];
        // every candidate is written to LDS, at sp, or at the lane's extra entry SHORT
        // once the LDS part is full (a write that is not kept is overwritten or never
        // read), so only the rare spill to global memory is a branch
#pragma unroll
        for (int k = 3; k >= 1; --k) {
            const bool v = key[k] < __builtin_inff();
            stack[min(s.sp, SHORT) * TBK + lane] = ref[k];
            if constexpr (SHORT < MAX_STACK)
                if (v && s.sp >= SHORT && s.sp < MAX_STACK) spill[(s.sp - SHORT) * TBK + lane] = ref[k];
            s.sp = v && s.sp < MAX_STACK ? s.sp + 1 : s.sp;
        }
    } else if (s.sp > 0) {
        --s.sp;
        // an LDS read always (clamped index) and a global read only for spilled entries:
        // two plain loads rather than one generic (flat) load
        int nn = stack[min(s.sp, SHORT - 1) * TBK + lane];
        if constexpr (SHORT < MAX_STACK)
            if (s.sp >= SHORT)   // (a relaxed atomic load: the compiler cannot fold it with the
                                 // LDS read into one generic load of a selected address,
                                 // which would wait on every memory counter each pop)
                nn = __hip_atomic_load(&spill[(s.sp - SHORT) * TBK + lane], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
        s.node = nn;
    } else {
        s.node = -1;
    }
}

template <bool ANY, int SHORT, int TBK, class VIS>
__device__ __forceinline__ bool traverse4(const float4* __restrict__ nodes, const float4* __restrict__ tris, V3 o,
                                          V3 d, float tmin, float tmax, int skip, Hit& h, int* stack, int* spill,
                                          int lane, VIS& vis, TopNodes top) {
    Trav4 s;
    trav4_start(s, o, d, tmin, tmax, skip);
    // the only exit is the loop test (node < 0 once the stack is empty or an any-hit
    // query has its hit): with no break inside, the compiler keeps the pop an ordinary
    // branch of the one loop, instead of a nested loop whose lanes wait until every
    // lane of the wave needs a pop
    while (s.node >= 0) trav4_visit<ANY, SHORT, TBK>(s, nodes, tris, stack, spill, lane, vis, top);
    // the barycentrics of the hit: the same test on its triangle again (same arithmetic,
    // same bits), which keeps them out of the loop's registers
    float bb1 = 0.f, bb2 = 0.f;
    int best_prim = -1;
    if (s.best_leaf >= 0) {
        V3 v0, v1, v2;
        load_tri(tris, s.best_leaf, v0, v1, v2, best_prim);
        wt_intersect(s.wr, v0, v1, v2, s.best_t, bb1, bb2);
    }
    h.t = s.best_t;
    h.leaf = s.best_leaf;
    h.prim = best_prim;
    h.b1 = bb1;
    h.b2 = bb2;
    return s.best_leaf >= 0;
}

// closest or any hit on the request's BVH (4-wide when built)
template <bool ANY, int SHORT, int TBK, class VIS>
__device__ __forceinline__ bool trace_ray(const float4* __restrict__ nodes4, const float4* __restrict__ nodes,
                                          const float4* __restrict__ tris, V3 o, V3 d, float tmin, float tmax,
                                          int skip, Hit& h, int* stack, int* spill, int lane, VIS& vis,
                                          TopNodes top = TopNodes{nullptr, 0u}) {
    if (nodes4)
        return traverse4<ANY, SHORT, TBK>(nodes4, tris, o, d, tmin, tmax, skip, h, stack, spill, lane, vis, top);
    return traverse<ANY, SHORT, TBK>(nodes, tris, o, d, tmin, tmax, skip, h, stack, spill, lane, vis);
}

// reference: every triangle in original order, same arithmetic and tie rule
template <bool ANY>
__device__ __forceinline__ bool brute_force(const float4* __restrict__ tris, const int* __restrict__ leaf_of_prim,
                                            int ntri, V3 o, V3 d, float tmin, float tmax, int skip, Hit& h) {
    const WtRay wr = wt_setup(o, d);
    float best_t = tmax;
    int best = -1, best_leaf = -1;
    for (int p = 0; p < ntri; ++p) {
        if (p == skip) continue;
        const int leaf = leaf_of_prim[p];
        V3 v0, v1, v2;
        int prim;
        load_tri(tris, leaf, v0, v1, v2, prim);
        float t;
        // triangles are visited in increasing original index, so on equal t the first wins
        if (wt_hit(wr, v0, v1, v2, t) && t > tmin && t < best_t) {
            best_t = t;
            best = prim;
            best_leaf = leaf;
            if (ANY) break;
        }
    }
    float bb1 = 0.f, bb2 = 0.f;
    if (best_leaf >= 0) {
        V3 v0, v1, v2;
        int prim;
        load_tri(tris, best_leaf, v0, v1, v2, prim);
        wt_intersect(wr, v0, v1, v2, best_t, bb1, bb2);
    }
    h.t = best_t;
    h.leaf = best_leaf;
    h.prim = best;
    h.b1 = bb1;
    h.b2 = bb2;
    return best >= 0;
}

}  // namespace dpcs
