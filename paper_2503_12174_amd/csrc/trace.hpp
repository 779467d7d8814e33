// trace.hpp -- ray queries on the device BVH.
//
// BVH2 node (64 B, 4 x float4): both children's boxes inline so one node fetch
// tests two boxes.
//   n0 = (lo0.x, lo0.y, lo0.z, hi0.x)  n1 = (hi0.y, hi0.z, lo1.x, lo1.y)
//   n2 = (lo1.z, hi1.x, hi1.y, hi1.z)  n3 = (child0, child1, -, -) as int bits
// BVH4 node (128 B, one cache line, 8 x float4): the four children's boxes as
// structure of arrays, lo.x[4], lo.y[4], lo.z[4], hi.x[4], hi.y[4], hi.z[4], then the
// four child references and 16 unused bytes.
// child >= 0: internal node index; child < 0: leaf ~child (one triangle, leaf order);
// WIDE_EMPTY: unused slot of a BVH4 node.
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
    int kx, ky, kz;
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
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.Sx = comp(d, kx) / dz;
    r.Sy = comp(d, ky) / dz;
    r.Sz = 1.0f / dz;
    return r;
}

// returns false on a miss; on a hit t and the barycentrics (b1 of v1, b2 of v2)
__device__ __forceinline__ bool wt_intersect(const WtRay& r, V3 v0, V3 v1, V3 v2, float& t, float& b1, float& b2) {
    const V3 A = v0 - r.o, B = v1 - r.o, C = v2 - r.o;
    const float Akz = comp(A, r.kz), Bkz = comp(B, r.kz), Ckz = comp(C, r.kz);
    const float Ax = comp(A, r.kx) - r.Sx * Akz, Ay = comp(A, r.ky) - r.Sy * Akz;
    const float Bx = comp(B, r.kx) - r.Sx * Bkz, By = comp(B, r.ky) - r.Sy * Bkz;
    const float Cx = comp(C, r.kx) - r.Sx * Ckz, Cy = comp(C, r.ky) - r.Sy * Ckz;
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

struct Hit {
    float t;
    int leaf;   // leaf-order triangle index, -1 on a miss
    int prim;   // original triangle index
    float b1, b2;
};

struct BoxRay {
    V3 o, inv;
};
__device__ __forceinline__ BoxRay box_setup(V3 o, V3 d) { return BoxRay{o, v3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z)}; }

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

// Traversal stack of internal node indices: the first SHORT entries live in LDS
// (entry k of thread tid at lds[k * TBK + tid], consecutive lanes on consecutive banks);
// deeper entries -- rare with near-child-first order -- go to the workgroup's region of
// global memory with the same interleaving (spill[k * TBK + tid]).  The host only
// launches on trees of depth <= 64, so at most 64 entries are ever live.
struct Visits {
    uint32_t nodes = 0, tris = 0;
};

template <bool ANY, int SHORT, int TBK>
__device__ __forceinline__ bool traverse(const float4* __restrict__ nodes, const float4* __restrict__ tris, V3 o, V3 d,
                                         float tmin, float tmax, int skip, Hit& h, int* stack, int* spill,
                                         Visits& vis) {
    const BoxRay br = box_setup(o, d);
    const WtRay wr = wt_setup(o, d);
    float best_t = tmax;
    int best_prim = 0x7fffffff, best_leaf = -1;
    float bb1 = 0.f, bb2 = 0.f;
    int sp = 0;
    int node = 0;
    while (true) {
        ++vis.nodes;
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
                ++vis.tris;
                load_tri(tris, leaf, v0, v1, v2, prim);
                float t, b1, b2;
                if (prim != skip && wt_intersect(wr, v0, v1, v2, t, b1, b2) && t > tmin &&
                    (t < best_t || (t == best_t && best_leaf >= 0 && prim < best_prim))) {
                    best_t = t;
                    best_prim = prim;
                    best_leaf = leaf;
                    bb1 = b1;
                    bb2 = b2;
                    if (ANY) {
                        h.t = t;
                        h.leaf = leaf;
                        h.prim = prim;
                        h.b1 = b1;
                        h.b2 = b2;
                        return true;
                    }
                }
            }
        }
        // a missed box reports +inf, which must not pass while best_t is still +inf
        const bool h0 = c0 >= 0 && t0 < __builtin_inff() && t0 <= best_t;
        const bool h1 = c1 >= 0 && t1 < __builtin_inff() && t1 <= best_t;
        if (h0 && h1) {
            const bool first0 = t0 <= t1;
            const int far = first0 ? c1 : c0;
            if (sp < SHORT) stack[sp * TBK] = far;
            else if constexpr (SHORT < MAX_STACK) {
                if (sp < MAX_STACK) spill[(sp - SHORT) * TBK] = far;
            }
            sp = sp < MAX_STACK ? sp + 1 : sp;   // depth <= 64 is checked on the host
            node = first0 ? c0 : c1;
        } else if (h0) {
            node = c0;
        } else if (h1) {
            node = c1;
        } else {
            if (sp == 0) break;
            --sp;
            if constexpr (SHORT < MAX_STACK) node = sp < SHORT ? stack[sp * TBK] : spill[(sp - SHORT) * TBK];
            else node = stack[sp * TBK];
        }
    }
    h.t = best_t;
    h.leaf = best_leaf;
    h.prim = best_leaf >= 0 ? best_prim : -1;
    h.b1 = bb1;
    h.b2 = bb2;
    return best_leaf >= 0;
}

constexpr int WIDE_EMPTY = (int)0x80000000;

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

// Same query on the 4-wide BVH: per node, four box tests; leaf children are tested at
// once, internal children still in range are visited nearest first (the others pushed,
// farthest first).  The host only builds a BVH4 whose worst-case stack fits MAX_STACK.
template <bool ANY, int SHORT, int TBK>
__device__ __forceinline__ bool traverse4(const float4* __restrict__ nodes, const float4* __restrict__ tris, V3 o,
                                          V3 d, float tmin, float tmax, int skip, Hit& h, int* stack, int* spill,
                                          Visits& vis) {
    const BoxRay br = box_setup(o, d);
    const WtRay wr = wt_setup(o, d);
    float best_t = tmax;
    int best_prim = 0x7fffffff, best_leaf = -1;
    float bb1 = 0.f, bb2 = 0.f;
    int sp = 0;
    int node = 0;
    while (true) {
        ++vis.nodes;
        const float4* nd = nodes + 8 * (size_t)node;
        const float4 lx = nd[0], ly = nd[1], lz = nd[2], hx = nd[3], hy = nd[4], hz = nd[5];
        const int4 cr = *reinterpret_cast<const int4*>(nd + 6);
        const int cc[4] = {cr.x, cr.y, cr.z, cr.w};
        float tc[4];
        tc[0] = box_enter(br, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, tmin, best_t);
        tc[1] = box_enter(br, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, tmin, best_t);
        tc[2] = box_enter(br, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, tmin, best_t);
        tc[3] = box_enter(br, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, tmin, best_t);
        // Leaf children whose box is hit.  Closest hit: every slot unrolled, so the
        // triangle fetches of all four are in flight together.  Any hit: one test per
        // pass of a loop, the wave runs it as often as its busiest lane needs.
        uint32_t lm = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (cc[k] == WIDE_EMPTY) tc[k] = __builtin_inff();
            if (cc[k] < 0 && tc[k] < __builtin_inff()) lm |= 1u << k;
        }
        auto test_leaf = [&](int leaf) {
            V3 v0, v1, v2;
            int prim;
            ++vis.tris;
            load_tri(tris, leaf, v0, v1, v2, prim);
            float t, b1, b2;
            if (prim != skip && wt_intersect(wr, v0, v1, v2, t, b1, b2) && t > tmin &&
                (t < best_t || (t == best_t && best_leaf >= 0 && prim < best_prim))) {
                best_t = t;
                best_prim = prim;
                best_leaf = leaf;
                bb1 = b1;
                bb2 = b2;
                return true;
            }
            return false;
        };
        if constexpr (ANY) {
            while (lm) {
                const int k = __builtin_ctz(lm);
                lm &= lm - 1u;
                if (test_leaf(~(k == 0 ? cc[0] : (k == 1 ? cc[1] : (k == 2 ? cc[2] : cc[3]))))) {
                    h.t = best_t;
                    h.leaf = best_leaf;
                    h.prim = best_prim;
                    h.b1 = bb1;
                    h.b2 = bb2;
                    return true;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (lm & (1u << k)) test_leaf(~cc[k]);
        }
        // internal children still in range (a missed box reports +inf)
        float key[4];
        int ref[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool in = cc[k] >= 0 && tc[k] < __builtin_inff() && tc[k] <= best_t;
            key[k] = in ? tc[k] : __builtin_inff();
            ref[k] = cc[k];
        }
        cmpx(key[0], ref[0], key[1], ref[1]);
        cmpx(key[2], ref[2], key[3], ref[3]);
        cmpx(key[0], ref[0], key[2], ref[2]);
        cmpx(key[1], ref[1], key[3], ref[3]);
        cmpx(key[1], ref[1], key[2], ref[2]);
        if (key[0] < __builtin_inff()) {
            node = ref[0];
#pragma unroll
            for (int k = 3; k >= 1; --k) {
                if (!(key[k] < __builtin_inff())) continue;
                if (sp < SHORT) stack[sp * TBK] = ref[k];
                else if constexpr (SHORT < MAX_STACK) {
                    if (sp < MAX_STACK) spill[(sp - SHORT) * TBK] = ref[k];
                }
                sp = sp < MAX_STACK ? sp + 1 : sp;
            }
        } else {
            if (sp == 0) break;
            --sp;
            if constexpr (SHORT < MAX_STACK) node = sp < SHORT ? stack[sp * TBK] : spill[(sp - SHORT) * TBK];
            else node = stack[sp * TBK];
        }
    }
    h.t = best_t;
    h.leaf = best_leaf;
    h.prim = best_leaf >= 0 ? best_prim : -1;
    h.b1 = bb1;
    h.b2 = bb2;
    return best_leaf >= 0;
}

// closest or any hit on the request's BVH (4-wide when built)
template <bool ANY, int SHORT, int TBK>
__device__ __forceinline__ bool trace_ray(const float4* __restrict__ nodes4, const float4* __restrict__ nodes,
                                          const float4* __restrict__ tris, V3 o, V3 d, float tmin, float tmax,
                                          int skip, Hit& h, int* stack, int* spill, Visits& vis) {
    if (nodes4) return traverse4<ANY, SHORT, TBK>(nodes4, tris, o, d, tmin, tmax, skip, h, stack, spill, vis);
    return traverse<ANY, SHORT, TBK>(nodes, tris, o, d, tmin, tmax, skip, h, stack, spill, vis);
}

// reference: every triangle in original order, same arithmetic and tie rule
template <bool ANY>
__device__ __forceinline__ bool brute_force(const float4* __restrict__ tris, const int* __restrict__ leaf_of_prim,
                                            int ntri, V3 o, V3 d, float tmin, float tmax, int skip, Hit& h) {
    const WtRay wr = wt_setup(o, d);
    float best_t = tmax;
    int best = -1, best_leaf = -1;
    float bb1 = 0.f, bb2 = 0.f;
    for (int p = 0; p < ntri; ++p) {
        if (p == skip) continue;
        const int leaf = leaf_of_prim[p];
        V3 v0, v1, v2;
        int prim;
        load_tri(tris, leaf, v0, v1, v2, prim);
        float t, b1, b2;
        // triangles are visited in increasing original index, so on equal t the first wins
        if (wt_intersect(wr, v0, v1, v2, t, b1, b2) && t > tmin && t < best_t) {
            best_t = t;
            best = prim;
            best_leaf = leaf;
            bb1 = b1;
            bb2 = b2;
            if (ANY) break;
        }
    }
    h.t = best_t;
    h.leaf = best_leaf;
    h.prim = best;
    h.b1 = bb1;
    h.b2 = bb2;
    return best >= 0;
}

}  // namespace dpcs
