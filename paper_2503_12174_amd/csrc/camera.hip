// camera.hip -- the camera-pose part of the VJP: d loss / d (R_c, t_c) (Sec. 3.2, theta
// holds the camera rotation and translation for refinement).
//
// The interior part (the boundary part, at the images of mesh edges, is edges.hip): per
// camera sample with a first hit, the camera vertex's radiance
// V(x, wo) -- projector next event, environment next event and the bounce factor, each as
// the forward evaluated it, with every decision (visibilities, the path going on), the
// sampled environment and bounce directions and everything beyond the first vertex held at
// the forward's values -- is differentiated w.r.t. the hit point x (within the triangle's
// plane) and the direction to the camera wo, by forward differences in FP64 along two
// in-plane and two tangent directions (the point's texture and projector lookups are
// reused for the direction steps).  The camera geometry is then chained analytically:
// the ray o = -R^T t, d = q / |q| with q = R^T K^-1 (px, py, 1) meets the plane at
// x = o + tau d, so dx = P (do + tau dd) with P = I - d n^T / (n.d), dwo = -dd and
// dd = (I - d d^T) dq / |q|.  The bounce's remaining radiance is recovered from the
// forward's sample radiance: L - Le - (next events) = B R_1 / pdf, so only d B / B is
// needed.  Per-workgroup partial sums of the 12 entries are summed in a fixed order.
#include "kernels.hpp"
#include "shade.hpp"

namespace dpcs {

constexpr int CAM_TB = 128;

// what the forward decided and sampled at the camera vertex
struct CamFrozen {
    int leaf;
    D3 n;            // two-sided geometric normal facing the camera
    bool prj, env, bounced;
    D3 we, wi;       // sampled environment and bounce directions
    D3 Se;           // L_env pi / (sampling normal . we)
    D3 W;            // R_1 / pdf per channel: the bounce factor's weight
};

// what the camera vertex's terms read at hit point x (in the triangle's plane): material,
// shading normal and the projector's direction, irradiance and falloff
struct CamSurf {
    D3 alb, ns, wp, E;
    double rough, spec, metal, g;   // g = 1 / (cos^3 alpha d^2)
};

__device__ __forceinline__ CamSurf cam_surface(const ReqDesc& r, const CamFrozen& z, D3 x) {
    Surf s;
    V3 f0, f1, f2;
    load_tri(r.tris, z.leaf, f0, f1, f2, s.prim);
    const D3 v0 = to_d(f0), e1 = to_d(f1) - v0, e2 = to_d(f2) - v0, p = x - v0;
    // barycentrics of x in the plane: normal equations of p = b1 e1 + b2 e2
    const double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2), r1 = dot(p, e1), r2 = dot(p, e2);
    const double inv = 1.0 / (a11 * a22 - a12 * a12);
    const double b1 = (a22 * r1 - a12 * r2) * inv, b2 = (a11 * r2 - a12 * r1) * inv, b0 = 1.0 - b1 - b2;
    s.x = x;
    s.n = z.n;
    const float4 ua = r.tri_uv[2 * z.leaf], ub = r.tri_uv[2 * z.leaf + 1];
    s.u = b0 * ua.x + b1 * ua.z + b2 * ub.x;
    s.v = b0 * ua.y + b1 * ua.w + b2 * ub.y;
    s.tb = bilinear(s.u * r.tw - 0.5, s.v * r.th - 0.5, r.tw, r.th);
    const D4 t4 = fetch4(r.tex4, s.tb);
    CamSurf c;
    c.alb = d3(t4.x, t4.y, t4.z);
    c.rough = t4.w;
    c.spec = r.brdf ? fetch1(r.spec, s.tb) : 0.0;
    c.ns = z.n;
    c.metal = 0.0;
    if (r.tex4b) {
        const Shading sh = shading(r, z.leaf, s);
        c.ns = sh.ns;
        c.metal = sh.metal;
    }
    c.wp = d3(0., 0., 0.);
    c.E = d3(0., 0., 0.);
    c.g = 0.0;
    if (z.prj) {   // the projector term in full, the frustum and cosine decisions held
        const D3 xp = mat3(r.prj_R, x) + d3(r.prj_t[0], r.prj_t[1], r.prj_t[2]);
        const double iz = 1.0 / xp.z;
        const double pu = (r.prj_K[0] * xp.x + r.prj_K[1] * xp.y + r.prj_K[2] * xp.z) * iz;
        const double pv = (r.prj_K[3] * xp.x + r.prj_K[4] * xp.y + r.prj_K[5] * xp.z) * iz;
        const D3 tow = d3(r.prj_o[0], r.prj_o[1], r.prj_o[2]) - x;
        const double dist = sqrt(dot(tow, tow));
        c.wp = tow * (1.0 / dist);
        const double ca = xp.z / sqrt(dot(xp, xp));
        const D4 E = fetch4(r.Ep, bilinear(pu - 0.5, pv - 0.5, r.Wp, r.Hp));
        c.E = d3(E.x, E.y, E.z);
        c.g = 1.0 / (ca * ca * ca * dist * dist);
    }
    return c;
}

// the camera vertex's terms seen along wo from a surface point: next events and the
// bounce factor f c (the bounce's weight applied by the caller)
__device__ __forceinline__ void cam_eval(const ReqDesc& r, const CamFrozen& z, const CamSurf& c, D3 wo, D3& nee,
                                         D3& bnc) {
    nee = d3(0., 0., 0.);
    bnc = d3(0., 0., 0.);
    if (z.prj) {
        const BrdfX f = brdf_x<false>(r.brdf, z.n, c.ns, wo, c.wp, c.alb, c.rough, c.spec, c.metal);
        nee = f.f * c.E * (f.c * c.g);
    }
    if (z.env) {
        const BrdfX f = brdf_x<false>(r.brdf, z.n, c.ns, wo, z.we, c.alb, c.rough, c.spec, c.metal);
        nee = nee + f.f * z.Se * f.c;
    }
    if (z.bounced) {
        const BrdfX f = brdf_x<false>(r.brdf, z.n, c.ns, wo, z.wi, c.alb, c.rough, c.spec, c.metal);
        bnc = f.f * f.c;
    }
}

__device__ __forceinline__ double cam_phi(const ReqDesc& r, const CamFrozen& z, const CamSurf& c, D3 wo, D3 delta) {
    D3 nee, bnc;
    cam_eval(r, z, c, wo, nee, bnc);
    return dot(delta, nee + bnc * z.W);
}

// one thread per camera sample of the wave [p0, p1) x spp; partials of the 12 entries
__global__ void __launch_bounds__(CAM_TB) k_cam_grad(Queues q, AdjQueues aq, ReqDesc r, uint32_t p0, uint32_t p1) {
    double acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    const uint32_t n = (p1 - p0) * (uint32_t)r.spp;
    const uint32_t k = blockIdx.x * CAM_TB + threadIdx.x;
    if (k < n) {
        const uint32_t g = p0 * (uint32_t)r.spp + k;
        const uint32_t sid = g - r.g_base + r.sid_base;
        const float4 dl = aq.delta[sid];
        const uint32_t rec = r.rec[(size_t)(g - r.rec_g0) * r.max_depth];
        const int leaf = (int)(rec & REC_LEAF) - 1;
        if (leaf >= 0 && (dl.x != 0.f || dl.y != 0.f || dl.z != 0.f)) {
            const D3 delta = d3(dl.x, dl.y, dl.z);
            // the forward's camera ray (the same jittered pixel position as camera_dir)
            const uint32_t pixel = g / (uint32_t)r.spp, si = g - pixel * (uint32_t)r.spp;
            const U4 u = philox4x32_10(pixel, si + r.sample_offset, 0u, 0u, r.seed_lo, r.seed_hi);
            const D3 m = mat3(r.cam_Ki, d3((double)(pixel % (uint32_t)r.Wc) + u24(u.x),
                                           (double)(pixel / (uint32_t)r.Wc) + u24(u.y), 1.0));
            const D3 qv = d3(r.cam_R[0] * m.x + r.cam_R[3] * m.y + r.cam_R[6] * m.z,
                             r.cam_R[1] * m.x + r.cam_R[4] * m.y + r.cam_R[7] * m.z,
                             r.cam_R[2] * m.x + r.cam_R[5] * m.y + r.cam_R[8] * m.z);
            const double ql = sqrt(dot(qv, qv));
            const D3 dir = qv * (1.0 / ql);
            const D3 o = d3(r.cam_o[0], r.cam_o[1], r.cam_o[2]);
            const Surf s0 = surface(r, leaf, o, dir);
            CamFrozen z;
            z.leaf = leaf;
            z.n = s0.n;
            z.prj = (rec & REC_PRJ) != 0u;
            z.env = (rec & REC_ENV) != 0u;
            const D3 ns0 = r.tex4b ? shading(r, leaf, s0).ns : s0.n;
            z.we = d3(0., 0., 0.);
            z.Se = d3(0., 0., 0.);
            if (r.env_on) {
                const U4 x = vertex_rng(r, g, 2u);
                z.we = sample_cosine(ns0, u24(x.x), u24(x.y));
                z.Se = d3(r.env[0], r.env[1], r.env[2]) * (PI / dot(ns0, z.we));
            }
            z.bounced = false;
            z.wi = d3(0., 0., 0.);
            if (r.max_depth > 1) {
                const U4 x = vertex_rng(r, g, 1u);
                z.wi = sample_bounce(r.brdf, ns0, s0.wo, s0.rough, u24(x.x), u24(x.y), u24(x.z));
                z.bounced = dot(s0.n, z.wi) > 0.0 && bounce_pdf(r.brdf, ns0, s0.wo, z.wi, s0.rough) > 0.0;
            }
            // the bounce's weight R_1 / pdf from the forward's sample radiance
            z.W = d3(0., 0., 0.);
            D3 nee0, b0;
            const CamSurf c0 = cam_surface(r, z, s0.x);
            cam_eval(r, z, c0, s0.wo, nee0, b0);
            if (z.bounced) {
                const float4 L = q.L[sid];
                D3 rest = d3(L.x, L.y, L.z) - nee0;
                if (r.emission) {
                    const float4 e = r.emission[leaf];
                    rest = rest - d3(e.x, e.y, e.z);
                }
                z.W = d3(b0.x > 0.0 ? rest.x / b0.x : 0.0, b0.y > 0.0 ? rest.y / b0.y : 0.0,
                         b0.z > 0.0 ? rest.z / b0.z : 0.0);
            }
            // central differences along two in-plane directions and two tangents of wo
            V3 f0, f1, f2;
            int prim;
            load_tri(r.tris, leaf, f0, f1, f2, prim);
            const D3 t1 = normalize(to_d(f1) - to_d(f0)), t2 = cross(s0.n, t1);
            // forward differences from the forward's own point and direction; steps 1e-8 of
            // the hit distance and 1e-7 rad: far below a texel, a projector pixel or the
            // narrowest GGX lobe (alpha >= 1e-3, so the one-sided error stays below ~1e-4),
            // and far above the FP64 rounding of the terms (~1e-8 relative in the slope)
            const double tau = dot(s0.x - o, dir);
            const double hx = 1e-8 * tau, hw = 1e-7;
            const double phi0 = cam_phi(r, z, c0, s0.wo, delta);
            D3 gx = d3(0., 0., 0.), gw = d3(0., 0., 0.);
            const D3 ta[2] = {t1, t2};
            for (int j = 0; j < 2; ++j) {
                const double fp = cam_phi(r, z, cam_surface(r, z, s0.x + ta[j] * hx), s0.wo, delta);
                gx = gx + ta[j] * ((fp - phi0) / hx);
            }
            const D3 w1 = local_to_world(s0.wo, 1.0, 0.0, 0.0), w2 = local_to_world(s0.wo, 0.0, 1.0, 0.0);
            const D3 wa[2] = {w1, w2};
            for (int j = 0; j < 2; ++j) {   // same point: its lookups reused
                const double fp = cam_phi(r, z, c0, normalize(s0.wo + wa[j] * hw), delta);
                gw = gw + wa[j] * ((fp - phi0) / hw);
            }
            // chain to (R, t): a = P^T gx, b = tau a - gw, c = (I - d d^T) b / |q|
            const D3 a = gx - s0.n * (dot(dir, gx) / dot(s0.n, dir));
            const D3 b = a * tau - gw;
            const D3 c = (b - dir * dot(dir, b)) * (1.0 / ql);
            const double mi[3] = {m.x, m.y, m.z}, ti[3] = {r.cam_t[0], r.cam_t[1], r.cam_t[2]};
            const double cj[3] = {c.x, c.y, c.z}, aj[3] = {a.x, a.y, a.z};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[3 * i + j] = cj[j] * mi[i] - aj[j] * ti[i];
                acc[9 + i] = -(r.cam_R[3 * i] * a.x + r.cam_R[3 * i + 1] * a.y + r.cam_R[3 * i + 2] * a.z);
            }
        }
    }
    // workgroup sums (wave shuffles, then the waves in order)
    __shared__ double red[12][CAM_TB / 64];
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
        for (int w = 0; w < CAM_TB / 64; ++w) v += red[threadIdx.x][w];
        r.d_cam_part[12 * (size_t)blockIdx.x + threadIdx.x] = (float)v;
    }
}

size_t cam_partial_floats(int64_t samples_per_wave) {
    return 12 * (size_t)((samples_per_wave + CAM_TB - 1) / CAM_TB);
}

void launch_cam_grad(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, uint32_t p0,
                     uint32_t p1) {
    const int64_t n = (int64_t)(p1 - p0) * r.spp;
    if (n <= 0 || !r.d_cam_part) return;
    const unsigned nb = (unsigned)((n + CAM_TB - 1) / CAM_TB);
    hipLaunchKernelGGL(k_cam_grad, dim3(nb), dim3(CAM_TB), 0, l.st, q, aq, r, p0, p1);
    launch_sum_partials(l, r.d_cam_part, (int)nb, 12, 12, r.d_acc + 20);   // after the PRF partials
}

}  // namespace dpcs
