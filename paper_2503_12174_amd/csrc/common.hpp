// common.hpp -- device-side building blocks shared by the gfx950 kernels:
// small vector math, the Philox4x32-10 counter-based generator, the BRDF (Lambert,
// Lambert + GGX microfacet specular) with its derivatives, the bounce sampler, and
// the per-request descriptor every kernel reads.
//
// Precision plan: BVH traversal runs in FP32 on rounded copies of the rays (it only
// decides which triangle is hit).  Everything that turns a hit into a number --
// hit point, texture and projector coordinates, directions, BRDF -- runs in FP64:
// FP32 texel coordinates of 512^2 maps carry ~3e-5 texel of rounding, which steep
// roughness maps turn into ~1e-3 relative error of a glossy GGX lobe.  CDNA4 runs
// FP64 vector math at half the FP32 rate, and shading is not the bottleneck.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpcs {

constexpr int BLOCK = 256;          // threads per workgroup (4 wave64)
constexpr int PIX_LANES = 8;        // lanes per pixel in the per-pixel sample reductions
constexpr double PI = 3.14159265358979323846;
constexpr double P_SPEC = 0.25;     // probability of sampling the GGX lobe
constexpr double ALPHA_MIN = 1e-3;  // GGX alpha floor
constexpr int MAX_STACK = 64;       // traversal stack entries a ray may hold (checked per scene)
constexpr int TOP_NODES = 32;       // top 4-wide nodes a traversal workgroup stages in LDS

// ---------------------------------------------------------------------------
// vectors
// ---------------------------------------------------------------------------
template <class T>
struct Vec3 {
    T x, y, z;
};
using V3 = Vec3<float>;
using D3 = Vec3<double>;

template <class T> __device__ __forceinline__ Vec3<T> mk3(T x, T y, T z) { return Vec3<T>{x, y, z}; }
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
template <class T> __device__ __forceinline__ Vec3<T> operator+(Vec3<T> a, Vec3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> __device__ __forceinline__ Vec3<T> operator-(Vec3<T> a, Vec3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> __device__ __forceinline__ Vec3<T> operator-(Vec3<T> a) { return {-a.x, -a.y, -a.z}; }
template <class T> __device__ __forceinline__ Vec3<T> operator*(Vec3<T> a, T s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> __device__ __forceinline__ Vec3<T> operator*(Vec3<T> a, Vec3<T> b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
template <class T> __device__ __forceinline__ T dot(Vec3<T> a, Vec3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> __device__ __forceinline__ Vec3<T> cross(Vec3<T> a, Vec3<T> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 normalize(V3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
__device__ __forceinline__ D3 normalize(D3 a) { return a * (1.0 / sqrt(dot(a, a))); }
__device__ __forceinline__ V3 xyz(float4 a) { return v3(a.x, a.y, a.z); }
__device__ __forceinline__ float4 f4(V3 a, float w) { return make_float4(a.x, a.y, a.z, w); }
__device__ __forceinline__ V3 to_f(D3 a) { return v3((float)a.x, (float)a.y, (float)a.z); }
__device__ __forceinline__ D3 to_d(V3 a) { return d3(a.x, a.y, a.z); }
__device__ __forceinline__ float comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
// 3x3 row-major times vector
__device__ __forceinline__ D3 mat3(const double* m, D3 a) {
    return d3(m[0] * a.x + m[1] * a.y + m[2] * a.z, m[3] * a.x + m[4] * a.y + m[5] * a.z,
              m[6] * a.x + m[7] * a.y + m[8] * a.z);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (c0..c3), 64-bit key
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}
// top 24 bits -> [0, 1), exact in float and double
__device__ __forceinline__ double u24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

// Non-temporal (streaming) access to queue records that a kernel reads or writes once:
// the line is not kept in the caches, which then keep more of what is reused -- BVH
// nodes and triangle records during traversal, texture and projector maps in shading.
template <int B> struct NtChunk;   // unsigned vector of B bytes
template <> struct NtChunk<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };
template <> struct NtChunk<8> { typedef unsigned int type __attribute__((ext_vector_type(2))); };
template <> struct NtChunk<4> { typedef unsigned int type; };
template <class T>
constexpr int nt_chunk() { return sizeof(T) % 16 == 0 ? 16 : (sizeof(T) % 8 == 0 ? 8 : 4); }
template <class T>
__device__ __forceinline__ T nt_ld(const T* p) {
    constexpr int B = nt_chunk<T>();
    static_assert(sizeof(T) % 4 == 0, "streamed records are 4-byte multiples");
    typedef typename NtChunk<B>::type C;
    T v;
    const C* s = reinterpret_cast<const C*>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / B); ++k) {
        const C x = __builtin_nontemporal_load(s + k);
        __builtin_memcpy(reinterpret_cast<char*>(&v) + B * k, &x, B);
    }
    return v;
}
template <class T>
__device__ __forceinline__ void nt_st(T* p, const T& v) {
    constexpr int B = nt_chunk<T>();
    static_assert(sizeof(T) % 4 == 0, "streamed records are 4-byte multiples");
    typedef typename NtChunk<B>::type C;
    C* d = reinterpret_cast<C*>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / B); ++k) {
        C x;
        __builtin_memcpy(&x, reinterpret_cast<const char*>(&v) + B * k, B);
        __builtin_nontemporal_store(x, d + k);
    }
}

// ---------------------------------------------------------------------------
// path state in HBM: 80 bytes per path
// ---------------------------------------------------------------------------
struct alignas(16) PathO {   // ray origin, request slot, triangle the ray leaves (-1: none)
    double x, y, z;
    int32_t slot, skip;
};
struct alignas(16) PathD {   // unit direction, global sample index
    double x, y, z;
    uint32_t g, pad;
};

// ---------------------------------------------------------------------------
// per-request descriptor (one per active request; kernels read it by slot)
// ---------------------------------------------------------------------------
struct ReqDesc {
    // camera: world direction of pixel position (px, py) is cam_M (px, py, 1)
    double cam_o[3];
    double cam_M[9];
    // the camera pose and inverse intrinsics themselves (camera-pose gradient)
    double cam_R[9], cam_t[3], cam_Ki[9];
    // projector: device coords R x + t, pixel (K (R x + t)).xy / z
    double prj_R[9];
    double prj_t[3];
    double prj_o[3];
    double prj_K[6];
    int32_t Wc, Hc, Wp, Hp;
    // scene (BVH + leaf-ordered triangle records)
    const float4* nodes;     // binary BVH (4 float4 per node)
    const float4* nodes4;    // 4-wide BVH (8 float4 per node), or null: traverse the binary one
    const float4* tris;      // 3 float4 per leaf: v0 (w = prim id bits), v1, v2
    int32_t top_nodes;       // leading 4-wide nodes (breadth-first order) staged in LDS, <= TOP_NODES
    const float4* tri_uv;    // 2 float4 per leaf: (u0 v0 u1 v1), (u2 v2 - -)
    const float4* emission;  // per leaf (rgb, -) or null
    float tmin;
    // material
    int32_t brdf;
    int32_t tw, th;
    const float4* tex4;      // packed (albedo rgb, roughness) per texel
    const float* spec;       // specular per texel
    const float4* tex4b;     // packed (normal map rgb, metallic) per texel, or null: neither map
    int32_t dtex_c;          // cotangent channels per texel of d_tex: 5, or 9 with tex4b
    // lights
    const float4* Ep;        // projector irradiance after the PRF, per texel (rgb, -)
    float env[3];
    int32_t env_on;
    // sampling
    int32_t spp, max_depth;
    uint32_t seed_lo, seed_hi, sample_offset;
    // responses
    float prf_gain, crf_gain;
    int32_t clip;
    float clip_k;
    float scal[18];          // gamma_p[3], M[9], gamma_c[3], w[3]
    const float* dscal;      // device override of scal (or null)
    // mapping of this wave's samples: batch index sid = g - g_base + sid_base
    uint32_t g_base, sid_base;
    // outputs
    const float* proj_image;
    float* out_image;
    float* out_linear;
    float* out_L;
    int32_t* out_hits;
    // adjoint
    const float* grad_image;   // dLoss/dI_c, or null with target set
    const float* target;       // L2 target (server compensation step)
    float* dEp;                // cotangent of E_p, 4 floats per texel
    float* d_tex;              // cotangent of (albedo rgb, roughness, specular[, metallic, normal
                               // map rgb]), dtex_c floats per texel
    float* d_acc;              // 8 floats: d gamma_c[3], d w[3], d threshold, pad
    float* d_cam_part;         // per-workgroup partials of the camera-pose gradient, or null: off
    float* d_part;             // per-workgroup partials of the scalar sums (summed in a fixed
                               // order by a second kernel), or null: float atomics into d_acc
    // path records: one word per (sample, depth) at rec[(g - rec_g0) * max_depth + depth];
    // the forward writes them when rec is set, the replay adjoint reads them
    uint32_t* rec;
    uint32_t rec_g0;
};

// path record word: bits 0..29 leaf + 1 of the vertex hit at that depth (0: the ray
// escaped), bit 30 environment shadow ray unoccluded, bit 31 projector shadow ray unoccluded
constexpr uint32_t REC_LEAF = 0x3fffffffu;
constexpr uint32_t REC_ENV = 1u << 30;
constexpr uint32_t REC_PRJ = 1u << 31;

__device__ __forceinline__ float scalar(const ReqDesc& r, int k) { return r.dscal ? r.dscal[k] : r.scal[k]; }
__device__ __forceinline__ float clip_threshold(const ReqDesc& r) {
    float w0 = scalar(r, 15), w1 = scalar(r, 16), w2 = scalar(r, 17);
    return r.clip_k / fminf(w0, fminf(w1, w2));
}

// ---------------------------------------------------------------------------
// BRDF: f = albedo / pi  [+ F D G / (4 cos_i cos_o)]  (GGX, Smith G, Schlick F)
// evaluated in FP64; the microfacet term uses sin^2 theta_h from |n x h|^2 so the
// GGX denominator has no cancellation near the lobe peak.
// ---------------------------------------------------------------------------
struct Brdf {
    D3 f;           // value per channel
    double ds_dr;   // d(specular term)/d roughness
    double ds_dsp;  // d(specular term)/d specular
};

__device__ __forceinline__ double ggx_alpha(double r) { return fmax(r * r, ALPHA_MIN); }

// The GGX terms use the unnormalised half vector v = wi + wo (|v|^2 = vv): with h =
// v / |v|, cos^2 = (n.v)^2 / vv, sin^2 = |n x v|^2 / vv and, wi and wo being unit,
// wi.h = sqrt(vv) / 2.  D G / (4 ci co), with D = a^2 / (pi k^2) and the Smith factors
// G1 = 2c / (c + q), q = sqrt(a^2 + (1 - a^2) c^2), is then
// a^2 vv^2 / (pi kv^2 (ci + qi)(co + qo)) with kv = k vv: two square roots and one
// division per evaluation.
template <bool GRAD>
__device__ __forceinline__ Brdf brdf_eval(int kind, D3 n, D3 wo, D3 wi, D3 alb, double r, double sp) {
    Brdf b{d3(0., 0., 0.), 0., 0.};
    const double ci = dot(n, wi), co = dot(n, wo);
    if (ci <= 0.0 || co <= 0.0) return b;
    b.f = alb * (1.0 / PI);
    if (kind == 0) return b;
    const D3 v = wi + wo;
    const double vv = dot(v, v), nv = dot(n, v);
    const D3 nxv = cross(n, v);
    const double c2v = nv * nv, s2v = dot(nxv, nxv);
    const double a = ggx_alpha(r);
    const double a2 = a * a;
    const double kv = a2 * c2v + s2v;
    const double qi = sqrt(a2 + (1.0 - a2) * ci * ci), qo = sqrt(a2 + (1.0 - a2) * co * co);
    const double F0 = 0.08 * sp;
    const double m = 1.0 - 0.5 * sqrt(vv);
    const double m5 = m * m * m * m * m;
    const double F = F0 + (1.0 - F0) * m5;
    const double DGw = a2 * vv * vv / (PI * kv * kv * (ci + qi) * (co + qo));   // D G / (4 ci co)
    const double s = F * DGw;
    b.f = b.f + d3(s, s, s);
    if (GRAD) {
        // d ln D / da = (2 / a)(1 - 2 a^2 cos^2 / k);  d ln G1 / da = -a (1 - c^2) / (q (c + q))
        const double dlnD = 2.0 / a * (1.0 - 2.0 * a2 * c2v / kv);
        const double dlnG = -a * ((1.0 - ci * ci) / (qi * (ci + qi)) + (1.0 - co * co) / (qo * (co + qo)));
        const double da_dr = (r * r > ALPHA_MIN) ? 2.0 * r : 0.0;
        b.ds_dr = s * (dlnD + dlnG) * da_dr;
        b.ds_dsp = 0.08 * (1.0 - m5) * DGw;
    }
    return b;
}

// The principled BRDF with metallic mu and a shading normal ns (Sec. 3.2; the readings of
// Burley's model and of the normal map are stated with dpcs_render_params): base colour
// a, f_c = (1 - mu) a_c / pi + F_c D G / (4 cos_i cos_o), F0_c = (1 - mu) 0.08 sp + mu a_c,
// cosines about ns; f = 0 unless wi and wo lie above ns and wi above the geometric
// normal ng.  GRAD adds the derivatives the adjoint needs: of f_c w.r.t. a_c, r, sp, mu
// and of f_c times c = ns.wi w.r.t. ns (as a free vector).  Same unnormalised-half-vector
// evaluation as brdf_eval.
struct BrdfX {
    D3 f;
    double c;       // ns . wi
    double dfa;     // d f_c / d a_c (every channel)
    D3 dfr;         // d f_c / d r
    double dfs;     // d f_c / d sp (every channel)
    D3 dfm;         // d f_c / d mu
    D3 dn[3];       // d (f_c c) / d ns, per channel
};
template <bool GRAD>
__device__ __forceinline__ BrdfX brdf_x(int kind, D3 ng, D3 ns, D3 wo, D3 wi, D3 alb, double r, double sp,
                                        double mu) {
    BrdfX b;
    b.f = d3(0., 0., 0.);
    b.c = dot(ns, wi);
    b.dfa = b.dfs = 0.0;
    b.dfr = b.dfm = d3(0., 0., 0.);
    b.dn[0] = b.dn[1] = b.dn[2] = d3(0., 0., 0.);
    const double ci = b.c, co = dot(ns, wo);
    if (ci <= 0.0 || co <= 0.0 || dot(ng, wi) <= 0.0) return b;
    if (kind == 0) {
        b.f = alb * (1.0 / PI);
        if (GRAD) {
            b.dfa = 1.0 / PI;
            b.dn[0] = wi * (alb.x / PI);
            b.dn[1] = wi * (alb.y / PI);
            b.dn[2] = wi * (alb.z / PI);
        }
        return b;
    }
    const D3 v = wi + wo;
    const double vv = dot(v, v), nv = dot(ns, v);
    const D3 nxv = cross(ns, v);
    const double c2v = nv * nv, s2v = dot(nxv, nxv);
    const double a = ggx_alpha(r);
    const double a2 = a * a;
    const double kv = a2 * c2v + s2v;
    const double qi = sqrt(a2 + (1.0 - a2) * ci * ci), qo = sqrt(a2 + (1.0 - a2) * co * co);
    const double m = 1.0 - 0.5 * sqrt(vv);
    const double m5 = m * m * m * m * m;
    const double DGw = a2 * vv * vv / (PI * kv * kv * (ci + qi) * (co + qo));   // D G / (4 ci co)
    const double kd = 1.0 - mu;
    const D3 F0 = d3(kd * (0.08 * sp) + mu * alb.x, kd * (0.08 * sp) + mu * alb.y, kd * (0.08 * sp) + mu * alb.z);
    const D3 F = d3(F0.x + (1.0 - F0.x) * m5, F0.y + (1.0 - F0.y) * m5, F0.z + (1.0 - F0.z) * m5);
    b.f = alb * (kd / PI) + F * DGw;
    if (GRAD) {
        const double dlnD = 2.0 / a * (1.0 - 2.0 * a2 * c2v / kv);
        const double dlnG = -a * ((1.0 - ci * ci) / (qi * (ci + qi)) + (1.0 - co * co) / (qo * (co + qo)));
        const double da_dr = (r * r > ALPHA_MIN) ? 2.0 * r : 0.0;
        const double dDGw_dr = DGw * (dlnD + dlnG) * da_dr;
        b.dfa = kd / PI + mu * (1.0 - m5) * DGw;
        b.dfr = F * dDGw_dr;
        b.dfs = kd * 0.08 * (1.0 - m5) * DGw;
        b.dfm = alb * (-1.0 / PI) + (alb - d3(0.08 * sp, 0.08 * sp, 0.08 * sp)) * ((1.0 - m5) * DGw);
        // f_c c = (1 - mu) a_c c / pi + F_c S, S = D G1i G1o / (4 co) = DGw ci; with
        // c_h = ns.h (h = v / |v|): dD/dc_h = -4 a^2 c_h (a^2 - 1) / (pi k^3), k = kv / vv,
        // dG1/dc = 2 a^2 / (q (c + q)^2), and dS/dns = (dD/dc_h h G1i G1o + D dG1i wi G1o
        // + D G1i dG1o wo) / (4 co) - S / co wo
        const double iv = 1.0 / sqrt(vv);
        const double ch = nv * iv;
        const double k = kv / vv;
        const double D = a2 / (PI * k * k);
        const double G1i = 2.0 * ci / (ci + qi), G1o = 2.0 * co / (co + qo);
        const double dD = -4.0 * a2 * ch * (a2 - 1.0) / (PI * k * k * k);
        const double dG1i = 2.0 * a2 / (qi * (ci + qi) * (ci + qi)), dG1o = 2.0 * a2 / (qo * (co + qo) * (co + qo));
        const double S = DGw * ci;
        const double i4 = 1.0 / (4.0 * co);
        const D3 dS = v * (dD * G1i * G1o * i4 * iv) + wi * (D * dG1i * G1o * i4) + wo * (D * G1i * dG1o * i4 - S / co);
        b.dn[0] = wi * (kd * alb.x / PI) + dS * F.x;
        b.dn[1] = wi * (kd * alb.y / PI) + dS * F.y;
        b.dn[2] = wi * (kd * alb.z / PI) + dS * F.z;
    }
    return b;
}

// branchless orthonormal basis (Duff et al., JCGT 2017)
__device__ __forceinline__ D3 local_to_world(D3 n, double x, double y, double z) {
    const double s = copysign(1.0, n.z);
    const double a = -1.0 / (s + n.z);
    const double b = n.x * n.y * a;
    const D3 t1 = d3(1.0 + s * n.x * n.x * a, s * b, -s * n.x);
    const D3 t2 = d3(b, s + n.y * n.y * a, -n.y);
    return t1 * x + t2 * y + n * z;
}

__device__ __forceinline__ D3 sample_cosine(D3 n, double u1, double u2) {
    const double rr = sqrt(u1);
    double sn, cs;
    sincos(2.0 * PI * u2, &sn, &cs);
    return local_to_world(n, rr * cs, rr * sn, sqrt(1.0 - u1));
}

// GGX normal-distribution sampling (Walter et al. 2007): tan^2 theta_h = a^2 u1 / (1 - u1)
__device__ __forceinline__ D3 sample_ggx_h(D3 n, double r, double u1, double u2) {
    const double a = ggx_alpha(r);
    const double t2 = a * a * u1 / (1.0 - u1);
    const double ct = 1.0 / sqrt(1.0 + t2);
    const double st = sqrt(t2) * ct;
    double sn, cs;
    sincos(2.0 * PI * u2, &sn, &cs);
    return local_to_world(n, st * cs, st * sn, ct);
}

__device__ __forceinline__ D3 sample_bounce(int kind, D3 n, D3 wo, double r, double ulobe, double u1, double u2) {
    if (kind == 1 && ulobe < P_SPEC) {
        const D3 h = sample_ggx_h(n, r, u1, u2);
        return h * (2.0 * dot(wo, h)) - wo;
    }
    return sample_cosine(n, u1, u2);
}

// density of sample_bounce (solid angle); the microfacet normal that produced wi is
// the one of +-(wi + wo) on n's side
// (GGX part: D(h) |n.h| / (4 |wo.h|) = a^2 vv^2 |n.v| / (4 pi kv^2 |wo.v|), v = wi + wo as
// in brdf_eval)
__device__ __forceinline__ double bounce_pdf(int kind, D3 n, D3 wo, D3 wi, double r) {
    const double ci = dot(n, wi);
    const double pd = ci > 0.0 ? ci * (1.0 / PI) : 0.0;
    if (kind == 0) return pd;
    const D3 v = wi + wo;
    const double nv = fabs(dot(n, v)), ov = fabs(dot(wo, v));
    double ps = 0.0;
    if (nv > 0.0 && ov > 0.0) {
        const D3 nxv = cross(n, v);
        const double vv = dot(v, v), a = ggx_alpha(r), a2 = a * a;
        const double kv = a2 * nv * nv + dot(nxv, nxv);
        ps = a2 * vv * vv * nv / (4.0 * PI * kv * kv * ov);
    }
    return (1.0 - P_SPEC) * pd + P_SPEC * ps;
}

// ---------------------------------------------------------------------------
// bilinear footprint, clamp-to-edge, texel centres at integer + 0.5; coordinates,
// weights and the interpolation in FP64 (map values are FP32 inputs)
// ---------------------------------------------------------------------------
struct Bilin {
    int i00, i10, i01, i11;
    double w00, w10, w01, w11;
};
// Corner texels (clamped to the map) and fractional offsets of a bilinear lookup at
// x, y in texel units with texel (i, j) centred at (i, j)
struct Corners {
    int x0, x1, y0, y1;
    double ax, ay;
};
__device__ __forceinline__ Corners bilinear_corners(double x, double y, int W, int H) {
    const double fx = floor(x), fy = floor(y);
    Corners c;
    c.ax = x - fx;
    c.ay = y - fy;
    const double cx = fmin(fmax(fx, -2.0), (double)W + 1.0), cy = fmin(fmax(fy, -2.0), (double)H + 1.0);
    const int x0 = (int)cx, y0 = (int)cy;
    c.x0 = min(max(x0, 0), W - 1);
    c.x1 = min(max(x0 + 1, 0), W - 1);
    c.y0 = min(max(y0, 0), H - 1);
    c.y1 = min(max(y0 + 1, 0), H - 1);
    return c;
}
__device__ __forceinline__ Bilin bilinear(double x, double y, int W, int H) {
    const Corners c = bilinear_corners(x, y, W, H);
    const int x0 = c.x0, x1 = c.x1, y0 = c.y0, y1 = c.y1;
    const double ax = c.ax, ay = c.ay;
    Bilin b;
    b.i00 = y0 * W + x0;
    b.i10 = y0 * W + x1;
    b.i01 = y1 * W + x0;
    b.i11 = y1 * W + x1;
    b.w00 = (1.0 - ax) * (1.0 - ay);
    b.w10 = ax * (1.0 - ay);
    b.w01 = (1.0 - ax) * ay;
    b.w11 = ax * ay;
    return b;
}

struct D4 {
    double x, y, z, w;
};
__device__ __forceinline__ D4 fetch4(const float4* __restrict__ t, const Bilin& b) {
    const float4 p = t[b.i00], q = t[b.i10], s = t[b.i01], u = t[b.i11];
    return D4{b.w00 * p.x + b.w10 * q.x + b.w01 * s.x + b.w11 * u.x,
              b.w00 * p.y + b.w10 * q.y + b.w01 * s.y + b.w11 * u.y,
              b.w00 * p.z + b.w10 * q.z + b.w01 * s.z + b.w11 * u.z,
              b.w00 * p.w + b.w10 * q.w + b.w01 * s.w + b.w11 * u.w};
}
__device__ __forceinline__ double fetch1(const float* __restrict__ t, const Bilin& b) {
    return b.w00 * t[b.i00] + b.w10 * t[b.i10] + b.w01 * t[b.i01] + b.w11 * t[b.i11];
}

}  // namespace dpcs
