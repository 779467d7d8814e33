/*
 * dpcs_oracle.c -- plain, slow FP64 CPU reference of the DPCS project-and-capture
 * path tracer and of its vector-Jacobian product.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or load
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes (paper Sec. 3):
 *   Eq. 1   PRF       E_p = g_p * I_p^gamma_p (per channel; with an optional 3x3 mixing
 *                     matrix M after the gamma, M = I reduces to Eq. 1)
 *   Eq. 2   L_p = E_p / phi; phi is folded into g_p (the projector is a pinhole
 *                     emitter whose radiant intensity along a direction through image
 *                     point (u,v) is E_p(u,v) / cos^3(alpha))
 *   Eq. 3   rendering equation, direct projector light + indirect interreflection
 *   Eq. 4   pixel value = mean radiance over the pixel footprint (box filter)
 *   Eq. 5   CRF       I_c = (g_c * w * E_c)^gamma_c
 *   Eq. 6   projective geometry x_c = K_c x_s, x_p = K_p [R_p | t_p] x_s (with the
 *                     perspective divide)
 *   Eq. 10  Monte-Carlo estimator with importance-sampled directions
 *   Eq. 12  radiance clipping min(L, k / min(w)) per camera sample
 *   Eq. 9/13 gradients of the rendered image w.r.t. I_p, the BRDF maps, the PRF and
 *            CRF parameters (the adjoint below), for scene fitting and compensation.
 *   Eq. 9   the L1 data term and the map regulariser L(m) with their gradients
 *   Eq. 11  the cross-bilateral denoiser D, its adjoint, and the per-pixel guide
 *            features (first-hit albedo, normal, distance) it is steered by.
 *
 * Structure: every camera sample is traced by a scalar loop; every ray is tested
 * against every triangle (no acceleration structure), the nearest hit wins, equal
 * distances go to the lower triangle index.  Random numbers come from the
 * counter-based Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, SC'11) keyed
 * by the seed and indexed by (pixel, sample, block, 0).
 *
 * The adjoint stores each sample's whole path and differentiates it by a plain
 * reverse sweep (suffix sums from the last vertex), sampling decisions held fixed.
 *
 * Each traced ray also records how far every discrete decision it took was from
 * flipping (edge distances, distance gaps, frustum borders, cosine signs, clip
 * threshold).  A sample whose smallest normalised margin is >= 1 is "clean": on it
 * any correct FP32 implementation must take exactly the same discrete decisions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* scene / parameter description (mirrored by the Python wrapper)            */
/* ------------------------------------------------------------------------- */
typedef struct {
    /* mesh: float32 inputs, read exactly into doubles */
    int32_t nv, nt;
    const float* V;        /* nv*3 */
    const int32_t* F;      /* nt*3 */
    const float* UV;       /* nt*3*2 per-corner texture coordinates */
    const float* Le;       /* nt*3 surface emission (test scenes) or NULL */
    /* camera and projector: world -> device [R|t], intrinsics K (row-major) */
    double Kc[9], Rc[9], tc[3];
    int32_t Wc, Hc;
    double Kp[9], Rp[9], tp[3];
    int32_t Wp, Hp;
    /* BRDF maps (H x W, row-major; albedo has 3 channels) */
    int32_t brdf;          /* 0 Lambert, 1 GGX */
    int32_t tw, th;
    const double* albedo;
    const double* rough;
    const double* spec;
    const double* rough_sample; /* roughness used to sample directions and pdfs (NULL: rough) */
    /* projector input image Hp x Wp x 3 */
    const double* Ip;
    double prf_gamma[3], prf_gain, prf_mix[9];
    double crf_gamma[3], crf_gain, wb[3];
    double env[3];
    int32_t clip;
    double clip_k;
    int32_t spp, max_depth;
    uint64_t seed;
    uint32_t sample_offset;
    int32_t nthreads;
    double tmin;           /* ray epsilon; <= 0 selects 1e-5 * scene diagonal */
    /* the principled BRDF's further maps (Sec. 3.2: theta holds the maps m and the normal
       map v_n; Sec. 4.3 lists base colour, roughness, metallic and the normal map), th x tw:
       metallic (NULL: 0 everywhere) and the normal map (x 3, NULL: none), whose stored
       values in [0, 1] decode to t = 2 v - 1 in the tangent frame of the surface, so
       (0.5, 0.5, 1) leaves the normal unchanged */
    const double* metal;
    const double* nmap;
    const double* nmap_sample; /* normal map whose shading normal samples directions and
                                  pdfs (NULL: nmap); the frozen-path estimator of the tests */
    double edge_density;   /* camera-pose gradient: edge samples per pixel of edge length
                              for the boundary part (0: interior part only) */
} orc_desc;

/* margin scales (see header comment); all margins are divided by these */
#define TAU_X   2e-6   /* x scene diagonal: distance of a hit point to a triangle edge */
#define TAU_T   1e-5   /* relative gap between the two nearest hits */
#define TAU_UV  1e-3   /* projector pixels to the frustum border */
#define TAU_COS 1e-5   /* |cosine| of a sign decision */
#define TAU_CLIP 1e-4  /* relative distance of a sample to the clip threshold */

/* ------------------------------------------------------------------------- */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------- */
void orc_philox(uint64_t seed, const uint32_t ctr_in[4], uint32_t out[4]) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    memcpy(out, c, sizeof c);
}

void orc_philox_batch(uint64_t seed, int64_t n, const uint32_t* ctr, uint32_t* out) {
    for (int64_t i = 0; i < n; ++i) orc_philox(seed, ctr + 4 * i, out + 4 * i);
}

/* four uniforms in [0,1): the top 24 bits of each word times 2^-24 */
static void uniforms(const orc_desc* d, uint32_t pixel, uint32_t sample, uint32_t block, double u[4]) {
    uint32_t c[4] = {pixel, sample + d->sample_offset, block, 0u}, x[4];
    orc_philox(d->seed, c, x);
    for (int i = 0; i < 4; ++i) u[i] = (double)(x[i] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
typedef struct { double x, y, z; } v3;
static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double len(v3 a) { return sqrt(dot(a, a)); }
static v3 nrm(v3 a) { return scl(a, 1.0 / len(a)); }
static v3 matv(const double* M, v3 a) {   /* M a, row-major */
    return mk(M[0] * a.x + M[1] * a.y + M[2] * a.z, M[3] * a.x + M[4] * a.y + M[5] * a.z,
              M[6] * a.x + M[7] * a.y + M[8] * a.z);
}
static v3 mattv(const double* M, v3 a) {  /* M^T a */
    return mk(M[0] * a.x + M[3] * a.y + M[6] * a.z, M[1] * a.x + M[4] * a.y + M[7] * a.z,
              M[2] * a.x + M[5] * a.y + M[8] * a.z);
}
static v3 vtx(const orc_desc* d, int32_t i) {
    return mk(d->V[3 * i], d->V[3 * i + 1], d->V[3 * i + 2]);
}
static double mind(double a, double b) { return a < b ? a : b; }
static double absd(double a) { return a < 0 ? -a : a; }

/* 3x3 inverse by cofactors */
static void inv3(const double* m, double* o) {
    double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7], i = m[8];
    double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    double det = a * A + b * B + c * C;
    o[0] = A / det; o[1] = -(b * i - c * h) / det; o[2] = (b * f - c * e) / det;
    o[3] = B / det; o[4] = (a * i - c * g) / det; o[5] = -(a * f - c * d) / det;
    o[6] = C / det; o[7] = -(a * h - b * g) / det; o[8] = (a * e - b * d) / det;
}

/* ------------------------------------------------------------------------- */
/* ray / triangle (Moller-Trumbore, i.e. Cramer's rule on o + t d = v0 + b1 e1 + b2 e2) */
/* ------------------------------------------------------------------------- */
typedef struct {
    int ok;          /* plane not parallel to the ray */
    double t, b0, b1, b2;
    double edge;     /* signed distance of the plane point to the nearest edge line, metres
                        (>= 0 inside the triangle) */
} tri_isect;

static tri_isect intersect_tri(const orc_desc* d, int32_t prim, v3 o, v3 dir) {
    tri_isect r;
    memset(&r, 0, sizeof r);
    v3 v0 = vtx(d, d->F[3 * prim]), v1 = vtx(d, d->F[3 * prim + 1]), v2 = vtx(d, d->F[3 * prim + 2]);
    v3 e1 = sub(v1, v0), e2 = sub(v2, v0);
    v3 p = cross(dir, e2);
    double det = dot(e1, p);
    if (det == 0.0) return r;
    double inv = 1.0 / det;
    v3 s = sub(o, v0);
    r.b1 = dot(s, p) * inv;
    v3 q = cross(s, e1);
    r.b2 = dot(dir, q) * inv;
    r.t = dot(e2, q) * inv;
    r.b0 = 1.0 - r.b1 - r.b2;
    r.ok = 1;
    /* barycentric b_i times the height over the opposite edge = distance to that edge */
    double area2 = len(cross(e1, e2));
    double h0 = area2 / len(sub(v2, v1)), h1 = area2 / len(e2), h2 = area2 / len(e1);
    r.edge = mind(mind(r.b0 * h0, r.b1 * h1), r.b2 * h2);
    return r;
}

static int inside(const tri_isect* h) { return h->b0 >= 0.0 && h->b1 >= 0.0 && h->b2 >= 0.0; }

typedef struct { double tmin, diag; } scene_scale;

/* Robustness of one triangle's hit decision "inside and t in range": the decision
 * flips only through a component that does not already settle it.  m_e and m_t are
 * the normalised distances of the edge test and of the range test from flipping. */
static double decision_margin(int in, int inr, double m_e, double m_t) {
    if (in && inr) return mind(m_e, m_t);
    if (in) return m_t;
    if (inr) return m_e;
    return m_e > m_t ? m_e : m_t;
}

/* closest hit over (tmin, tmax), skipping `skip`; ties -> lowest index.
 * *margin receives the normalised distance from the nearest decision boundary. */
static int closest_hit(const orc_desc* d, const scene_scale* sc, v3 o, v3 dir, double tmax, int skip,
                       tri_isect* best, double* margin) {
    int bp = -1;
    double bt = tmax;
    for (int32_t p = 0; p < d->nt; ++p) {
        if (p == skip) continue;
        tri_isect h = intersect_tri(d, p, o, dir);
        if (!h.ok || !inside(&h) || !(h.t > sc->tmin) || !(h.t < tmax)) continue;
        if (h.t < bt || (h.t == bt && p < bp)) { bt = h.t; bp = p; *best = h; }
    }
    if (margin) {
        double m = 1e300;
        double tx = TAU_X * sc->diag;
        double tlim = bp >= 0 ? bt : tmax;
        for (int32_t p = 0; p < d->nt; ++p) {
            if (p == skip) continue;
            tri_isect h = intersect_tri(d, p, o, dir);
            if (!h.ok) continue;
            double m_e = absd(h.edge) / tx;
            double m_t = absd(h.t - sc->tmin) / (0.5 * sc->tmin);
            int in = inside(&h), above = h.t > sc->tmin;
            if (p == bp) {
                m = mind(m, mind(m_e, m_t));
            } else if (h.t <= tlim * (1.0 + TAU_T) + tx) {
                /* at or before the nearest hit: could take its place */
                if (in && above)
                    m = mind(m, bp >= 0 ? absd(h.t - bt) / (bt * TAU_T + tx) : 1e300);
                else
                    m = mind(m, decision_margin(in, above, m_e, m_t));
            }
        }
        *margin = m;
    }
    return bp;
}

/* any hit over (tmin, tmax) skipping `skip` */
static int occluded(const orc_desc* d, const scene_scale* sc, v3 o, v3 dir, double tmax, int skip,
                    double* margin) {
    int occ = 0;
    double tx = TAU_X * sc->diag;
    double best_occ = 0.0, m_clear = 1e300;
    for (int32_t p = 0; p < d->nt; ++p) {
        if (p == skip) continue;
        tri_isect h = intersect_tri(d, p, o, dir);
        if (!h.ok) continue;
        double m_e = absd(h.edge) / tx;
        double m_t = mind(absd(h.t - sc->tmin), absd(h.t - tmax)) / (0.5 * sc->tmin);
        int in = inside(&h), inr = h.t > sc->tmin && h.t < tmax;
        double dm = decision_margin(in, inr, m_e, m_t);
        if (in && inr) {
            occ = 1;
            if (dm > best_occ) best_occ = dm;
        } else {
            m_clear = mind(m_clear, dm);
        }
    }
    /* occluded: robust when one occluder is far from all its boundaries;
       clear: robust when every candidate is */
    if (margin) *margin = occ ? best_occ : m_clear;
    return occ;
}

/* ------------------------------------------------------------------------- */
/* texture lookup: bilinear, clamp-to-edge, texel centres at (i + 0.5)       */
/* ------------------------------------------------------------------------- */
typedef struct { int idx[4]; double w[4]; } bilin;

/* x, y in texel units where texel (i, j) has its centre at (i, j) */
static bilin bilinear_at(double x, double y, int W, int H) {
    bilin b;
    double fx = floor(x), fy = floor(y);
    double ax = x - fx, ay = y - fy;
    int x0 = (int)fx, y0 = (int)fy;
    int xs[2] = {x0, x0 + 1}, ys[2] = {y0, y0 + 1};
    for (int k = 0; k < 2; ++k) {
        if (xs[k] < 0) xs[k] = 0;
        if (xs[k] > W - 1) xs[k] = W - 1;
        if (ys[k] < 0) ys[k] = 0;
        if (ys[k] > H - 1) ys[k] = H - 1;
    }
    b.idx[0] = ys[0] * W + xs[0]; b.w[0] = (1 - ax) * (1 - ay);
    b.idx[1] = ys[0] * W + xs[1]; b.w[1] = ax * (1 - ay);
    b.idx[2] = ys[1] * W + xs[0]; b.w[2] = (1 - ax) * ay;
    b.idx[3] = ys[1] * W + xs[1]; b.w[3] = ax * ay;
    return b;
}

/* the projector image's bilinear footprint at projector pixel position (pu, pv), texel
 * centres at half-integer pixel coordinates */
static bilin projector_texels(const orc_desc* d, double pu, double pv) {
    return bilinear_at(pu - 0.5, pv - 0.5, d->Wp, d->Hp);
}

static bilin tex_lookup(const orc_desc* d, double u, double v) {
    return bilinear_at(u * d->tw - 0.5, v * d->th - 0.5, d->tw, d->th);
}

static double fetch1(const double* tex, const bilin* b) {
    double s = 0;
    for (int k = 0; k < 4; ++k) s += b->w[k] * tex[b->idx[k]];
    return s;
}
static void fetch3(const double* tex, const bilin* b, double out[3]) {
    for (int c = 0; c < 3; ++c) {
        out[c] = 0;
        for (int k = 0; k < 4; ++k) out[c] += b->w[k] * tex[3 * b->idx[k] + c];
    }
}

/* ------------------------------------------------------------------------- */
/* BRDF: Lambert, or Lambert + GGX microfacet specular (reduced principled)  */
/* ------------------------------------------------------------------------- */
#define P_SPEC 0.25
#define ALPHA_MIN 1e-3

static double ggx_alpha(double r) { double a = r * r; return a > ALPHA_MIN ? a : ALPHA_MIN; }
static double ggx_dalpha(double r) { return r * r > ALPHA_MIN ? 2.0 * r : 0.0; }

static double ggx_D(double nh, double a) {
    double k = nh * nh * (a * a - 1.0) + 1.0;
    return a * a / (PI * k * k);
}
static double ggx_dD(double nh, double a) {
    double k = nh * nh * (a * a - 1.0) + 1.0;
    return 2.0 * a / (PI * k * k) - a * a * 2.0 * (2.0 * a * nh * nh) / (PI * k * k * k);
}
static double ggx_G1(double c, double a) {
    return 2.0 * c / (c + sqrt(a * a + (1.0 - a * a) * c * c));
}
static double ggx_dG1(double c, double a) {
    double q = sqrt(a * a + (1.0 - a * a) * c * c);
    double dq = a * (1.0 - c * c) / q;
    return -2.0 * c * dq / ((c + q) * (c + q));
}

/* dD/d(n.h) at fixed alpha: D = a^2 / (pi k^2), k = c^2 (a^2 - 1) + 1 */
static double ggx_dD_dc(double c, double a) {
    double k = c * c * (a * a - 1.0) + 1.0;
    return -4.0 * a * a * c * (a * a - 1.0) / (PI * k * k * k);
}
/* dG1/dc at fixed alpha: G1 = 2c / (c + q), q = sqrt(a^2 + (1 - a^2) c^2) */
static double ggx_dG1_dc(double c, double a) {
    double q = sqrt(a * a + (1.0 - a * a) * c * c);
    return 2.0 * a * a / (q * (c + q) * (c + q));
}

/* The principled BRDF with a metallic parameter and a shading normal (Sec. 3.2, Burley's
 * reading): base colour a, metallic mu, roughness r, specular sp,
 *   f_c = (1 - mu) a_c / pi + F_c D G / (4 cos_i cos_o),
 *   F_c = F0_c + (1 - F0_c)(1 - wi.h)^5,  F0_c = (1 - mu) 0.08 sp + mu a_c,
 * with the cosines taken about the shading normal ns.  f = 0 unless wi and wo lie above
 * ns and wi lies above the geometric normal ng (no light through the surface).  The
 * Lambert kind is a_c / pi (metallic does not apply).  Returned with the derivatives the
 * adjoint needs, every one of them of f_c (or of f_c times the cosine c = ns.wi, the
 * factor of the rendering equation, for the normal). */
typedef struct {
    double f[3];     /* f_c */
    double c;        /* ns . wi */
    double dfa;      /* d f_c / d a_c (the same for every channel) */
    double dfr[3];   /* d f_c / d r */
    double dfs;      /* d f_c / d sp (the same for every channel) */
    double dfm[3];   /* d f_c / d mu */
    v3 dfcn[3];      /* d (f_c c) / d ns */
} brdf_full_t;

static brdf_full_t brdf_full(int kind, v3 ng, v3 ns, v3 wo, v3 wi, const double a[3], double r, double sp,
                             double mu) {
    brdf_full_t b;
    memset(&b, 0, sizeof b);
    double ci = dot(ns, wi), co = dot(ns, wo);
    b.c = ci;
    if (ci <= 0.0 || co <= 0.0 || dot(ng, wi) <= 0.0) return b;
    if (kind == 0) {
        b.dfa = 1.0 / PI;
        for (int c = 0; c < 3; ++c) {
            b.f[c] = a[c] / PI;
            b.dfcn[c] = scl(wi, a[c] / PI);
        }
        return b;
    }
    v3 h = nrm(add(wi, wo));
    double nh = dot(ns, h), ih = dot(wi, h);
    double al = ggx_alpha(r), dal = ggx_dalpha(r);
    double D = ggx_D(nh, al), G1i = ggx_G1(ci, al), G1o = ggx_G1(co, al), G = G1i * G1o;
    double m5 = pow(1.0 - ih, 5.0);
    double den = 4.0 * ci * co;
    double DGw = D * G / den;
    double dG = ggx_dG1(ci, al) * G1o + G1i * ggx_dG1(co, al);
    double dDGw_dr = (ggx_dD(nh, al) * G + D * dG) / den * dal;
    /* S = D G / (4 co) = DGw ci: the microfacet part of f_c c without F_c */
    double S = D * G / (4.0 * co);
    v3 dS = add(add(scl(h, ggx_dD_dc(nh, al) * G / (4.0 * co)), scl(wi, D * ggx_dG1_dc(ci, al) * G1o / (4.0 * co))),
                scl(wo, D * G1i * ggx_dG1_dc(co, al) / (4.0 * co) - S / co));
    b.dfa = (1.0 - mu) / PI + mu * (1.0 - m5) * DGw;
    b.dfs = (1.0 - mu) * 0.08 * (1.0 - m5) * DGw;
    for (int c = 0; c < 3; ++c) {
        double F0 = (1.0 - mu) * (0.08 * sp) + mu * a[c];
        double F = F0 + (1.0 - F0) * m5;
        b.f[c] = (1.0 - mu) * a[c] / PI + F * DGw;
        b.dfr[c] = F * dDGw_dr;
        b.dfm[c] = -a[c] / PI + (a[c] - 0.08 * sp) * (1.0 - m5) * DGw;
        b.dfcn[c] = add(scl(wi, (1.0 - mu) * a[c] / PI), scl(dS, F));
    }
    return b;
}

/* mixture pdf of the bounce sampler (solid-angle measure) */
static double bounce_pdf(int kind, v3 n, v3 wo, v3 wi, double r) {
    double ci = dot(n, wi);
    if (kind == 0) return ci > 0 ? ci / PI : 0.0;
    double pd = ci > 0 ? ci / PI : 0.0;
    /* the sampled microfacet normal is +-normalize(wi + wo), whichever faces n */
    v3 h = nrm(add(wi, wo));
    double nh = absd(dot(n, h)), oh = absd(dot(wo, h));
    double ps = (nh > 0 && oh > 0) ? ggx_D(nh, ggx_alpha(r)) * nh / (4.0 * oh) : 0.0;
    return (1.0 - P_SPEC) * pd + P_SPEC * ps;
}

/* orthonormal basis around n (Duff et al., JCGT 2017) */
static void onb(v3 n, v3* b1, v3* b2) {
    double s = n.z >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + n.z);
    double b = n.x * n.y * a;
    *b1 = mk(1.0 + s * n.x * n.x * a, s * b, -s * n.x);
    *b2 = mk(b, s + n.y * n.y * a, -n.y);
}

static v3 to_world(v3 n, double x, double y, double z) {
    v3 b1, b2;
    onb(n, &b1, &b2);
    return add(add(scl(b1, x), scl(b2, y)), scl(n, z));
}

/* cosine-weighted hemisphere about n (Malley's method on the unit disk, polar map) */
static v3 sample_cosine(v3 n, double u1, double u2) {
    double rr = sqrt(u1), phi = 2.0 * PI * u2;
    return to_world(n, rr * cos(phi), rr * sin(phi), sqrt(1.0 - u1));
}

/* GGX normal distribution sampling (Walter et al. 2007): tan^2 theta_h = a^2 u1/(1-u1) */
static v3 sample_ggx_h(v3 n, double r, double u1, double u2) {
    double a = ggx_alpha(r);
    double t2 = a * a * u1 / (1.0 - u1);
    double ct = 1.0 / sqrt(1.0 + t2), st = sqrt(t2) * ct, phi = 2.0 * PI * u2;
    return to_world(n, st * cos(phi), st * sin(phi), ct);
}

static v3 sample_bounce(int kind, v3 n, v3 wo, double r, double ulobe, double u1, double u2) {
    if (kind == 1 && ulobe < P_SPEC) {
        v3 h = sample_ggx_h(n, r, u1, u2);
        return sub(scl(h, 2.0 * dot(wo, h)), wo);
    }
    return sample_cosine(n, u1, u2);
}

/* ------------------------------------------------------------------------- */
/* path record (one entry per surface vertex of a camera sample)             */
/* ------------------------------------------------------------------------- */
typedef struct {
    int prim;
    double beta[3];
    double Le[3];
    bilin tex;                  /* texture footprint of the vertex */
    double alb[3], r, sp, mu;
    /* normal map: tangent frame (T, B, geometric n) and the decoded t / |t|, |t| */
    int nm;
    v3 fT, fB, fN, th;
    double tlen;
    /* projector next-event estimation: BRDF at (wo, wp), bilinear E_p, 1/(cos^3 d^2) */
    int proj;                   /* unoccluded and inside the frustum */
    bilin ptex;                 /* projector image footprint */
    brdf_full_t pf;
    double pE[3], pg0;
    /* environment next-event estimation: BRDF at (wo, we), pi / (sampling cosine) */
    int env;
    brdf_full_t ef;
    double es;
    /* bounce to the next vertex: BRDF at (wo, wi), the sampler's pdf (held fixed) */
    int bounced;
    brdf_full_t bf;
    double bpdf;
    /* the sampled environment and bounce directions (held fixed by the camera-pose
       derivative) */
    v3 we, wi;
} vrec;

typedef struct {
    double L[3];       /* unclipped sample radiance */
    int nv;            /* vertices recorded */
    double margin;     /* forward decisions */
    int reason;        /* which decision set the margin: 10*depth + check id */
} sample_out;

/* check ids: 1 closest hit, 2 facing sign, 3 projector depth, 4 frustum border,
 * 5 projector cosine sign, 6 projector shadow ray, 7 environment shadow ray, 8 bounce sign,
 * with a normal map also 9 outgoing side of the shading normal, 10 environment direction
 * side of the geometric normal, 11 bounce direction side of the shading normal */
static void UPD(sample_out* so, int depth, double m, int check) {
    if (m < so->margin) { so->margin = m; so->reason = 10 * depth + check; }
}

/* Tangent frame of the normal map at a hit (Sec. 3.2: v_n is given relative to the
 * surface normal): T along dP/du of the triangle's texture parameterisation, made
 * orthogonal to the two-sided geometric normal n (the Duff et al. basis when the
 * parameterisation is degenerate), and B = n x T. */
static void tangent_frame(const orc_desc* d, int32_t prim, v3 n, v3* T, v3* B) {
    v3 v0 = vtx(d, d->F[3 * prim]), v1 = vtx(d, d->F[3 * prim + 1]), v2 = vtx(d, d->F[3 * prim + 2]);
    v3 e1 = sub(v1, v0), e2 = sub(v2, v0);
    const float* uv = d->UV + 6 * (size_t)prim;
    double du1 = (double)uv[2] - uv[0], dv1 = (double)uv[3] - uv[1];
    double du2 = (double)uv[4] - uv[0], dv2 = (double)uv[5] - uv[1];
    double det = du1 * dv2 - du2 * dv1;
    v3 t = mk(0, 0, 0);
    if (det != 0.0) {
        v3 dpdu = scl(sub(scl(e1, dv2), scl(e2, dv1)), 1.0 / det);
        t = sub(dpdu, scl(n, dot(n, dpdu)));
    }
    double l = len(t);
    if (l > 0.0) {
        *T = scl(t, 1.0 / l);
    } else {
        v3 b2;
        onb(n, T, &b2);
    }
    *B = cross(n, *T);
}

/* shading normal of the map value v at footprint tb: t = 2 v - 1 in the frame (T, B, n),
 * normalised; n itself when t = 0.  th, tlen receive t / |t| and |t|. */
static v3 shading_normal(const double* map, const bilin* tb, v3 T, v3 B, v3 n, v3* th, double* tlen) {
    double v[3];
    fetch3(map, tb, v);
    v3 t = mk(2.0 * v[0] - 1.0, 2.0 * v[1] - 1.0, 2.0 * v[2] - 1.0);
    double l = len(t);
    if (!(l > 0.0)) {
        *th = mk(0, 0, 1);
        *tlen = 0.0;
        return n;
    }
    *th = scl(t, 1.0 / l);
    *tlen = l;
    return add(add(scl(T, th->x), scl(B, th->y)), scl(n, th->z));
}

typedef struct {
    const orc_desc* d;
    scene_scale sc;
    double Kc_inv[9];
    v3 cam_o, proj_o;
    double* Ep;        /* Hp*Wp*3 projector irradiance after the PRF */
} ctx_t;

/* Eq. 1 (with mixing M): E_p = max(0, g_p * M * max(I_p,0)^gamma_p) per texel */
static void prf_forward(const orc_desc* d, double* Ep) {
    int64_t n = (int64_t)d->Wp * d->Hp;
    for (int64_t t = 0; t < n; ++t) {
        double y[3];
        for (int c = 0; c < 3; ++c) {
            double x = d->Ip[3 * t + c];
            y[c] = x > 0 ? pow(x, d->prf_gamma[c]) : 0.0;
        }
        for (int c = 0; c < 3; ++c) {
            double z = d->prf_gain * (d->prf_mix[3 * c] * y[0] + d->prf_mix[3 * c + 1] * y[1] +
                                      d->prf_mix[3 * c + 2] * y[2]);
            Ep[3 * t + c] = z > 0 ? z : 0.0;
        }
    }
}

static void ctx_init(ctx_t* cx, const orc_desc* d) {
    cx->d = d;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t i = 0; i < d->nv; ++i)
        for (int k = 0; k < 3; ++k) {
            double v = d->V[3 * i + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    cx->sc.diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                       (hi[2] - lo[2]) * (hi[2] - lo[2]));
    cx->sc.tmin = d->tmin > 0 ? d->tmin : 1e-5 * cx->sc.diag;
    inv3(d->Kc, cx->Kc_inv);
    cx->cam_o = scl(mattv(d->Rc, mk(d->tc[0], d->tc[1], d->tc[2])), -1.0);
    cx->proj_o = scl(mattv(d->Rp, mk(d->tp[0], d->tp[1], d->tp[2])), -1.0);
    cx->Ep = (double*)malloc(sizeof(double) * 3 * (size_t)d->Wp * d->Hp);
    prf_forward(d, cx->Ep);
}

static void ctx_free(ctx_t* cx) { free(cx->Ep); }

/* Trace one path that leaves the camera centre along dir (Eq. 3, 10); its random numbers
 * are those of (pixel, s) under cx->d's key.  rec (may be NULL) receives max_depth
 * vertices; hits (may be NULL) receives the hit triangle per vertex (-1 miss, -2 not
 * reached). */
static sample_out trace_path(const ctx_t* cx, v3 dir, int32_t pixel, int32_t s, vrec* rec, int32_t* hits) {
    const orc_desc* d = cx->d;
    sample_out so;
    memset(&so, 0, sizeof so);
    so.margin = 1e300;
    const double tx = TAU_X * cx->sc.diag;
    if (hits)
        for (int k = 0; k < d->max_depth; ++k) hits[k] = -2;
    v3 o = cx->cam_o;
    int skip = -1;
    double beta[3] = {1, 1, 1};
    double* L = so.L;

    for (int depth = 0; depth < d->max_depth; ++depth) {
        tri_isect h;
        double m;
        int prim = closest_hit(d, &cx->sc, o, dir, 1e300, skip, &h, &m);
        UPD(&so, depth, m, 1);
        if (hits) hits[depth] = prim;
        if (prim < 0) {
            /* only a camera ray that escapes sees the environment directly */
            if (depth == 0)
                for (int c = 0; c < 3; ++c) L[c] += beta[c] * d->env[c];
            break;
        }
        vrec* vr = rec ? &rec[depth] : NULL;
        if (vr) {
            memset(vr, 0, sizeof *vr);
            vr->prim = prim;
            for (int c = 0; c < 3; ++c) vr->beta[c] = beta[c];
            so.nv = depth + 1;
        }
        /* hit attributes from barycentrics; flat, two-sided geometric normal */
        int32_t i0 = d->F[3 * prim], i1 = d->F[3 * prim + 1], i2 = d->F[3 * prim + 2];
        v3 v0 = vtx(d, i0), v1 = vtx(d, i1), v2 = vtx(d, i2);
        v3 x = add(add(scl(v0, h.b0), scl(v1, h.b1)), scl(v2, h.b2));
        v3 n = nrm(cross(sub(v1, v0), sub(v2, v0)));
        v3 wo = scl(dir, -1.0);
        double ndo = dot(n, wo);
        UPD(&so, depth, absd(ndo) / TAU_COS, 2);
        if (ndo < 0) { n = scl(n, -1.0); ndo = -ndo; }
        const float* uvp = d->UV + 6 * (size_t)prim;
        double tu = h.b0 * uvp[0] + h.b1 * uvp[2] + h.b2 * uvp[4];
        double tv = h.b0 * uvp[1] + h.b1 * uvp[3] + h.b2 * uvp[5];
        bilin tb = tex_lookup(d, tu, tv);
        double alb[3], r = 0, sp = 0, rs = 0, mu = 0;
        fetch3(d->albedo, &tb, alb);
        if (d->brdf == 1) {
            r = fetch1(d->rough, &tb);
            sp = fetch1(d->spec, &tb);
            rs = d->rough_sample ? fetch1(d->rough_sample, &tb) : r;
            if (d->metal) mu = fetch1(d->metal, &tb);
        }
        /* shading normal (evaluation) and the one that samples directions and pdfs */
        v3 ns = n, nss = n, fT = n, fB = n, th = mk(0, 0, 1);
        double tlen = 0.0;
        if (d->nmap) {
            tangent_frame(d, prim, n, &fT, &fB);
            ns = shading_normal(d->nmap, &tb, fT, fB, n, &th, &tlen);
            if (d->nmap_sample) {
                v3 th2;
                double tl2;
                nss = shading_normal(d->nmap_sample, &tb, fT, fB, n, &th2, &tl2);
            } else {
                nss = ns;
            }
            UPD(&so, depth, absd(dot(ns, wo)) / TAU_COS, 9);
        }
        if (vr) {
            vr->tex = tb;
            for (int c = 0; c < 3; ++c) vr->alb[c] = alb[c];
            vr->r = r;
            vr->sp = sp;
            vr->mu = mu;
            vr->nm = d->nmap != NULL;
            vr->fT = fT;
            vr->fB = fB;
            vr->fN = n;
            vr->th = th;
            vr->tlen = tlen;
        }

        /* surface emission (white-furnace test scenes only) */
        if (d->Le) {
            for (int c = 0; c < 3; ++c) {
                double e = d->Le[3 * prim + c];
                L[c] += beta[c] * e;
                if (vr) vr->Le[c] = e;
            }
        }

        /* next-event estimation toward the projector (Eq. 2, 3, 6) */
        {
            v3 xp = add(matv(d->Rp, x), mk(d->tp[0], d->tp[1], d->tp[2]));
            UPD(&so, depth, absd(xp.z) / tx, 3);
            if (xp.z > 0) {
                double pu = (d->Kp[0] * xp.x + d->Kp[1] * xp.y + d->Kp[2] * xp.z) / xp.z;
                double pv = (d->Kp[3] * xp.x + d->Kp[4] * xp.y + d->Kp[5] * xp.z) / xp.z;
                double bu = mind(mind(absd(pu), absd(d->Wp - pu)), mind(absd(pv), absd(d->Hp - pv)));
                UPD(&so, depth, bu / TAU_UV, 4);
                if (pu >= 0 && pu < d->Wp && pv >= 0 && pv < d->Hp) {
                    v3 tow = sub(cx->proj_o, x);
                    double dist = len(tow);
                    v3 wp = scl(tow, 1.0 / dist);
                    double cp = dot(n, wp);
                    UPD(&so, depth, absd(cp) / TAU_COS, 5);
                    if (d->nmap) UPD(&so, depth, absd(dot(ns, wp)) / TAU_COS, 5);
                    if (cp > 0) {
                        double mo;
                        int occ = occluded(d, &cx->sc, x, wp, dist - cx->sc.tmin, prim, &mo);
                        UPD(&so, depth, mo, 6);
                        if (!occ) {
                            bilin pb = projector_texels(d, pu, pv);
                            double E[3];
                            fetch3(cx->Ep, &pb, E);
                            double ca = xp.z / len(xp);              /* cos alpha off the axis */
                            brdf_full_t fb = brdf_full(d->brdf, n, ns, wo, wp, alb, r, sp, mu);
                            /* the cosine of the rendering equation is taken about ns */
                            double geom = fb.c / (ca * ca * ca * dist * dist);
                            for (int c = 0; c < 3; ++c) L[c] += beta[c] * fb.f[c] * E[c] * geom;
                            if (vr) {
                                vr->proj = 1;
                                vr->ptex = pb;
                                vr->pf = fb;
                                vr->pg0 = 1.0 / (ca * ca * ca * dist * dist);
                                for (int c = 0; c < 3; ++c) vr->pE[c] = E[c];
                            }
                        }
                    }
                }
            }
        }

        /* next-event estimation toward a constant environment (only if it is non-zero):
           direction cosine-distributed about the sampling normal, pdf = cos / pi */
        if (d->env[0] != 0 || d->env[1] != 0 || d->env[2] != 0) {
            double ue[4];
            uniforms(d, (uint32_t)pixel, (uint32_t)s, 2u + 2u * depth, ue);
            v3 we = sample_cosine(nss, ue[0], ue[1]);
            if (d->nmap) UPD(&so, depth, absd(dot(n, we)) / TAU_COS, 10);
            double mo;
            int occ = occluded(d, &cx->sc, x, we, 1e300, prim, &mo);
            UPD(&so, depth, mo, 7);
            if (!occ) {
                brdf_full_t fb = brdf_full(d->brdf, n, ns, wo, we, alb, r, sp, mu);
                /* f * L_env * cos / (cos_sample / pi): pi when both normals are the same */
                double es = d->nmap_sample ? PI * fb.c / dot(nss, we) : PI;
                for (int c = 0; c < 3; ++c) L[c] += beta[c] * fb.f[c] * d->env[c] * es;
                if (vr) {
                    vr->env = 1;
                    vr->we = we;
                    vr->ef = fb;
                    vr->es = d->nmap_sample ? PI / dot(nss, we) : (fb.c > 0 ? PI / fb.c : 0.0);
                }
            }
        }

        if (depth == d->max_depth - 1) break;

        /* bounce: sample a direction, pdf and lobe choice held fixed (detached); the path
           goes on while the direction leaves above the geometric surface */
        double ub[4];
        uniforms(d, (uint32_t)pixel, (uint32_t)s, 1u + 2u * depth, ub);
        v3 wi = sample_bounce(d->brdf, nss, wo, rs, ub[0], ub[1], ub[2]);
        double ci = dot(n, wi);
        UPD(&so, depth, absd(ci) / TAU_COS, 8);
        if (d->nmap) UPD(&so, depth, absd(dot(ns, wi)) / TAU_COS, 11);
        double pdf = bounce_pdf(d->brdf, nss, wo, wi, rs);
        if (ci <= 0 || pdf <= 0) break;
        brdf_full_t fb = brdf_full(d->brdf, n, ns, wo, wi, alb, r, sp, mu);
        double w = fb.c / pdf;
        for (int c = 0; c < 3; ++c) beta[c] *= fb.f[c] * w;
        if (vr) {
            vr->bounced = 1;
            vr->wi = wi;
            vr->bf = fb;
            vr->bpdf = pdf;
        }
        o = x;
        dir = wi;
        skip = prim;
    }
    return so;
}

/* Trace one camera sample: the ray through the jittered pixel position (Eq. 6 inverted). */
static sample_out trace_sample(const ctx_t* cx, int32_t pixel, int32_t s, vrec* rec, int32_t* hits) {
    const orc_desc* d = cx->d;
    int32_t i = pixel % d->Wc, j = pixel / d->Wc;
    double u[4];
    uniforms(d, (uint32_t)pixel, (uint32_t)s, 0u, u);
    v3 dir = nrm(mattv(d->Rc, matv(cx->Kc_inv, mk(i + u[0], j + u[1], 1.0))));
    return trace_path(cx, dir, pixel, s, rec, hits);
}

/* The camera vertex's radiance for a camera pose (R, t) other than the forward's (Sec.
 * 3.2: R_c, t_c are part of theta and refined with it), everything the forward decided
 * held at its value: the camera ray of the same jittered pixel position meets the plane of
 * the forward's triangle at x; the projector term is evaluated there in full (texture and
 * normal map at the new texture coordinates, projector coordinates, distance, cosines,
 * BRDF toward the camera), while the environment and bounce terms keep their sampled
 * directions and remaining factors Se = L_env pi / c_sample and Sb = R_1 / pdf.  Its
 * derivative w.r.t. (R, t) is the interior part of the camera-pose gradient: the
 * visibility decisions and the later vertices of the path are held fixed. */
static void camera_vertex(const ctx_t* cx, int32_t pixel, int32_t s, const double* Rc, const double* tc,
                          const vrec* v, const double Se[3], const double Sb[3], double out[3]) {
    const orc_desc* d = cx->d;
    int32_t i = pixel % d->Wc, j = pixel / d->Wc;
    double u[4];
    uniforms(d, (uint32_t)pixel, (uint32_t)s, 0u, u);
    v3 dir = nrm(mattv(Rc, matv(cx->Kc_inv, mk(i + u[0], j + u[1], 1.0))));
    v3 o = scl(mattv(Rc, mk(tc[0], tc[1], tc[2])), -1.0);
    int32_t prim = v->prim;
    v3 v0 = vtx(d, d->F[3 * prim]), v1 = vtx(d, d->F[3 * prim + 1]), v2 = vtx(d, d->F[3 * prim + 2]);
    v3 e1 = sub(v1, v0), e2 = sub(v2, v0);
    v3 n = v->fN;                                        /* the forward's two-sided normal */
    v3 x = add(o, scl(dir, dot(n, sub(v0, o)) / dot(n, dir)));
    /* barycentrics of x in the triangle's plane (normal equations of x - v0 = b1 e1 + b2 e2) */
    v3 p = sub(x, v0);
    double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2), r1 = dot(p, e1), r2 = dot(p, e2);
    double den = a11 * a22 - a12 * a12;
    double b1 = (a22 * r1 - a12 * r2) / den, b2 = (a11 * r2 - a12 * r1) / den, b0 = 1.0 - b1 - b2;
    const float* uvp = d->UV + 6 * (size_t)prim;
    bilin tb = tex_lookup(d, b0 * uvp[0] + b1 * uvp[2] + b2 * uvp[4], b0 * uvp[1] + b1 * uvp[3] + b2 * uvp[5]);
    double alb[3], r = 0, sp = 0, mu = 0;
    fetch3(d->albedo, &tb, alb);
    if (d->brdf == 1) {
        r = fetch1(d->rough, &tb);
        sp = fetch1(d->spec, &tb);
        if (d->metal) mu = fetch1(d->metal, &tb);
    }
    v3 ns = n;
    if (d->nmap) {
        v3 th;
        double tlen;
        ns = shading_normal(d->nmap, &tb, v->fT, v->fB, n, &th, &tlen);
    }
    v3 wo = scl(dir, -1.0);
    for (int c = 0; c < 3; ++c) out[c] = 0.0;
    if (v->proj) {
        v3 xp = add(matv(d->Rp, x), mk(d->tp[0], d->tp[1], d->tp[2]));
        double pu = (d->Kp[0] * xp.x + d->Kp[1] * xp.y + d->Kp[2] * xp.z) / xp.z;
        double pv = (d->Kp[3] * xp.x + d->Kp[4] * xp.y + d->Kp[5] * xp.z) / xp.z;
        v3 tow = sub(cx->proj_o, x);
        double dist = len(tow);
        v3 wp = scl(tow, 1.0 / dist);
        bilin pb = projector_texels(d, pu, pv);
        double E[3];
        fetch3(cx->Ep, &pb, E);
        double ca = xp.z / len(xp);
        brdf_full_t fb = brdf_full(d->brdf, n, ns, wo, wp, alb, r, sp, mu);
        for (int c = 0; c < 3; ++c) out[c] += fb.f[c] * fb.c * E[c] / (ca * ca * ca * dist * dist);
    }
    if (v->env) {
        brdf_full_t fb = brdf_full(d->brdf, n, ns, wo, v->we, alb, r, sp, mu);
        for (int c = 0; c < 3; ++c) out[c] += fb.f[c] * fb.c * Se[c];
    }
    if (v->bounced) {
        brdf_full_t fb = brdf_full(d->brdf, n, ns, wo, v->wi, alb, r, sp, mu);
        for (int c = 0; c < 3; ++c) out[c] += fb.f[c] * fb.c * Sb[c];
    }
}

/* central-difference step of the camera-pose derivative (entries of R and t) */
#define CAM_FD_H 1e-7

static double clip_threshold(const orc_desc* d, int* argmin) {
    int a = 0;
    for (int c = 1; c < 3; ++c)
        if (d->wb[c] < d->wb[a]) a = c;
    if (argmin) *argmin = a;
    return d->clip_k / d->wb[a];
}

/* Eq. 5 */
static double crf(const orc_desc* d, int c, double Ec) {
    double y = d->crf_gain * d->wb[c] * Ec;
    return y > 0 ? pow(y, d->crf_gamma[c]) : 0.0;
}

static int nthreads_of(const orc_desc* d) {
#ifdef _OPENMP
    return d->nthreads > 0 ? d->nthreads : omp_get_max_threads();
#else
    (void)d;
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* camera pose: the boundary part at the images of mesh edges                 */
/* ------------------------------------------------------------------------- */
/* A pixel (i, j) is the integral of the sample radiance over the square [i, i+1] x
 * [j, j+1] of image coordinates x = (K X)_{1,2} / (K X)_3, X = R_c P + t_c (the uniform
 * jitter of the camera samples, Eq. 6).  Where the radiance jumps along a curve of the
 * image, moving the camera moves the curve, and the pixel's integral changes by the jump
 * times the curve's normal speed: d I / d theta gains the line integral of
 * (f- - f+) (n . dx/dtheta) over the curve's part inside the pixel, n the unit normal
 * toward the f+ side (Reynolds transport).  The curves taken here are the images of the
 * mesh edges across which the first surface seen changes discontinuously (vertices of
 * triangles at the same position are one vertex here, and faces of no area take no part):
 *   - edges of one face, or of three or more faces;
 *   - edges whose two faces are not coplanar: creases, and every silhouette edge (two
 *     faces that meet at a silhouette as seen from the camera centre, i.e. lie on one side
 *     of the plane through it and the edge, are never coplanar unless folded flat);
 *   - coplanar faces folded onto one side of the edge;
 *   - seams: the texture coordinates or the emission differ across the edge.
 * Shadow and projector-frustum boundaries on the surfaces are not among them.
 * Each such edge, clipped to w >= tmin in front of the camera and to the image, gets
 * n_e = ceil(density * l_e) stratified points, l_e its length in pixels: point k at
 * (k + u) / n_e along the clipped segment, weight l_e / n_e; f-, f+ are the sample
 * radiances (clipped as in Eq. 12) of two paths through x -/+ EDGE_EPS n that share the
 * point's random numbers.  Edge samples are numbered over the edges in order of (lower,
 * higher welded vertex index, a vertex's welded index being the lowest index at its
 * position); sample k draws its uniforms from counter (k, 0, block, 0) under
 * the key seed ^ EDGE_KEY (u is the first of block 0). */
#define EDGE_EPS 1e-2
#define EDGE_KEY 0x9E3779B97F4A7C15ull

typedef struct { int32_t a, b, f0, f1, nf; } orc_edge;   /* a < b; f1 only when nf == 2 */

static int cmp_edge_key(const void* x, const void* y) {
    const int32_t* p = (const int32_t*)x;
    const int32_t* q = (const int32_t*)y;
    for (int k = 0; k < 3; ++k)
        if (p[k] != q[k]) return p[k] < q[k] ? -1 : 1;
    return 0;
}

typedef struct { float p[3]; int32_t i; } vpos_t;
static int cmp_vertex_pos(const void* x, const void* y) {
    const vpos_t* a = (const vpos_t*)x;
    const vpos_t* b = (const vpos_t*)y;
    for (int k = 0; k < 3; ++k)
        if (a->p[k] != b->p[k]) return a->p[k] < b->p[k] ? -1 : 1;
    return a->i < b->i ? -1 : (a->i > b->i);
}

/* canonical vertex of each vertex that a triangle uses: the lowest such index at the same
 * position (a mesh that repeats vertices per face still has one edge where two faces
 * meet); vertices no triangle uses take no part */
static int32_t* weld_vertices(const orc_desc* d) {
    char* used = (char*)calloc((size_t)d->nv, 1);
    for (int64_t k = 0; k < 3 * (int64_t)d->nt; ++k) used[d->F[k]] = 1;
    vpos_t* v = (vpos_t*)malloc(sizeof(vpos_t) * (size_t)d->nv);
    int32_t* canon = (int32_t*)malloc(sizeof(int32_t) * (size_t)d->nv);
    int32_t n = 0;
    for (int32_t i = 0; i < d->nv; ++i) {
        canon[i] = i;
        if (!used[i]) continue;
        for (int k = 0; k < 3; ++k) v[n].p[k] = d->V[3 * (size_t)i + k];
        v[n++].i = i;
    }
    qsort(v, (size_t)n, sizeof(vpos_t), cmp_vertex_pos);
    for (int32_t i = 0; i < n; ++i) {
        int same = i && v[i].p[0] == v[i - 1].p[0] && v[i].p[1] == v[i - 1].p[1] && v[i].p[2] == v[i - 1].p[2];
        canon[v[i].i] = same ? canon[v[i - 1].i] : v[i].i;
    }
    free(v);
    free(used);
    return canon;
}

/* does the triangle cover any area?  (exact: the cross product of float differences is
 * computed without rounding in double) */
static int has_area(const orc_desc* d, int32_t f) {
    v3 a = vtx(d, d->F[3 * f]), b = vtx(d, d->F[3 * f + 1]), c = vtx(d, d->F[3 * f + 2]);
    v3 m = cross(sub(b, a), sub(c, a));
    return m.x != 0 || m.y != 0 || m.z != 0;
}

/* the unique edges of the mesh's faces of non-zero area with those faces, sorted by
 * (a, b), over welded vertices (a face of no area is never seen, so it bounds nothing) */
static orc_edge* mesh_edges(const orc_desc* d, const int32_t* canon, int64_t* ne) {
    int32_t* key = (int32_t*)malloc(sizeof(int32_t) * 9 * (size_t)d->nt);
    int64_t nk = 0;
    for (int32_t f = 0; f < d->nt; ++f)
        if (has_area(d, f))
            for (int k = 0; k < 3; ++k) {
                int32_t u = canon[d->F[3 * f + k]], v = canon[d->F[3 * f + (k + 1) % 3]];
                int32_t* e = key + 3 * nk++;
                e[0] = u < v ? u : v;
                e[1] = u < v ? v : u;
                e[2] = f;
            }
    qsort(key, (size_t)nk, 3 * sizeof(int32_t), cmp_edge_key);
    orc_edge* E = (orc_edge*)malloc(sizeof(orc_edge) * ((size_t)nk + 1));
    int64_t n = 0;
    for (int64_t i = 0; i < nk;) {
        int64_t j = i;
        while (j < nk && key[3 * j] == key[3 * i] && key[3 * j + 1] == key[3 * i + 1]) ++j;
        orc_edge e = {key[3 * i], key[3 * i + 1], key[3 * i + 2], j - i > 1 ? key[3 * i + 5] : -1, (int32_t)(j - i)};
        E[n++] = e;
        i = j;
    }
    free(key);
    *ne = n;
    return E;
}

static int corner_of(const orc_desc* d, const int32_t* canon, int32_t f, int32_t v) {
    for (int k = 0; k < 3; ++k)
        if (canon[d->F[3 * f + k]] == v) return k;
    return -1;
}

/* does the first surface seen change discontinuously across the edge's image? */
static int edge_is_discontinuous(const ctx_t* cx, const int32_t* canon, const orc_edge* e) {
    const orc_desc* d = cx->d;
    if (e->nf != 2) return 1;
    v3 A = vtx(d, e->a), B = vtx(d, e->b);
    int a0 = corner_of(d, canon, e->f0, e->a), b0 = corner_of(d, canon, e->f0, e->b);
    int a1 = corner_of(d, canon, e->f1, e->a), b1 = corner_of(d, canon, e->f1, e->b);
    v3 C0 = vtx(d, d->F[3 * e->f0 + 3 - a0 - b0]), C1 = vtx(d, d->F[3 * e->f1 + 3 - a1 - b1]);
    /* faces at an angle: a crease, or a silhouette from where the camera is */
    v3 n0 = nrm(cross(sub(B, A), sub(C0, A))), n1 = nrm(cross(sub(B, A), sub(C1, A)));
    if (len(cross(n0, n1)) > 1e-9) return 1;
    /* coplanar faces folded onto the same side of the edge */
    if (dot(sub(C0, A), sub(C1, A)) - dot(sub(C0, A), sub(B, A)) * dot(sub(C1, A), sub(B, A)) / dot(sub(B, A), sub(B, A)) > 0)
        return 1;
    const float* u0 = d->UV + 6 * (size_t)e->f0;
    const float* u1 = d->UV + 6 * (size_t)e->f1;
    if (u0[2 * a0] != u1[2 * a1] || u0[2 * a0 + 1] != u1[2 * a1 + 1] || u0[2 * b0] != u1[2 * b1] ||
        u0[2 * b0 + 1] != u1[2 * b1 + 1])
        return 1;
    if (d->Le)
        for (int c = 0; c < 3; ++c)
            if (d->Le[3 * e->f0 + c] != d->Le[3 * e->f1 + c]) return 1;
    return 0;
}

/* the edge's image, clipped: 3D end points A1, B1 with homogeneous depths wA, wB and
 * their image points; the kept part of the image segment is lambda in [l0, l1] */
typedef struct {
    v3 A1, B1;
    double wA, wB, ax, ay, dx, dy, l0, l1, len;
} edge_clip;

static v3 homog(const orc_desc* d, v3 P) {
    return matv(d->Kc, add(matv(d->Rc, P), mk(d->tc[0], d->tc[1], d->tc[2])));
}

static int clip_edge(const ctx_t* cx, const orc_edge* e, edge_clip* c) {
    const orc_desc* d = cx->d;
    v3 A = vtx(d, e->a), B = vtx(d, e->b);
    v3 hA = homog(d, A), hB = homog(d, B);
    double wmin = cx->sc.tmin, s0 = 0, s1 = 1;
    if (hA.z < wmin && hB.z < wmin) return 0;
    if (hA.z < wmin) s0 = (wmin - hA.z) / (hB.z - hA.z);
    if (hB.z < wmin) s1 = (wmin - hA.z) / (hB.z - hA.z);
    c->A1 = add(A, scl(sub(B, A), s0));
    c->B1 = add(A, scl(sub(B, A), s1));
    v3 gA = add(hA, scl(sub(hB, hA), s0)), gB = add(hA, scl(sub(hB, hA), s1));
    c->wA = gA.z;
    c->wB = gB.z;
    c->ax = gA.x / gA.z;
    c->ay = gA.y / gA.z;
    c->dx = gB.x / gB.z - c->ax;
    c->dy = gB.y / gB.z - c->ay;
    /* Liang-Barsky against [0, Wc] x [0, Hc] */
    double p[4] = {-c->dx, c->dx, -c->dy, c->dy};
    double q[4] = {c->ax, d->Wc - c->ax, c->ay, d->Hc - c->ay};
    double l0 = 0, l1 = 1;
    for (int k = 0; k < 4; ++k) {
        if (p[k] == 0) {
            if (q[k] < 0) return 0;
        } else {
            double r = q[k] / p[k];
            if (p[k] < 0) {
                if (r > l0) l0 = r;
            } else if (r < l1) {
                l1 = r;
            }
        }
    }
    if (!(l0 < l1)) return 0;
    c->l0 = l0;
    c->l1 = l1;
    c->len = (l1 - l0) * sqrt(c->dx * c->dx + c->dy * c->dy);
    return c->len > 0;
}

static int64_t edge_samples(const ctx_t* cx, const int32_t* canon, const orc_edge* e, double density,
                            edge_clip* c) {
    if (!edge_is_discontinuous(cx, canon, e) || !clip_edge(cx, e, c)) return 0;
    return (int64_t)ceil(density * c->len);
}

/* The boundary part of d loss / d(R_c, t_c) (out12: R row-major, then t) for the
 * per-pixel cotangents dE (Hc x Wc x 3) of the pixel means of the clipped sample
 * radiance.  Per-edge sums are added in edge order. */
int orc_camera_boundary(const orc_desc* d, const double* dE, double* out12, int64_t* n_samples) {
    ctx_t cx;
    ctx_init(&cx, d);
    orc_desc de = *d;
    de.seed = d->seed ^ EDGE_KEY;
    de.sample_offset = 0;
    ctx_t ce = cx;
    ce.d = &de;
    int64_t ne;
    int32_t* canon = weld_vertices(d);
    orc_edge* E = mesh_edges(d, canon, &ne);
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne + 1));
    off[0] = 0;
    for (int64_t i = 0; i < ne; ++i) {
        edge_clip c;
        off[i + 1] = off[i] + edge_samples(&cx, canon, &E[i], d->edge_density, &c);
    }
    double* per = (double*)calloc(12 * (size_t)ne, sizeof(double));
    double thr = clip_threshold(d, NULL);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_of(d))
    for (int64_t i = 0; i < ne; ++i) {
        edge_clip c;
        int64_t n = edge_samples(&cx, canon, &E[i], d->edge_density, &c);
        if (n == 0) continue;
        double el = sqrt(c.dx * c.dx + c.dy * c.dy);
        double nx = -c.dy / el, ny = c.dx / el;     /* unit normal toward the f+ side */
        for (int64_t k = 0; k < n; ++k) {
            uint32_t gk = (uint32_t)(off[i] + k);
            double u[4];
            uniforms(&de, gk, 0u, 0u, u);
            double lam = c.l0 + (c.l1 - c.l0) * ((double)k + u[0]) / (double)n;
            double x = c.ax + lam * c.dx, y = c.ay + lam * c.dy;
            double mu = lam * c.wA / (lam * c.wA + (1.0 - lam) * c.wB);
            v3 P = add(c.A1, scl(sub(c.B1, c.A1), mu));
            int32_t pi = (int32_t)floor(x), pj = (int32_t)floor(y);
            if (pi > d->Wc - 1) pi = d->Wc - 1;
            if (pj > d->Hc - 1) pj = d->Hc - 1;
            if (pi < 0) pi = 0;
            if (pj < 0) pj = 0;
            const double* g = dE + 3 * ((size_t)pj * d->Wc + pi);
            if (g[0] == 0 && g[1] == 0 && g[2] == 0) continue;
            double f[2][3];
            for (int side = 0; side < 2; ++side) {
                double sg = side ? EDGE_EPS : -EDGE_EPS;
                v3 dir = nrm(mattv(d->Rc, matv(cx.Kc_inv, mk(x + sg * nx, y + sg * ny, 1.0))));
                sample_out so = trace_path(&ce, dir, (int32_t)gk, 0, NULL, NULL);
                for (int ch = 0; ch < 3; ++ch) f[side][ch] = d->clip && so.L[ch] > thr ? thr : so.L[ch];
            }
            double J = 0;
            for (int ch = 0; ch < 3; ++ch) J += g[ch] * (f[0][ch] - f[1][ch]);
            J *= c.len / (double)n;
            /* image speed of the edge point: dx/dR_ij = c_i P_j, dx/dt_i = c_i with
               c_i = (K_{.i} - x K_{3i}) / w over the image rows */
            v3 h = homog(d, P);
            double Pj[3] = {P.x, P.y, P.z};
            for (int r = 0; r < 3; ++r) {
                double ci_x = (d->Kc[r] - x * d->Kc[6 + r]) / h.z;
                double ci_y = (d->Kc[3 + r] - y * d->Kc[6 + r]) / h.z;
                double a = nx * ci_x + ny * ci_y;
                for (int j = 0; j < 3; ++j) per[12 * (size_t)i + 3 * r + j] += J * a * Pj[j];
                per[12 * (size_t)i + 9 + r] += J * a;
            }
        }
    }
    for (int k = 0; k < 12; ++k) out12[k] = 0;
    for (int64_t i = 0; i < ne; ++i)
        for (int k = 0; k < 12; ++k) out12[k] += per[12 * (size_t)i + k];
    if (n_samples) *n_samples = off[ne];
    free(per);
    free(off);
    free(E);
    free(canon);
    ctx_free(&cx);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* forward render of a set of pixels                                           */
/*   pixels: npix pixel indices (j*Wc + i), or NULL for all Wc*Hc in order     */
/*   out_Ec/out_Ic: npix*3; out_L: npix*spp*3 unclipped sample radiance;       */
/*   out_hits: npix*spp*max_depth; out_margin: npix*spp; out_margin_clip:      */
/*   npix*spp (forward margin combined with the clip-threshold margin);        */
/*   out_reason: npix*spp, which decision set the forward margin               */
/* ------------------------------------------------------------------------- */
int orc_render(const orc_desc* d, int32_t npix, const int32_t* pixels, double* out_Ec, double* out_Ic,
               double* out_L, int32_t* out_hits, double* out_margin, double* out_margin_clip,
               int32_t* out_reason) {
    ctx_t cx;
    ctx_init(&cx, d);
    int thr_arg;
    double thr = clip_threshold(d, &thr_arg);
    int nth = nthreads_of(d);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
    for (int32_t q = 0; q < npix; ++q) {
        int32_t pixel = pixels ? pixels[q] : q;
        double acc[3] = {0, 0, 0};
        for (int32_t s = 0; s < d->spp; ++s) {
            int64_t sid = (int64_t)q * d->spp + s;
            sample_out so = trace_sample(&cx, pixel, s, NULL,
                                         out_hits ? out_hits + sid * d->max_depth : NULL);
            double mclip = so.margin;
            for (int c = 0; c < 3; ++c) {
                double v = so.L[c];
                if (out_L) out_L[3 * sid + c] = v;
                if (d->clip) {
                    mclip = mind(mclip, absd(v - thr) / (thr * TAU_CLIP));
                    if (v > thr) v = thr;   /* Eq. 12 */
                }
                acc[c] += v;
            }
            if (out_margin) out_margin[sid] = so.margin;
            if (out_reason) out_reason[sid] = so.reason;
            if (out_margin_clip) out_margin_clip[sid] = mclip;
        }
        for (int c = 0; c < 3; ++c) {
            double Ec = acc[c] / d->spp;   /* Eq. 4 as a box-filtered mean */
            if (out_Ec) out_Ec[3 * q + c] = Ec;
            if (out_Ic) out_Ic[3 * q + c] = crf(d, c, Ec);
        }
    }
    ctx_free(&cx);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* vector-Jacobian product                                                    */
/*   G: Hc*Wc*3 cotangent of I_c.  Only the listed pixels (NULL: all) are     */
/*   differentiated, i.e. G is taken as zero elsewhere.                       */
/*   Outputs are overwritten (any may be NULL):                                */
/*     d_Ip Hp*Wp*3, d_albedo th*tw*3, d_rough th*tw, d_spec th*tw,            */
/*     d_scalars[18] = gamma_p(3), M(9 row-major), gamma_c(3), w(3),           */
/*     d_metal th*tw, d_nmap th*tw*3 (the stored normal-map values)            */
/*   d_Ep (optional, Hp*Wp*3) receives the cotangent of E_p before the PRF.    */
/* ------------------------------------------------------------------------- */
int orc_render_vjp(const orc_desc* d, const double* G, int32_t npix, const int32_t* pixels,
                   double* d_Ip, double* d_albedo, double* d_rough, double* d_spec, double* d_scalars,
                   double* d_Ep_out, double* d_metal, double* d_nmap, double* d_cam) {
    ctx_t cx;
    ctx_init(&cx, d);
    int thr_arg;
    double thr = clip_threshold(d, &thr_arg);
    int nth = nthreads_of(d);
    size_t nEp = 3 * (size_t)d->Wp * d->Hp, nT = (size_t)d->tw * d->th;
    /* per-thread accumulators: dEp, dalb (3), drough, dspec, dmetal, dnmap (3), 6 CRF
       scalars, 1 threshold, 12 camera-pose entries (R row-major, t) */
    size_t per = nEp + 3 * nT + nT + nT + nT + 3 * nT + 7 + 12;
    double* acc = (double*)calloc((size_t)nth * per, sizeof(double));
    int npix_all = d->Wc * d->Hc;
    if (!pixels) npix = npix_all;
    /* per-pixel cotangents of the clipped pixel means (the camera pose's boundary part) */
    double* dE_pix = d_cam && d->edge_density > 0 ? (double*)calloc(3 * (size_t)npix_all, sizeof(double)) : NULL;

#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* a = acc + (size_t)tid * per;
        double* gEp = a;
        double* galb = gEp + nEp;
        double* grough = galb + 3 * nT;
        double* gspec = grough + nT;
        double* gmetal = gspec + nT;
        double* gnmap = gmetal + nT;
        double* gsc = gnmap + 3 * nT;  /* gamma_c(3), w(3), threshold(1) */
        double* gcam = gsc + 7;
        vrec* rec = (vrec*)malloc(sizeof(vrec) * (size_t)d->spp * d->max_depth);
        sample_out* so = (sample_out*)malloc(sizeof(sample_out) * (size_t)d->spp);
#pragma omp for schedule(dynamic, 1)
        for (int32_t q = 0; q < npix; ++q) {
            int32_t pixel = pixels ? pixels[q] : q;
            /* forward for this pixel */
            double Ec[3] = {0, 0, 0};
            for (int32_t s = 0; s < d->spp; ++s) {
                so[s] = trace_sample(&cx, pixel, s, rec + (size_t)s * d->max_depth, NULL);
                for (int c = 0; c < 3; ++c) {
                    double v = so[s].L[c];
                    if (d->clip && v > thr) v = thr;
                    Ec[c] += v;
                }
            }
            for (int c = 0; c < 3; ++c) Ec[c] /= d->spp;
            /* CRF backward (Eq. 5): y = g_c w E_c, I_c = y^gamma_c */
            double dEc[3];
            for (int c = 0; c < 3; ++c) {
                double g = G[3 * (size_t)pixel + c];
                double y = d->crf_gain * d->wb[c] * Ec[c];
                dEc[c] = 0;
                if (y > 0 && g != 0) {
                    double gc = d->crf_gamma[c];
                    double dy = g * gc * pow(y, gc - 1.0);
                    dEc[c] = dy * d->crf_gain * d->wb[c];
                    gsc[c] += g * pow(y, gc) * log(y);
                    gsc[3 + c] += dy * d->crf_gain * Ec[c];
                }
                if (dE_pix) dE_pix[3 * (size_t)pixel + c] = dEc[c];
            }
            /* per sample: clip (Eq. 12) then the path's own reverse sweep */
            for (int32_t s = 0; s < d->spp; ++s) {
                double delta[3];
                for (int c = 0; c < 3; ++c) {
                    double g = dEc[c] / d->spp;
                    if (d->clip && so[s].L[c] > thr) {
                        gsc[6] += g;        /* flows into the threshold k / min(w) */
                        delta[c] = 0;
                    } else {
                        delta[c] = g;
                    }
                }
                if (delta[0] == 0 && delta[1] == 0 && delta[2] == 0) continue;
                vrec* pr = rec + (size_t)s * d->max_depth;
                int nv = so[s].nv;
                /* R[k]: radiance leaving vertex k toward the previous vertex, unit throughput.
                   Every term of a vertex is beta_c f_c c S_c with c the cosine about the
                   shading normal and S_c its remaining factor: E_c / (cos^3 alpha d^2) for
                   the projector, L_env pi / c_sample for the environment, R_{k+1} / pdf for
                   the bounce; its derivative w.r.t. a map value is beta_c (d(f_c c)) S_c. */
                double Rn[3] = {0, 0, 0};   /* R of vertex k+1 */
                for (int k = nv - 1; k >= 0; --k) {
                    vrec* v = &pr[k];
                    double Rk[3];
                    double ga[3] = {0, 0, 0}, gr = 0, gs = 0, gm = 0;
                    v3 gn = mk(0, 0, 0);
                    const brdf_full_t* fv[3] = {v->proj ? &v->pf : NULL, v->env ? &v->ef : NULL,
                                                v->bounced ? &v->bf : NULL};
                    double S[3][3];
                    for (int c = 0; c < 3; ++c) {
                        S[0][c] = v->pE[c] * v->pg0;
                        S[1][c] = d->env[c] * v->es;
                        S[2][c] = v->bounced ? Rn[c] / v->bpdf : 0.0;
                    }
                    if (d_cam && k == 0) {
                        /* camera pose: central differences of the camera vertex's radiance
                           over the 12 entries of (R, t), contracted with the cotangent */
                        double pose[12], Se[3], Sb[3];
                        memcpy(pose, d->Rc, sizeof(double) * 9);
                        memcpy(pose + 9, d->tc, sizeof(double) * 3);
                        for (int c = 0; c < 3; ++c) {
                            Se[c] = S[1][c];
                            Sb[c] = S[2][c];
                        }
                        for (int e = 0; e < 12; ++e) {
                            double vp[3], vm[3], keep = pose[e];
                            pose[e] = keep + CAM_FD_H;
                            camera_vertex(&cx, pixel, s, pose, pose + 9, v, Se, Sb, vp);
                            pose[e] = keep - CAM_FD_H;
                            camera_vertex(&cx, pixel, s, pose, pose + 9, v, Se, Sb, vm);
                            pose[e] = keep;
                            for (int c = 0; c < 3; ++c)
                                gcam[e] += delta[c] * v->beta[c] * (vp[c] - vm[c]) / (2.0 * CAM_FD_H);
                        }
                    }
                    for (int c = 0; c < 3; ++c) {
                        double own = v->Le[c];
                        double bd = delta[c] * v->beta[c];  /* dL/d(term of vertex k) */
                        for (int j = 0; j < 3; ++j) {
                            const brdf_full_t* b = fv[j];
                            if (!b) continue;
                            double cs = b->c * S[j][c];
                            own += b->f[c] * cs;
                            ga[c] += bd * b->dfa * cs;
                            gr += bd * b->dfr[c] * cs;
                            gs += bd * b->dfs * cs;
                            gm += bd * b->dfm[c] * cs;
                            gn = add(gn, scl(b->dfcn[c], bd * S[j][c]));
                        }
                        if (v->proj) {
                            /* d/dE_p through the bilinear weights */
                            double gE = bd * v->pf.f[c] * v->pf.c * v->pg0;
                            for (int t = 0; t < 4; ++t) gEp[3 * (size_t)v->ptex.idx[t] + c] += gE * v->ptex.w[t];
                        }
                        Rk[c] = own;
                    }
                    /* the normal's cotangent in map values: ns = F t / |t|, t = 2 v - 1 */
                    double gnm[3] = {0, 0, 0};
                    if (v->nm && v->tlen > 0) {
                        v3 gl = mk(dot(v->fT, gn), dot(v->fB, gn), dot(v->fN, gn));
                        v3 gt = scl(sub(gl, scl(v->th, dot(v->th, gl))), 1.0 / v->tlen);
                        gnm[0] = 2.0 * gt.x;
                        gnm[1] = 2.0 * gt.y;
                        gnm[2] = 2.0 * gt.z;
                    }
                    for (int t = 0; t < 4; ++t) {
                        size_t ti = (size_t)v->tex.idx[t];
                        double w = v->tex.w[t];
                        for (int c = 0; c < 3; ++c) galb[3 * ti + c] += ga[c] * w;
                        if (d->brdf == 1) {
                            grough[ti] += gr * w;
                            gspec[ti] += gs * w;
                            gmetal[ti] += gm * w;
                        }
                        for (int c = 0; c < 3; ++c) gnmap[3 * ti + c] += gnm[c] * w;
                    }
                    for (int c = 0; c < 3; ++c) Rn[c] = Rk[c];
                }
            }
        }
        free(rec);
        free(so);
    }
    /* reduce the per-thread accumulators in thread order */
    double* tot = (double*)calloc(per, sizeof(double));
    for (int t = 0; t < nth; ++t)
        for (size_t k = 0; k < per; ++k) tot[k] += acc[(size_t)t * per + k];
    double* gEp = tot;
    double* galb = gEp + nEp;
    double* grough = galb + 3 * nT;
    double* gspec = grough + nT;
    double* gmetal = gspec + nT;
    double* gnmap = gmetal + nT;
    double* gsc = gnmap + 3 * nT;
    if (d_cam) memcpy(d_cam, gsc + 7, sizeof(double) * 12);
    if (dE_pix) {
        double bnd[12];
        orc_camera_boundary(d, dE_pix, bnd, NULL);
        for (int k = 0; k < 12; ++k) d_cam[k] += bnd[k];
        free(dE_pix);
    }
    double sc[18];
    memset(sc, 0, sizeof sc);
    for (int c = 0; c < 3; ++c) { sc[12 + c] = gsc[c]; sc[15 + c] = gsc[3 + c]; }
    if (d->clip) sc[15 + thr_arg] += -gsc[6] * d->clip_k / (d->wb[thr_arg] * d->wb[thr_arg]);

    /* PRF backward (Eq. 1 with mixing): z = g_p M y, y = I_p^gamma_p, E_p = max(0, z) */
    if (d_Ip) memset(d_Ip, 0, sizeof(double) * nEp);
    for (size_t t = 0; t < (size_t)d->Wp * d->Hp; ++t) {
        double y[3], z[3], dz[3], dy[3];
        for (int c = 0; c < 3; ++c) {
            double x = d->Ip[3 * t + c];
            y[c] = x > 0 ? pow(x, d->prf_gamma[c]) : 0.0;
        }
        for (int c = 0; c < 3; ++c) {
            z[c] = d->prf_gain * (d->prf_mix[3 * c] * y[0] + d->prf_mix[3 * c + 1] * y[1] +
                                  d->prf_mix[3 * c + 2] * y[2]);
            dz[c] = z[c] > 0 ? gEp[3 * t + c] : 0.0;
        }
        for (int c = 0; c < 3; ++c)
            dy[c] = d->prf_gain * (d->prf_mix[c] * dz[0] + d->prf_mix[3 + c] * dz[1] + d->prf_mix[6 + c] * dz[2]);
        for (int c = 0; c < 3; ++c) {
            double x = d->Ip[3 * t + c];
            if (x > 0) {
                if (d_Ip) d_Ip[3 * t + c] = dy[c] * d->prf_gamma[c] * pow(x, d->prf_gamma[c] - 1.0);
                sc[c] += dy[c] * y[c] * log(x);
            }
            for (int k = 0; k < 3; ++k) sc[3 + 3 * c + k] += d->prf_gain * dz[c] * y[k];
        }
    }
    if (d_Ep_out) memcpy(d_Ep_out, gEp, sizeof(double) * nEp);
    if (d_albedo) memcpy(d_albedo, galb, sizeof(double) * 3 * nT);
    if (d_rough) memcpy(d_rough, grough, sizeof(double) * nT);
    if (d_spec) memcpy(d_spec, gspec, sizeof(double) * nT);
    if (d_metal) memcpy(d_metal, gmetal, sizeof(double) * nT);
    if (d_nmap) memcpy(d_nmap, gnmap, sizeof(double) * 3 * nT);
    if (d_scalars) memcpy(d_scalars, sc, sizeof sc);
    free(tot);
    free(acc);
    ctx_free(&cx);
    (void)npix_all;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* test hooks                                                                 */
/* ------------------------------------------------------------------------- */

/* brute-force closest hit for n rays: rays = n*8 (o.xyz, d.xyz, tmax, skip) */
void orc_intersect(const orc_desc* d, int64_t n, const double* rays, int32_t* prim, double* t,
                   double* b1, double* b2, double* margin) {
    ctx_t cx;
    ctx_init(&cx, d);
    for (int64_t k = 0; k < n; ++k) {
        const double* r = rays + 8 * k;
        tri_isect h;
        memset(&h, 0, sizeof h);
        double m = 0;
        int p = closest_hit(d, &cx.sc, mk(r[0], r[1], r[2]), mk(r[3], r[4], r[5]), r[6], (int)r[7], &h,
                            margin ? &m : NULL);
        prim[k] = p;
        if (t) t[k] = p >= 0 ? h.t : INFINITY;
        if (b1) b1[k] = p >= 0 ? h.b1 : 0;
        if (b2) b2[k] = p >= 0 ? h.b2 : 0;
        if (margin) margin[k] = m;
    }
    ctx_free(&cx);
}

/* BRDF value and its derivatives: out[0..2] f, out[3] ds/dr, out[4] ds/dsp */
void orc_brdf(int32_t kind, const double* n, const double* wo, const double* wi, const double* a, double r,
              double sp, double* out) {
    v3 N = mk(n[0], n[1], n[2]);
    brdf_full_t b = brdf_full(kind, N, N, mk(wo[0], wo[1], wo[2]), mk(wi[0], wi[1], wi[2]), a, r, sp, 0.0);
    /* without metallic the specular term is the same in every channel */
    out[0] = b.f[0]; out[1] = b.f[1]; out[2] = b.f[2]; out[3] = b.dfr[0]; out[4] = b.dfs;
}

/* the principled BRDF with metallic and a shading normal: out[0..2] f, [3] cos(ns, wi),
 * [4] df/da, [5..7] df/dr, [8] df/dsp, [9..11] df/dmu, [12..20] d(f_c cos)/dns (c-major) */
void orc_brdf_full(int32_t kind, const double* ng, const double* ns, const double* wo, const double* wi,
                   const double* a, double r, double sp, double mu, double* out) {
    brdf_full_t b = brdf_full(kind, mk(ng[0], ng[1], ng[2]), mk(ns[0], ns[1], ns[2]), mk(wo[0], wo[1], wo[2]),
                              mk(wi[0], wi[1], wi[2]), a, r, sp, mu);
    for (int c = 0; c < 3; ++c) {
        out[c] = b.f[c];
        out[5 + c] = b.dfr[c];
        out[9 + c] = b.dfm[c];
        out[12 + 3 * c] = b.dfcn[c].x;
        out[13 + 3 * c] = b.dfcn[c].y;
        out[14 + 3 * c] = b.dfcn[c].z;
    }
    out[3] = b.c;
    out[4] = b.dfa;
    out[8] = b.dfs;
}

/* tangent frame and shading normal of one hit, for tests: out[0..2] T, [3..5] B,
 * [6..8] n (two-sided, facing -dir), [9..11] ns (n when the descriptor has no normal map) */
void orc_shading_frame(const orc_desc* d, int32_t prim, const double* dir, const double* uv, double* out) {
    v3 v0 = vtx(d, d->F[3 * prim]), v1 = vtx(d, d->F[3 * prim + 1]), v2 = vtx(d, d->F[3 * prim + 2]);
    v3 n = nrm(cross(sub(v1, v0), sub(v2, v0)));
    if (dot(n, mk(dir[0], dir[1], dir[2])) > 0) n = scl(n, -1.0);
    v3 T, B, th, ns = n;
    double tl;
    tangent_frame(d, prim, n, &T, &B);
    if (d->nmap) {
        bilin tb = tex_lookup(d, uv[0], uv[1]);
        ns = shading_normal(d->nmap, &tb, T, B, n, &th, &tl);
    }
    v3 o[4] = {T, B, n, ns};
    for (int k = 0; k < 4; ++k) { out[3 * k] = o[k].x; out[3 * k + 1] = o[k].y; out[3 * k + 2] = o[k].z; }
}

/* bounce sampler: u[3] = (lobe, u1, u2) -> wi, pdf */
void orc_sample(int32_t kind, const double* n, const double* wo, double r, int64_t count, const double* u,
                double* wi, double* pdf) {
    v3 N = mk(n[0], n[1], n[2]), WO = mk(wo[0], wo[1], wo[2]);
    for (int64_t k = 0; k < count; ++k) {
        v3 w = sample_bounce(kind, N, WO, r, u[3 * k], u[3 * k + 1], u[3 * k + 2]);
        wi[3 * k] = w.x; wi[3 * k + 1] = w.y; wi[3 * k + 2] = w.z;
        pdf[k] = bounce_pdf(kind, N, WO, w, r);
    }
}

double orc_pdf(int32_t kind, const double* n, const double* wo, const double* wi, double r) {
    return bounce_pdf(kind, mk(n[0], n[1], n[2]), mk(wo[0], wo[1], wo[2]), mk(wi[0], wi[1], wi[2]), r);
}

double orc_ggx_D(double nh, double r) { return ggx_D(nh, ggx_alpha(r)); }
double orc_ggx_G1(double c, double r) { return ggx_G1(c, ggx_alpha(r)); }

/* per-texel PRF (Eq. 1 with mixing) for tests */
void orc_prf(const orc_desc* d, double* Ep) { prf_forward(d, Ep); }

/* bilinear lookup of an arbitrary Hx W x C image at texel-centred coordinates */
void orc_bilinear(const double* img, int32_t W, int32_t H, int32_t C, int64_t n, const double* xy, double* out) {
    for (int64_t k = 0; k < n; ++k) {
        bilin b = bilinear_at(xy[2 * k], xy[2 * k + 1], W, H);
        for (int c = 0; c < C; ++c) {
            double s = 0;
            for (int t = 0; t < 4; ++t) s += b.w[t] * img[(size_t)C * b.idx[t] + c];
            out[(size_t)C * k + c] = s;
        }
    }
}

int orc_threads(const orc_desc* d) { return nthreads_of(d); }

/* camera ray and first-hit attributes of sample (pixel, s):
 * out[0..2] ray origin, [3..5] direction, [6] t (inf on miss), [7] prim, [8..10] x,
 * [11..13] two-sided normal, [14..15] texture uv, [16..17] projector (u,v) of x (nan if behind) */
void orc_first_hit(const orc_desc* d, int32_t pixel, int32_t s, double* out) {
    ctx_t cx;
    ctx_init(&cx, d);
    int32_t i = pixel % d->Wc, j = pixel / d->Wc;
    double u[4];
    uniforms(d, (uint32_t)pixel, (uint32_t)s, 0u, u);
    v3 dir = nrm(mattv(d->Rc, matv(cx.Kc_inv, mk(i + u[0], j + u[1], 1.0))));
    v3 o = cx.cam_o;
    tri_isect h;
    int prim = closest_hit(d, &cx.sc, o, dir, 1e300, -1, &h, NULL);
    for (int k = 0; k < 18; ++k) out[k] = NAN;
    out[0] = o.x; out[1] = o.y; out[2] = o.z; out[3] = dir.x; out[4] = dir.y; out[5] = dir.z;
    out[6] = INFINITY;
    out[7] = prim;
    if (prim >= 0) {
        v3 v0 = vtx(d, d->F[3 * prim]), v1 = vtx(d, d->F[3 * prim + 1]), v2 = vtx(d, d->F[3 * prim + 2]);
        v3 x = add(add(scl(v0, h.b0), scl(v1, h.b1)), scl(v2, h.b2));
        v3 n = nrm(cross(sub(v1, v0), sub(v2, v0)));
        if (dot(n, dir) > 0) n = scl(n, -1.0);
        const float* uvp = d->UV + 6 * (size_t)prim;
        out[6] = h.t;
        out[8] = x.x; out[9] = x.y; out[10] = x.z;
        out[11] = n.x; out[12] = n.y; out[13] = n.z;
        out[14] = h.b0 * uvp[0] + h.b1 * uvp[2] + h.b2 * uvp[4];
        out[15] = h.b0 * uvp[1] + h.b1 * uvp[3] + h.b2 * uvp[5];
        v3 xp = add(matv(d->Rp, x), mk(d->tp[0], d->tp[1], d->tp[2]));
        if (xp.z > 0) {
            out[16] = (d->Kp[0] * xp.x + d->Kp[1] * xp.y + d->Kp[2] * xp.z) / xp.z;
            out[17] = (d->Kp[3] * xp.x + d->Kp[4] * xp.y + d->Kp[5] * xp.z) / xp.z;
        }
    }
    ctx_free(&cx);
}

/* mixture pdf for many directions */
void orc_pdf_batch(int32_t kind, const double* n, const double* wo, double r, int64_t count, const double* wi,
                   double* out) {
    v3 N = mk(n[0], n[1], n[2]), WO = mk(wo[0], wo[1], wo[2]);
    for (int64_t k = 0; k < count; ++k)
        out[k] = bounce_pdf(kind, N, WO, mk(wi[3 * k], wi[3 * k + 1], wi[3 * k + 2]), r);
}

/* ------------------------------------------------------------------------- */
/* Eq. 11: the cross-bilateral denoiser D and its adjoint                     */
/* ------------------------------------------------------------------------- */
/* The paper applies a differentiable cross-bilateral filter to the rendered
 * image before the loss and fixes neither its window nor its weights.  Reading
 * taken here: over the (2r+1) x (2r+1) window around pixel p, clipped to the image,
 *     D(I)_p = sum_q w(p,q) I_q / W_p,     W_p = sum_q w(p,q),
 *     w(p,q) = exp(-a_s |p - q|^2 - sum_k a_k (g_k(p) - g_k(q))^2),
 * where g is a per-pixel guide image of G channels and a = 1 / (2 sigma^2) per
 * channel.  The guide carries no gradient, so D is linear in I and its VJP is the
 * transposed operator:  (D^T G)_q = sum_p w(p,q) G_p / W_p.
 * Images are H x W x 3 and guides H x W x G, row-major. */
static double bil_weight(const double* guide, int32_t G, const double* a_g, double a_s, int32_t W,
                         int32_t px, int32_t py, int32_t qx, int32_t qy) {
    double e = a_s * ((double)(px - qx) * (px - qx) + (double)(py - qy) * (py - qy));
    const double* gp = guide + (size_t)G * ((size_t)py * W + px);
    const double* gq = guide + (size_t)G * ((size_t)qy * W + qx);
    for (int32_t k = 0; k < G; ++k) e += a_g[k] * (gp[k] - gq[k]) * (gp[k] - gq[k]);
    return exp(-e);
}

static double bil_norm(const double* guide, int32_t G, const double* a_g, double a_s, int32_t W, int32_t H,
                       int32_t r, int32_t px, int32_t py) {
    double s = 0;
    for (int32_t qy = py - r; qy <= py + r; ++qy)
        for (int32_t qx = px - r; qx <= px + r; ++qx)
            if (qx >= 0 && qx < W && qy >= 0 && qy < H)
                s += bil_weight(guide, G, a_g, a_s, W, px, py, qx, qy);
    return s;
}

void orc_denoise(const double* img, const double* guide, int32_t W, int32_t H, int32_t G, const double* a_g,
                 double a_s, int32_t r, double* out) {
#pragma omp parallel for schedule(static)
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px) {
            double acc[3] = {0, 0, 0}, wsum = 0;
            for (int32_t qy = py - r; qy <= py + r; ++qy)
                for (int32_t qx = px - r; qx <= px + r; ++qx) {
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                    double w = bil_weight(guide, G, a_g, a_s, W, px, py, qx, qy);
                    wsum += w;
                    for (int c = 0; c < 3; ++c) acc[c] += w * img[3 * ((size_t)qy * W + qx) + c];
                }
            for (int c = 0; c < 3; ++c) out[3 * ((size_t)py * W + px) + c] = acc[c] / wsum;
        }
}

void orc_denoise_vjp(const double* grad, const double* guide, int32_t W, int32_t H, int32_t G,
                     const double* a_g, double a_s, int32_t r, double* out) {
    /* output pixel q gathers from every p whose window holds q */
#pragma omp parallel for schedule(static)
    for (int32_t qy = 0; qy < H; ++qy)
        for (int32_t qx = 0; qx < W; ++qx) {
            double acc[3] = {0, 0, 0};
            for (int32_t py = qy - r; py <= qy + r; ++py)
                for (int32_t px = qx - r; px <= qx + r; ++px) {
                    if (px < 0 || px >= W || py < 0 || py >= H) continue;
                    double w = bil_weight(guide, G, a_g, a_s, W, px, py, qx, qy) /
                               bil_norm(guide, G, a_g, a_s, W, H, r, px, py);
                    for (int c = 0; c < 3; ++c) acc[c] += w * grad[3 * ((size_t)py * W + px) + c];
                }
            for (int c = 0; c < 3; ++c) out[3 * ((size_t)qy * W + qx) + c] = acc[c];
        }
}

/* ------------------------------------------------------------------------- */
/* Eq. 9: regulariser L(m) and data term                                      */
/* ------------------------------------------------------------------------- */
static double sgn(double x) { return x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0); }

/* L(m) for an h x w x c map: the paper calls it a total-variation loss without a
 * formula.  Reading taken here: the anisotropic L1 form, mean |m(y+1,x) - m(y,x)|
 * over all c (h-1) w vertical pairs plus mean |m(y,x+1) - m(y,x)| over all
 * c h (w-1) horizontal pairs (a term without pairs is 0).  grad (may be NULL,
 * h x w x c) receives dL/dm with d|x|/dx = sign(x), sign(0) = 0. */
double orc_tv(const double* m, int32_t h, int32_t w, int32_t c, double* grad) {
    const double nv = (double)c * (h - 1) * w, nh = (double)c * h * (w - 1);
    double sv = 0, sh = 0;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)h * w * c);
    for (int32_t y = 0; y < h; ++y)
        for (int32_t x = 0; x < w; ++x)
            for (int32_t k = 0; k < c; ++k) {
                size_t i = ((size_t)y * w + x) * c + k;
                if (y + 1 < h) {
                    size_t j = i + (size_t)w * c;
                    double dv = m[j] - m[i];
                    sv += absd(dv);
                    if (grad) { grad[j] += sgn(dv) / nv; grad[i] -= sgn(dv) / nv; }
                }
                if (x + 1 < w) {
                    size_t j = i + (size_t)c;
                    double dh = m[j] - m[i];
                    sh += absd(dh);
                    if (grad) { grad[j] += sgn(dh) / nh; grad[i] -= sgn(dh) / nh; }
                }
            }
    return (nv > 0 ? sv / nv : 0.0) + (nh > 0 ? sh / nh : 0.0);
}

/* data term of Eq. 9 for one image pair: mean |a - b| over n values;
 * grad (may be NULL) receives d/da = sign(a - b) / n with sign(0) = 0. */
double orc_l1(const double* a, const double* b, int64_t n, double* grad) {
    double s = 0;
    for (int64_t i = 0; i < n; ++i) {
        s += absd(a[i] - b[i]);
        if (grad) grad[i] = sgn(a[i] - b[i]) / (double)n;
    }
    return n > 0 ? s / (double)n : 0.0;
}

/* ------------------------------------------------------------------------- */
/* guide features for D: one camera ray through each pixel centre (Eq. 6)     */
/* ------------------------------------------------------------------------- */
/* out: npix x 8 = albedo rgb of the first hit (bilinear texture lookup), unit
 * geometric normal turned toward the camera, hit distance t, 1; all 8 are 0 where
 * the ray escapes.  margin (may be NULL): the hit decision's normalised margin. */
void orc_gbuffer(const orc_desc* d, int32_t npix, const int32_t* pixels, double* out, double* margin) {
    ctx_t cx;
    ctx_init(&cx, d);
    int nth = nthreads_of(d);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
    for (int32_t q = 0; q < npix; ++q) {
        int32_t pixel = pixels ? pixels[q] : q;
        int32_t i = pixel % d->Wc, j = pixel / d->Wc;
        v3 dir = nrm(mattv(d->Rc, matv(cx.Kc_inv, mk(i + 0.5, j + 0.5, 1.0))));
        tri_isect h;
        double m;
        int prim = closest_hit(d, &cx.sc, cx.cam_o, dir, 1e300, -1, &h, &m);
        double* o = out + 8 * (size_t)q;
        for (int k = 0; k < 8; ++k) o[k] = 0.0;
        if (margin) margin[q] = m;
        if (prim < 0) continue;
        v3 v0 = vtx(d, d->F[3 * prim]), v1 = vtx(d, d->F[3 * prim + 1]), v2 = vtx(d, d->F[3 * prim + 2]);
        v3 n = nrm(cross(sub(v1, v0), sub(v2, v0)));
        if (dot(n, dir) > 0) n = scl(n, -1.0);
        const float* uvp = d->UV + 6 * (size_t)prim;
        double tu = h.b0 * uvp[0] + h.b1 * uvp[2] + h.b2 * uvp[4];
        double tv = h.b0 * uvp[1] + h.b1 * uvp[3] + h.b2 * uvp[5];
        bilin tb = tex_lookup(d, tu, tv);
        fetch3(d->albedo, &tb, o);
        o[3] = n.x; o[4] = n.y; o[5] = n.z;
        o[6] = h.t;
        o[7] = 1.0;
    }
    ctx_free(&cx);
}
