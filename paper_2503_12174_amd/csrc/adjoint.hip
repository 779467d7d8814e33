// adjoint.hip -- vector-Jacobian product of the renderer by path replay.
//
// Sampling is detached: directions, pdfs and lobe choices are constants of the
// estimator, so replaying the forward path with the same Philox counters gives the
// same vertices, and the derivative of a sample's radiance
//     L = sum_k beta_k (Le_k + NEE_k),   beta_{k+1} = beta_k f_k(wo, wi) cos / pdf
// w.r.t. anything inside f_k of the bounce at vertex k is (remaining radiance after
// vertex k) / f_k * df_k (path-replay backpropagation, Vicini et al. 2021).  The
// remaining radiance starts at the sample's total and loses each vertex's own
// contributions as the replay passes them.
//
//   adj_pixel   CRF backward (Eq. 5) and the clip backward (Eq. 12) per pixel; seeds
//               the per-sample cotangent delta and the remaining radiance
//   (raygen, trace: the forward kernels)
//   adj_shade   settles the previous vertex's bounce derivative, removes emission,
//               emits next-event shadow rays with their gradient payloads, bounces
//   adj_shadow  visible: scatter dE_p and BRDF-map cotangents, subtract the
//               contribution from the path's remaining radiance
//   adj_replay  with the forward's path records: adj_shade and adj_shadow in one pass,
//               visibility and hit leaf read from the records instead of traced
//   adj_finish  PRF backward (Eq. 1) per texel and the scalar reductions
#include <algorithm>

#include "kernels.hpp"
#include "shade.hpp"

namespace dpcs {

constexpr int TB = TRACE_TB;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Adds v[0..N) to base[stride * idx + j] for every active lane.  Must be called by all
// lanes of the wave.  Lanes that share an index (common: neighbouring samples of one
// pixel) are summed across the wave first and written by one atomic per distinct index;
// once a group has a single lane the remaining lanes add directly.
template <int N>
__device__ __forceinline__ void wave_scatter_add(bool active, int idx, float* base, int stride, const float* v) {
    unsigned long long todo = __ballot(active);
    const int lane = __lane_id();
    while (todo) {
        const int leader = __ffsll(todo) - 1;
        const int lidx = __shfl(idx, leader);
        const bool mine = active && idx == lidx;
        const unsigned long long m = __ballot(mine);
        if (__popcll(m) < 2) break;
        float sum[N];
#pragma unroll
        for (int j = 0; j < N; ++j) sum[j] = wave_sum(mine ? v[j] : 0.0f);
        if (lane == leader) {
            float* t = base + (size_t)stride * lidx;
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (sum[j] != 0.0f) atomicAdd(t + j, sum[j]);
        }
        if (mine) active = false;
        todo &= ~m;
    }
    if (active) {
        float* t = base + (size_t)stride * idx;
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (v[j] != 0.0f) atomicAdd(t + j, v[j]);
    }
}

// BRDF-map cotangents g = (albedo rgb, roughness, specular) at texture coordinate
// (u, v), spread over the four texels of the bilinear lookup.  Per-lane form:
__device__ __forceinline__ void scatter_tex_lane(const ReqDesc& r, double u, double v, const float* gv) {
    if (!r.d_tex) return;
    const Bilin b = bilinear(u * r.tw - 0.5, v * r.th - 0.5, r.tw, r.th);
    const int idx[4] = {b.i00, b.i10, b.i01, b.i11};
    const double wt[4] = {b.w00, b.w10, b.w01, b.w11};
    const int nc = r.brdf ? 5 : 3;
    for (int k = 0; k < 4; ++k) {
        if (wt[k] == 0.0) continue;
        float* t = r.d_tex + 5 * (size_t)idx[k];
        for (int j = 0; j < nc; ++j) {
            const float val = (float)(gv[j] * wt[k]);
            if (val != 0.0f) atomicAdd(t + j, val);
        }
    }
}

// wave-uniform form (inactive lanes pass active = false)
__device__ __forceinline__ void scatter_tex(const ReqDesc& r, bool active, double u, double v, const float* gv) {
    if (!r.d_tex) return;
    Bilin b = bilinear(active ? u * r.tw - 0.5 : 0.0, active ? v * r.th - 0.5 : 0.0, r.tw, r.th);
    const int idx[4] = {b.i00, b.i10, b.i01, b.i11};
    const double wt[4] = {b.w00, b.w10, b.w01, b.w11};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float val[5] = {(float)(gv[0] * wt[k]), (float)(gv[1] * wt[k]), (float)(gv[2] * wt[k]),
                              (float)(gv[3] * wt[k]), (float)(gv[4] * wt[k])};
        const bool on = active && wt[k] != 0.0;
        if (r.brdf) wave_scatter_add<5>(on, idx[k], r.d_tex, 5, val);
        else wave_scatter_add<3>(on, idx[k], r.d_tex, 5, val);
    }
}

// cotangent of E_p (rgb per texel, stride 4) at projector pixel position (pu, pv)
__device__ __forceinline__ void scatter_ep_lane(const ReqDesc& r, double pu, double pv, const float* gE) {
    const Bilin b = bilinear(pu - 0.5, pv - 0.5, r.Wp, r.Hp);
    const int idx[4] = {b.i00, b.i10, b.i01, b.i11};
    const double wt[4] = {b.w00, b.w10, b.w01, b.w11};
    for (int k = 0; k < 4; ++k) {
        if (wt[k] == 0.0) continue;
        float* t = r.dEp + 4 * (size_t)idx[k];
        for (int j = 0; j < 3; ++j) atomicAdd(t + j, (float)(gE[j] * wt[k]));
    }
}

__device__ __forceinline__ void scatter_ep(const ReqDesc& r, bool active, double pu, double pv, const float* gE) {
    const Bilin b = bilinear(active ? pu - 0.5 : 0.0, active ? pv - 0.5 : 0.0, r.Wp, r.Hp);
    const int idx[4] = {b.i00, b.i10, b.i01, b.i11};
    const double wt[4] = {b.w00, b.w10, b.w01, b.w11};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float val[3] = {(float)(gE[0] * wt[k]), (float)(gE[1] * wt[k]), (float)(gE[2] * wt[k])};
        wave_scatter_add<3>(active && wt[k] != 0.0, idx[k], r.dEp, 4, val);
    }
}

// ---------------------------------------------------------------- binned map cotangents
// A record starts with one header word: base texel y0 * W + x0 of the bilinear corners
// (bits 0..27), x1 - x0 (bit 28) and y1 - y0 (bit 29), then the offsets ax, ay and the
// C cotangent values.
constexpr int TEX_RS = 8, EP_RS = 6;   // floats per record (C = 5, C = 3)

__device__ __forceinline__ uint32_t map_head(const Corners& c, int W) {
    return (uint32_t)(c.y0 * W + c.x0) | ((uint32_t)(c.x1 - c.x0) << 28) | ((uint32_t)(c.y1 - c.y0) << 29);
}
__device__ __forceinline__ int map_bin(const MapBins& mb, uint32_t head) {
    const uint32_t base = head & 0x0fffffffu;
    const int y0 = (int)(base / (uint32_t)mb.W), x0 = (int)(base - (uint32_t)y0 * (uint32_t)mb.W);
    return (y0 / mb.T) * mb.nbx + x0 / mb.T;
}
// BRDF-map record at texture coordinate (u, v); false when the buffer is full
__device__ __forceinline__ bool put_tex_rec(const MapBins& mb, uint32_t slot, double u, double v, const float* g) {
    if ((int64_t)slot >= mb.cap) return false;
    const Corners c = bilinear_corners(u * mb.W - 0.5, v * mb.H - 0.5, mb.W, mb.H);
    float4* p = (float4*)(mb.rec + (size_t)slot * TEX_RS);
    nt_st(p, make_float4(__uint_as_float(map_head(c, mb.W)), (float)c.ax, (float)c.ay, g[0]));
    nt_st(p + 1, make_float4(g[1], g[2], g[3], g[4]));
    return true;
}
// BRDF-map record with the metallic and normal-map cotangents (C = 9)
constexpr int TEX9_RS = 12;
__device__ __forceinline__ bool put_tex9_rec(const MapBins& mb, uint32_t slot, double u, double v, const float* g) {
    if ((int64_t)slot >= mb.cap) return false;
    const Corners c = bilinear_corners(u * mb.W - 0.5, v * mb.H - 0.5, mb.W, mb.H);
    float4* p = (float4*)(mb.rec + (size_t)slot * TEX9_RS);
    nt_st(p, make_float4(__uint_as_float(map_head(c, mb.W)), (float)c.ax, (float)c.ay, g[0]));
    nt_st(p + 1, make_float4(g[1], g[2], g[3], g[4]));
    nt_st(p + 2, make_float4(g[5], g[6], g[7], g[8]));
    return true;
}
// per-lane and wave-uniform scatter of the 9 cotangents (stride 9 per texel)
__device__ __forceinline__ void scatter_tex9_lane(const ReqDesc& r, double u, double v, const float* gv) {
    if (!r.d_tex) return;
    const Bilin b = bilinear(u * r.tw - 0.5, v * r.th - 0.5, r.tw, r.th);
    const int idx[4] = {b.i00, b.i10, b.i01, b.i11};
    const double wt[4] = {b.w00, b.w10, b.w01, b.w11};
    for (int k = 0; k < 4; ++k) {
        if (wt[k] == 0.0) continue;
        float* t = r.d_tex + 9 * (size_t)idx[k];
        for (int j = 0; j < 9; ++j) {
            const float val = (float)(gv[j] * wt[k]);
            if (val != 0.0f) atomicAdd(t + j, val);
        }
    }
}
__device__ __forceinline__ void scatter_tex9(const ReqDesc& r, bool active, double u, double v, const float* gv) {
    if (!r.d_tex) return;
    Bilin b = bilinear(active ? u * r.tw - 0.5 : 0.0, active ? v * r.th - 0.5 : 0.0, r.tw, r.th);
    const int idx[4] = {b.i00, b.i10, b.i01, b.i11};
    const double wt[4] = {b.w00, b.w10, b.w01, b.w11};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float val[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) val[j] = (float)(gv[j] * wt[k]);
        wave_scatter_add<9>(active && wt[k] != 0.0, idx[k], r.d_tex, 9, val);
    }
}

// E_p record at projector pixel position (pu, pv); false when the buffer is full
__device__ __forceinline__ bool put_ep_rec(const MapBins& mb, uint32_t slot, double pu, double pv, const float* g) {
    if ((int64_t)slot >= mb.cap) return false;
    const Corners c = bilinear_corners(pu - 0.5, pv - 0.5, mb.W, mb.H);
    float2* p = (float2*)(mb.rec + (size_t)slot * EP_RS);
    nt_st(p, make_float2(__uint_as_float(map_head(c, mb.W)), (float)c.ax));
    nt_st(p + 1, make_float2((float)c.ay, g[0]));
    nt_st(p + 2, make_float2(g[1], g[2]));
    return true;
}

// ---------------------------------------------------------------- per pixel
// Eq. 5 backward: y = g_c w E_c, I_c = y^gamma_c;  Eq. 12 backward per sample.
// PIX_LANES lanes per pixel stride over its samples, reductions inside the lane group.
__global__ void __launch_bounds__(BLOCK) k_adj_pixel(Queues q, AdjQueues aq, ReqDesc r, uint32_t p0, uint32_t p1,
                                                     const float* sample_L, float4* pix_dE) {
    const uint32_t p = p0 + (blockIdx.x * BLOCK + threadIdx.x) / PIX_LANES;
    const int lane = threadIdx.x & (PIX_LANES - 1);
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};   // d gamma_c[3], d w[3], d threshold
    if (p < p1) {   // uniform per lane group
        const float thr = clip_threshold(r);
        float Ls[3] = {0.f, 0.f, 0.f};
        for (int s = lane; s < r.spp; s += PIX_LANES) {
            const uint32_t g = p * (uint32_t)r.spp + (uint32_t)s;
            float4 L;
            if (sample_L) {
                L = make_float4(sample_L[3 * (size_t)g], sample_L[3 * (size_t)g + 1], sample_L[3 * (size_t)g + 2], 0.f);
                q.L[g - r.g_base + r.sid_base] = L;
            } else {
                L = q.L[g - r.g_base + r.sid_base];
            }
            Ls[0] += r.clip ? fminf(L.x, thr) : L.x;
            Ls[1] += r.clip ? fminf(L.y, thr) : L.y;
            Ls[2] += r.clip ? fminf(L.z, thr) : L.z;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int off = PIX_LANES / 2; off > 0; off >>= 1) Ls[c] += __shfl_xor(Ls[c], off);
        float dE[3];
        for (int c = 0; c < 3; ++c) {
            const float Ec = Ls[c] / (float)r.spp;
            const float w = scalar(r, 15 + c), gc = scalar(r, 12 + c);
            const float y = r.crf_gain * w * Ec;
            float G = 0.f;
            if (r.grad_image) {
                G = r.grad_image[3 * (size_t)p + c];
            } else if (r.target) {   // L2 loss mean over Hc x Wc x 3
                const float I = y > 0.f ? powf(y, gc) : 0.f;
                G = 2.f * (I - r.target[3 * (size_t)p + c]) / (3.f * (float)r.Wc * (float)r.Hc);
            }
            dE[c] = 0.f;
            if (y > 0.f && G != 0.f) {
                const float dy = G * gc * powf(y, gc - 1.f);
                dE[c] = dy * r.crf_gain * w;
                if (lane == 0) {   // per-pixel terms, once
                    acc[c] += G * powf(y, gc) * logf(y);
                    acc[3 + c] += dy * r.crf_gain * Ec;
                }
            }
        }
        if (pix_dE && lane == 0) pix_dE[p] = make_float4(dE[0], dE[1], dE[2], 0.f);
        for (int s = lane; s < r.spp; s += PIX_LANES) {
            const uint32_t g = p * (uint32_t)r.spp + (uint32_t)s;
            const uint32_t sid = g - r.g_base + r.sid_base;
            const float4 L = q.L[sid];
            const float l[3] = {L.x, L.y, L.z};
            float dl[3];
            for (int c = 0; c < 3; ++c) {
                const float gs = dE[c] / (float)r.spp;
                if (r.clip && l[c] > thr) {   // clipped: the sample's radiance does not matter
                    acc[6] += gs;
                    dl[c] = 0.f;
                } else {
                    dl[c] = gs;
                }
            }
            aq.delta[sid] = make_float4(dl[0], dl[1], dl[2], 0.f);
        }
    }
    // block reduction of the scalar partials, one atomic per value per workgroup
    __shared__ float red[7][BLOCK / 64];
    const int wv = threadIdx.x >> 6;
    for (int k = 0; k < 7; ++k) {
        float v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        float v = 0.f;
        for (int k = 0; k < BLOCK / 64; ++k) v += red[threadIdx.x][k];
        if (r.d_part) r.d_part[8 * (size_t)blockIdx.x + threadIdx.x] = v;
        else if (v != 0.f) atomicAdd(&r.d_acc[threadIdx.x], v);
    }
}

// dst[k] += the sum over nb workgroup partials part[b * stride + k], k < nv, in a fixed
// order (FP64), so the scalar gradients are the same on every run
// one workgroup per value k < nv (grid nv): dst[k] += the sum of the nb partials of k, in
// a fixed order (per thread a strided run, then a tree)
// value k of nb per-block partials (stride floats apart) added to dst[k] by thread 0, in
// a fixed order (strided FP64 sums, then a tree); a 256-thread workgroup calls it whole
__device__ __forceinline__ void sum_partial(const float* __restrict__ part, int nb, int stride, int k,
                                            float* __restrict__ dst, double* red) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(size_t)b * stride + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0.0) dst[k] += (float)red[0];
    __syncthreads();   // (red is reused by the next call)
}
__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ part, int nb, int stride, int nv,
                                                      float* __restrict__ dst) {
    __shared__ double red[256];
    if ((int)blockIdx.x >= nv) return;
    sum_partial(part, nb, stride, blockIdx.x, dst, red);
}

// replay camera rays at queue index = batch sample index (the depth-0 shading takes
// the remaining radiance, the sample's total, from q.L at that index and starts with
// no pending bounce, so nothing else is written here)
__global__ void k_adj_raygen(Queues q, AdjQueues, ReqDesc r, int slot, uint32_t g0, uint32_t n) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t g = g0 + k;
    const uint32_t sid = g - r.g_base + r.sid_base;
    const D3 d = camera_dir(r, g);
    q.po[0][sid] = PathO{r.cam_o[0], r.cam_o[1], r.cam_o[2], slot, -1};
    q.pd[0][sid] = PathD{d.x, d.y, d.z, g, 0u};
    q.pb[0][sid] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
}

// ---------------------------------------------------------------- shading
template <bool UNI>
__global__ void __launch_bounds__(BLOCK) k_adj_shade(Queues q, AdjQueues aq, int cur, int depth, ReqDesc uni,
                                                     const ReqDesc* __restrict__ table) {
    const int nxt = cur ^ 1;
    const uint32_t n = q.cnt[cur];
    // one path per thread (the grid covers the queue): with no grid-stride loop no
    // descriptor field is held across iterations, which saves ~60 VGPRs
    const uint32_t base = blockIdx.x * BLOCK;
    if (base >= n) return;   // uniform per workgroup
    {
        const uint32_t i = base + threadIdx.x;
        bool cont = false, shp = false, she = false;
        PathO no{};
        PathD nd{};
        float4 nb = {}, nrl = {}, npenda = {};
        float2 npend = {};
        double2 npuv = {}, pxp = {}, pxt = {}, ext = {};
        float4 po = {}, pd = {}, pc = {}, pg = {}, pa = {};
        float4 eo = {}, ed = {}, ec = {}, ea = {};
        float ptmax = 0.f, ps = 0.f, es = 0.f;
        bool pend_on = false;
        double pend_u = 0.0, pend_v = 0.0;
        float pend_g[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        const ReqDesc* rp = &sel<UNI>(uni, table, 0);
        if (i < n) {
            const PathO o = q.po[cur][i];
            const PathD dd = q.pd[cur][i];
            const float4 b = q.pb[cur][i];
            const int leaf = q.hit[i];
            const ReqDesc& r = sel<UNI>(uni, table, o.slot);
            rp = &r;
            const uint32_t g = dd.g;
            const uint32_t sid = g - r.g_base + r.sid_base;
            const float4 dl = aq.delta[sid];
            const D3 delta = d3(dl.x, dl.y, dl.z);
            const D3 beta = d3(b.x, b.y, b.z);
            // depth 0: the camera wave (queue index = batch sample index) starts from the
            // sample's total radiance with no pending bounce
            float4 rl = depth == 0 ? q.L[i] : aq.rl[cur][i];
            const float4 penda = depth == 0 ? make_float4(0.f, 0.f, 0.f, -1.f) : aq.penda[cur][i];
            if (leaf >= 0) {
                const Surf s = surface(r, leaf, d3(o.x, o.y, o.z), d3(dd.x, dd.y, dd.z));
                // the previous vertex's bounce: d/df of beta_k f cos/pdf R_{k+1} = L_r / f
                if (penda.w >= 0.f) {
                    const D3 t = delta * d3(rl.x, rl.y, rl.z) * d3(penda.x, penda.y, penda.z);
                    const double sum = t.x + t.y + t.z;
                    const float2 pend = aq.pend[cur][i];
                    const double2 puv = aq.puv[cur][i];
                    pend_on = true;
                    pend_u = puv.x;
                    pend_v = puv.y;
                    pend_g[0] = (float)(t.x * (1.0 / PI));
                    pend_g[1] = (float)(t.y * (1.0 / PI));
                    pend_g[2] = (float)(t.z * (1.0 / PI));
                    pend_g[3] = (float)(sum * pend.x);
                    pend_g[4] = (float)(sum * pend.y);
                }
                if (r.emission) {
                    const float4 e = r.emission[leaf];
                    rl.x -= (float)(beta.x * e.x);
                    rl.y -= (float)(beta.y * e.y);
                    rl.z -= (float)(beta.z * e.z);
                }
                const D3 db = delta * beta;
                ProjNee p;
                if (projector_nee(r, s, p)) {
                    const D4 E = fetch4(r.Ep, p.pb);
                    const Brdf f = brdf_eval<true>(r.brdf, s.n, s.wo, p.wp, s.alb, s.rough, s.spec);
                    const D3 Ex = d3(E.x, E.y, E.z) * p.geom;
                    const D3 C = beta * f.f * Ex;
                    const D3 gE = db * f.f * p.geom;        // d/dE_p before the bilinear weights
                    const D3 ga = db * Ex * (1.0 / PI);
                    const double sx = db.x * Ex.x + db.y * Ex.y + db.z * Ex.z;
                    shp = true;
                    po = f4(to_f(s.x), __int_as_float(o.slot));
                    pd = f4(to_f(p.wp), __int_as_float(s.prim));
                    pc = f4(to_f(C), __int_as_float(-1));   // w: next-queue index, set below
                    pxp = make_double2(p.pu, p.pv);
                    pxt = make_double2(s.u, s.v);
                    pg = f4(to_f(gE), 0.f);
                    pa = f4(to_f(ga), (float)(sx * f.ds_dr));
                    ps = (float)(sx * f.ds_dsp);
                    ptmax = (float)(p.dist - r.tmin);
                }
                if (r.env_on) {
                    const U4 x = vertex_rng(r, g, 2u + 2u * depth);
                    const D3 we = sample_cosine(s.n, u24(x.x), u24(x.y));
                    const Brdf f = brdf_eval<true>(r.brdf, s.n, s.wo, we, s.alb, s.rough, s.spec);
                    const D3 Ee = d3(r.env[0], r.env[1], r.env[2]) * PI;
                    const D3 C = beta * f.f * Ee;
                    const D3 ga = db * Ee * (1.0 / PI);
                    const double sx = db.x * Ee.x + db.y * Ee.y + db.z * Ee.z;
                    she = true;
                    eo = f4(to_f(s.x), __int_as_float(o.slot));
                    ed = f4(to_f(we), __int_as_float(s.prim));
                    ec = f4(to_f(C), __int_as_float(-1));
                    ext = make_double2(s.u, s.v);
                    ea = f4(to_f(ga), (float)(sx * f.ds_dr));
                    es = (float)(sx * f.ds_dsp);
                }
                if (depth < r.max_depth - 1) {
                    const U4 x = vertex_rng(r, g, 1u + 2u * depth);
                    const D3 wi = sample_bounce(r.brdf, s.n, s.wo, s.rough, u24(x.x), u24(x.y), u24(x.z));
                    const double ci = dot(s.n, wi);
                    const double pdf = bounce_pdf(r.brdf, s.n, s.wo, wi, s.rough);
                    if (ci > 0.0 && pdf > 0.0) {
                        const Brdf f = brdf_eval<true>(r.brdf, s.n, s.wo, wi, s.alb, s.rough, s.spec);
                        const D3 nbeta = beta * (f.f * (ci / pdf));
                        cont = true;
                        no = PathO{s.x.x, s.x.y, s.x.z, o.slot, s.prim};
                        nd = PathD{wi.x, wi.y, wi.z, g, 0u};
                        nb = make_float4((float)nbeta.x, (float)nbeta.y, (float)nbeta.z, 0.0f);
                        nrl = rl;
                        npuv = make_double2(s.u, s.v);
                        npend = make_float2((float)f.ds_dr, (float)f.ds_dsp);
                        npenda = make_float4(f.f.x > 0.0 ? (float)(1.0 / f.f.x) : 0.f,
                                             f.f.y > 0.0 ? (float)(1.0 / f.f.y) : 0.f,
                                             f.f.z > 0.0 ? (float)(1.0 / f.f.z) : 0.f, 1.f);
                    }
                }
            }
        }
        const bool to_rec = UNI && aq.tb.rec && pend_on;
        const bool pred[4] = {cont, shp, she, to_rec};
        uint32_t* const ctr[4] = {&q.cnt[nxt], &q.cnt[shadow_slot(cur, 0)], &q.cnt[shadow_slot(cur, 1)], aq.tb.count};
        uint32_t at[4];
        block_append<4>(pred, ctr, at);
        const uint32_t jn = at[0], jp = at[1], je = at[2];
        if (UNI && aq.tb.rec) {
            if (pend_on && !put_tex_rec(aq.tb, at[3], pend_u, pend_v, pend_g)) scatter_tex_lane(*rp, pend_u, pend_v, pend_g);
        } else if (UNI) {
            scatter_tex(*rp, pend_on, pend_u, pend_v, pend_g);
        } else if (pend_on) {
            scatter_tex_lane(*rp, pend_u, pend_v, pend_g);
        }
        if (cont) {
            q.po[nxt][jn] = no;
            q.pd[nxt][jn] = nd;
            q.pb[nxt][jn] = nb;
            aq.rl[nxt][jn] = nrl;
            aq.pend[nxt][jn] = npend;
            aq.puv[nxt][jn] = npuv;
            aq.penda[nxt][jn] = npenda;
        }
        const int next_idx = cont ? (int)jn : -1;
        if (shp) {
            pc.w = __int_as_float(next_idx);
            q.so[0][jp] = po;
            q.sd[0][jp] = pd;
            q.sc[0][jp] = pc;
            q.st[0][jp] = ptmax;
            aq.sproj[0][jp] = pxp;
            aq.suv[0][jp] = pxt;
            aq.sg[0][jp] = pg;
            aq.sa[0][jp] = pa;
            aq.ss[0][jp] = ps;
        }
        if (she) {
            ec.w = __int_as_float(next_idx);
            q.so[1][je] = eo;
            q.sd[1][je] = ed;
            q.sc[1][je] = ec;
            q.st[1][je] = __builtin_inff();
            aq.suv[1][je] = ext;
            aq.sg[1][je] = make_float4(0.f, 0.f, 0.f, 0.f);
            aq.sa[1][je] = ea;
            aq.ss[1][je] = es;
        }
    }
}

// ---------------------------------------------------------------- shadows
// PROF: the counting pass's instantiation (visit counters summed into q.stats)
template <bool UNI, bool PROF>
__global__ void __launch_bounds__(TB) ADJ_SHADOW_OCCUPANCY k_adj_shadow(Queues q, AdjQueues aq, int which, int nxt, ReqDesc uni,
                                                   const ReqDesc* __restrict__ table) {
    __shared__ int stack[(SHORT_STACK + 1) * TB];
    __shared__ float4 ltop[UNI ? 8 * TOP_NODES : 1];
    int* spill = q.spill + (size_t)blockIdx.x * TB * SPILL;
    const uint32_t n = q.cnt[shadow_slot(nxt ^ 1, which)];
    TopNodes top{nullptr, 0u};
    if constexpr (UNI)   // one tree for the whole launch: stage its top levels
        if (uni.nodes4) top = stage_top<TB>(ltop, uni.nodes4, uni.top_nodes);
    // the loop bound is uniform per workgroup so every lane reaches the wave-level scatter
    for (uint32_t base = blockIdx.x * TB; base < n; base += gridDim.x * TB) {
        const uint32_t i = base + threadIdx.x;
        const bool live = i < n;
        const uint32_t ii = live ? i : base;
        const float4 o = q.so[which][ii], d = q.sd[which][ii];
        const ReqDesc& r = sel<UNI>(uni, table, __float_as_int(o.w));
        bool occ = true;
        if (live) {
            Hit h;
            Visits<PROF> vis;
            occ = trace_ray<true, SHORT_STACK, TB>(r.nodes4, r.nodes, r.tris, xyz(o), xyz(d), r.tmin, q.st[which][i],
                                                  __float_as_int(d.w), h, stack, spill, threadIdx.x, vis, top);
            if constexpr (PROF)
                if (q.stats) {
                    atomicAdd(&q.stats[0], (unsigned long long)vis.nodes);
                    atomicAdd(&q.stats[1], (unsigned long long)vis.tris);
                }
        }
        const float4 c = q.sc[which][ii], a = aq.sa[which][ii];
        const double2 xt = aq.suv[which][ii];
        const double2 xp = which == 0 ? aq.sproj[0][ii] : make_double2(0.0, 0.0);
        const float sv = aq.ss[which][ii];
        if (!occ) {
            const int j = __float_as_int(c.w);
            if (j >= 0) {
                float4 rl = aq.rl[nxt][j];
                rl.x -= c.x;
                rl.y -= c.y;
                rl.z -= c.z;
                aq.rl[nxt][j] = rl;
            }
        }
        const float gt[5] = {a.x, a.y, a.z, a.w, sv};
        if (!UNI) {   // paths of several requests: per-lane atomics
            if (!occ) {
                if (which == 0 && r.dEp) {
                    const float4 gE = aq.sg[which][i];
                    const float ge[3] = {gE.x, gE.y, gE.z};
                    scatter_ep_lane(r, xp.x, xp.y, ge);
                }
                scatter_tex_lane(r, xt.x, xt.y, gt);
            }
            continue;
        }
        if (aq.tb.rec) {   // one request, binned flush: records (direct atomics if full)
            const bool vis = !occ;
            const bool to_e = vis && which == 0 && r.dEp && aq.eb.rec;
            const bool pred[2] = {vis, to_e};
            uint32_t* const ctr[2] = {aq.tb.count, aq.eb.count};
            uint32_t at[2];
            block_append<2, TB>(pred, ctr, at);
            if (vis && !put_tex_rec(aq.tb, at[0], xt.x, xt.y, gt)) scatter_tex_lane(r, xt.x, xt.y, gt);
            if (vis && which == 0 && r.dEp) {
                const float4 gE = aq.sg[which][i];
                const float ge[3] = {gE.x, gE.y, gE.z};
                if (!(to_e && put_ep_rec(aq.eb, at[1], xp.x, xp.y, ge))) scatter_ep_lane(r, xp.x, xp.y, ge);
            }
            continue;
        }
        // one request: lanes of one wave sum shared texels before the atomics
        if (which == 0 && r.dEp) {   // d/dE_p at the four projector texels
            const float4 gE = aq.sg[which][ii];
            const float ge[3] = {gE.x, gE.y, gE.z};
            scatter_ep(r, !occ, xp.x, xp.y, ge);
        }
        scatter_tex(r, !occ, xt.x, xt.y, gt);
    }
}

// lanes of the wave whose (12-bit) bin equals this lane's, among the valid lanes
__device__ __forceinline__ unsigned long long bin_peers(bool valid, uint32_t bin) {
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 12; ++bit) {
        const bool set = (bin >> bit) & 1u;
        const unsigned long long m = __ballot(set);
        peers &= set ? m : ~m;
    }
    return peers;
}
// LDS counter add aggregated over the lanes of a wave with the same bin; returns the
// counter's old value plus the lane's rank among those lanes.  Whole wave must call.
__device__ __forceinline__ uint32_t lds_bin_add(uint32_t* cnt, bool valid, uint32_t bin) {
    const unsigned long long peers = bin_peers(valid, bin);
    const int lane = __lane_id();
    const int leader = valid ? __ffsll(peers) - 1 : lane;
    uint32_t base = 0u;
    if (valid && lane == leader) base = atomicAdd(&cnt[bin], (uint32_t)__popcll(peers));
    base = (uint32_t)__shfl((int)base, leader);
    return base + (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ uint32_t map_records(const MapBins& mb) {
    const uint32_t n = *mb.count;
    return (int64_t)n < mb.cap ? n : (uint32_t)mb.cap;
}

// a record of RS floats into registers in 16-byte loads (8-byte ones for RS = 6); returns v
template <int RS>
__device__ __forceinline__ const float* load_record(const float* __restrict__ p, float* v) {
    if constexpr (RS % 4 == 0) {
#pragma unroll
        for (int k = 0; k < RS / 4; ++k) {
            const float4 x = ((const float4*)p)[k];
            v[4 * k] = x.x, v[4 * k + 1] = x.y, v[4 * k + 2] = x.z, v[4 * k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < RS / 2; ++k) {
            const float2 x = ((const float2*)p)[k];
            v[2 * k] = x.x, v[2 * k + 1] = x.y;
        }
    }
    return v;
}
// the store of load_record (16-byte aligned records)
template <int RS>
__device__ __forceinline__ void store_record(float* __restrict__ p, const float* v) {
    if constexpr (RS % 4 == 0) {
#pragma unroll
        for (int k = 0; k < RS / 4; ++k) ((float4*)p)[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < RS / 2; ++k) ((float2*)p)[k] = make_float2(v[2 * k], v[2 * k + 1]);
    }
}

// records per tile: workgroup histogram in LDS, then one returning atomic per touched
// tile, whose old value -- where this chunk's records start inside the tile's range --
// goes to rowbase for the placement; also the largest |cotangent| of any record (for
// the fixed-point accumulation)
template <int C, int RS>
__device__ __forceinline__ void bin_hist(const MapBins& mb, uint32_t chunk, uint32_t* h, uint32_t& hmax) {
    const uint32_t n = map_records(mb);
    const uint32_t b0 = chunk * BIN_CHUNK;
    if (b0 >= n) return;   // uniform per workgroup
    for (int k = threadIdx.x; k < mb.nb; k += BIN_TB) h[k] = 0u;
    if (threadIdx.x == 0) hmax = 0u;
    __syncthreads();
    const uint32_t e = min(n, b0 + BIN_CHUNK);
    float m = 0.f;
    for (uint32_t base = b0; base < e; base += BIN_TB) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < e;
        const float* p = mb.rec + (size_t)(valid ? i : b0) * RS;
        float v[RS];
        load_record<RS>(p, v);
        const uint32_t bin = valid ? (uint32_t)map_bin(mb, __float_as_uint(v[0])) : 0u;
        lds_bin_add(h, valid, bin);
        if (valid)
#pragma unroll
            for (int c = 0; c < C; ++c) m = fmaxf(m, fabsf(v[3 + c]));   // NaN is dropped here; see accum
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (__lane_id() == 0) atomicMax(&hmax, __float_as_uint(m));   // non-negative floats order as integers
    __syncthreads();
    uint32_t* const rb = mb.rowbase + (size_t)chunk * mb.nb;
    for (int k = threadIdx.x; k < mb.nb; k += BIN_TB)
        if (h[k]) rb[k] = atomicAdd(&mb.bins[k], h[k]);
    if (threadIdx.x == 0 && hmax) atomicMax(&mb.bins[3 * mb.nb + 1], hmax);
}
// the flush kernels serve two maps at once (their chunks fill the chip together):
// workgroups [0, ga) map a, the rest map b (none when only a is flushed)
template <int CA, int RSA, int CB, int RSB>
__global__ void __launch_bounds__(BIN_TB) k_bin_hist(MapBins a, MapBins b, uint32_t ga) {
    __shared__ uint32_t h[MAP_MAX_BINS];
    __shared__ uint32_t hmax;
    if (blockIdx.x < ga) bin_hist<CA, RSA>(a, blockIdx.x, h, hmax);
    else bin_hist<CB, RSB>(b, blockIdx.x - ga, h, hmax);
}

// tile offsets (exclusive scan of the counts, nb <= 4096); clears the counts
__device__ __forceinline__ void bin_scan(const MapBins& mb, uint32_t* part) {
    uint32_t* off = mb.bins + mb.nb;
    const int per = (mb.nb + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(b + per, mb.nb);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += mb.bins[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int i = b; i < e; ++i) {
        const uint32_t v = mb.bins[i];
        off[i] = run;
        run += v;
        mb.bins[i] = 0u;
    }
    if (threadIdx.x == 1023) off[mb.nb] = part[1023];
}
// workgroup 0: map a, workgroup 1: map b
__global__ void __launch_bounds__(1024) k_bin_scan(MapBins a, MapBins b) {
    __shared__ uint32_t part[1024];
    bin_scan(blockIdx.x == 0 ? a : b, part);
}

// copy every record to its tile's range: the chunk's start inside each tile from the
// histogram pass (rowbase), ranks inside the chunk from LDS atomics over the same records
// the histogram counted (entries of tiles the chunk does not touch are stale and never
// read).  The order of a tile's records does not matter: the accumulation's integer sums
// are exact.
template <int RS>
__device__ __forceinline__ void bin_place(const MapBins& mb, uint32_t chunk, uint32_t* cnt) {
    const uint32_t n = map_records(mb);
    const uint32_t b0 = chunk * BIN_CHUNK;
    if (b0 >= n) return;   // uniform per workgroup
    const uint32_t e = min(n, b0 + BIN_CHUNK);
    const uint32_t* off = mb.bins + mb.nb;
    const uint32_t* rb = mb.rowbase + (size_t)chunk * mb.nb;
    for (int k = threadIdx.x; k < mb.nb; k += BIN_TB) cnt[k] = off[k] + rb[k];
    __syncthreads();
    for (uint32_t base = b0; base < e; base += BIN_TB * BIN_U) {
        float v[BIN_U][RS];   // BIN_U whole records in flight per thread, stored from registers
        bool valid[BIN_U];
#pragma unroll
        for (int u = 0; u < BIN_U; ++u) {
            const uint32_t i = base + u * BIN_TB + threadIdx.x;
            valid[u] = i < e;
            load_record<RS>(mb.rec + (size_t)(valid[u] ? i : b0) * RS, v[u]);
        }
#pragma unroll
        for (int u = 0; u < BIN_U; ++u) {
            const uint32_t bin = valid[u] ? (uint32_t)map_bin(mb, __float_as_uint(v[u][0])) : 0u;
            const uint32_t pos = lds_bin_add(cnt, valid[u], bin);
            if (!valid[u] || (int64_t)pos >= mb.cap) continue;   // pos < cap always for consistent counts
            store_record<RS>(mb.sorted + (size_t)pos * RS, v[u]);
        }
    }
}
template <int RSA, int RSB>
__global__ void __launch_bounds__(BIN_TB) k_bin_place(MapBins a, MapBins b, uint32_t ga) {
    __shared__ uint32_t cnt[MAP_MAX_BINS];
    if (blockIdx.x < ga) bin_place<RSA>(a, blockIdx.x, cnt);
    else bin_place<RSB>(b, blockIdx.x - ga, cnt);
}

// Accumulation over fixed chunks of the tile-sorted records (balanced whatever the
// tile sizes): a workgroup walks the tiles its chunk covers and, per tile, sums the
// records in LDS over the tile plus one halo row/column and stores the (T + 1)^2 x C
// block at pair index chunk + tile (unique: both grow along the sorted records).
template <int C, int RS>
__device__ __forceinline__ void bin_accum(const MapBins& mb, uint32_t c, long long* t) {
    // Sums in 64-bit fixed point (integer LDS atomics are exact and much faster than
    // FP32 ones): values scaled by 2^E with |chunk sum| < 2^62 for every texel, i.e.
    // 2^-50 of the largest record value as resolution.  The chunk sums are stored as
    // integers, so the texel totals the gather forms do not depend on how the records
    // were split into chunks (which varies with the order atomics placed them in).
    const uint32_t* off = mb.bins + mb.nb;
    const uint32_t total = off[mb.nb];
    const uint32_t i0 = c * ACC_CHUNK;
    if (c == 0 && threadIdx.x == 0) *mb.count = 0u;   // the counting passes are done
    if (i0 >= total) return;   // uniform per workgroup
    const uint32_t i1 = min(total, i0 + ACC_CHUNK);
    const float gmax = __uint_as_float(mb.bins[3 * mb.nb + 1]);
    int ge = 0;
    frexpf(gmax, &ge);                              // gmax < 2^ge
    const int E = 62 - 12 - ge;                     // ACC_CHUNK = 2^12 contributions at most
    const double up = ldexp(1.0, E);
    if (c == 0 && threadIdx.x == 0) mb.bins[2 * mb.nb + 1] = (uint32_t)E;   // for the gather
    int lo = 0, hi = mb.nb;   // the tile holding record i0: last b with off[b] <= i0
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i0) lo = mid;
        else hi = mid;
    }
    int b = lo;
    const int S = mb.T + 1, SS = S * S * C;
    for (;;) {
        const uint32_t s0 = max(off[b], i0), s1 = min(off[b + 1], i1);
        for (int k = threadIdx.x; k < SS; k += ACC_TB) t[k] = 0;
        __syncthreads();
        const int tx0 = (b % mb.nbx) * mb.T, ty0 = (b / mb.nbx) * mb.T;
        bool bad = false;
        float rv[RS];
        // The samples of one pixel sit together in the sorted records and share texels,
        // and an LDS atomic instruction whose lanes meet at one address is serialised: the
        // lanes of a wave take records m = ceil(n / 64) apart (lane l: slot [l m, l m + m)
        // of the tile's n records), i.e. from different pixels
        const uint32_t n = s1 - s0, m = (n + 63u) >> 6;
        for (uint32_t k = threadIdx.x; k < 64u * m; k += ACC_TB) {
            const uint32_t j = (k & 63u) * m + (k >> 6);
            if (j >= n) continue;
            const float* p = load_record<RS>(mb.sorted + (size_t)(s0 + j) * RS, rv);
            const uint32_t head = __float_as_uint(p[0]);
            const uint32_t base = head & 0x0fffffffu;
            const int y0 = (int)(base / (uint32_t)mb.W), x0 = (int)(base - (uint32_t)y0 * (uint32_t)mb.W);
            const int lx = x0 - tx0, ly = y0 - ty0;
            const int dx = (int)((head >> 28) & 1u), dy = (int)((head >> 29) & 1u);
            const double ax = p[1], ay = p[2];
            const double w[4] = {(1.0 - ax) * (1.0 - ay), ax * (1.0 - ay), (1.0 - ax) * ay, ax * ay};
            const int idx[4] = {ly * S + lx, ly * S + lx + dx, (ly + dy) * S + lx, (ly + dy) * S + lx + dx};
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const double g = (double)p[3 + ch] * up;
                bad = bad || !(fabs(g) <= 0x1p62);       // non-finite cotangent
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const long long q = bad ? 0ll : __double2ll_rn(g * w[k]);
                    if (q != 0ll) atomicAdd((unsigned long long*)&t[idx[k] * C + ch], (unsigned long long)q);
                }
            }
        }
        const bool any_bad = __syncthreads_or(bad);
        long long* st = mb.stage + (size_t)(c + b) * SS;
        for (int k = threadIdx.x; k < SS; k += ACC_TB) st[k] = any_bad ? STAGE_NAN : t[k];
        __syncthreads();
        if (off[b + 1] >= i1) break;
        ++b;
        while (off[b + 1] == off[b]) ++b;   // skip empty tiles (a later tile holds record i1 - 1)
    }
}
template <int CA, int RSA, int CB, int RSB>
__global__ void __launch_bounds__(ACC_TB) k_bin_accum(MapBins a, MapBins b, uint32_t ga) {
    __shared__ long long t[(MAP_MAX_T + 1) * (MAP_MAX_T + 1) * (CA > CB ? CA : CB)];
    if (blockIdx.x < ga) bin_accum<CA, RSA>(a, blockIdx.x, t);
    else bin_accum<CB, RSB>(b, blockIdx.x - ga, t);
}

// one thread per texel: the blocks of every (chunk, tile) pair of its own tile plus
// the halos of the tiles to the left, above and above-left, added into the map (each
// texel written by one thread)
template <int C>
__device__ __forceinline__ void bin_gather(const MapBins& mb, float* __restrict__ out, int stride, int64_t t) {
    if (t == 0) mb.bins[3 * mb.nb + 1] = 0u;   // largest |value|: read by the accumulation only
    if (t >= (int64_t)mb.W * mb.H) return;
    const int y = (int)(t / mb.W), x = (int)(t - (int64_t)y * mb.W);
    const int T = mb.T, S = T + 1, SS = S * S * C;
    const int tx = x / T, ty = y / T, lx = x - tx * T, ly = y - ty * T;
    const uint32_t* off = mb.bins + mb.nb;
    // exact 128-bit two's-complement totals of the integer block sums (a texel can take
    // more blocks than 64 bits hold), converted to floating point once
    unsigned long long lo[C];
    long long hi[C];
    bool nan = false;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
        lo[ch] = 0ull;
        hi[ch] = 0ll;
    }
    auto add = [&](int bx, int by, int ix, int iy) {
        const int b = by * mb.nbx + bx;
        const uint32_t a = off[b], e = off[b + 1];
        if (a == e) return;
        for (uint32_t c = a / ACC_CHUNK; c <= (e - 1) / ACC_CHUNK; ++c) {
            const long long* p = mb.stage + (size_t)(c + b) * SS + ((size_t)iy * S + ix) * C;
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const long long q = p[ch];
                nan = nan || q == STAGE_NAN;
                const unsigned long long s = lo[ch] + (unsigned long long)q;
                hi[ch] += (q < 0 ? -1ll : 0ll) + (s < lo[ch] ? 1ll : 0ll);
                lo[ch] = s;
            }
        }
    };
    add(tx, ty, lx, ly);
    if (lx == 0 && tx > 0) add(tx - 1, ty, T, ly);
    if (ly == 0 && ty > 0) add(tx, ty - 1, lx, T);
    if (lx == 0 && ly == 0 && tx > 0 && ty > 0) add(tx - 1, ty - 1, T, T);
    const double down = ldexp(1.0, -(int)mb.bins[2 * mb.nb + 1]);
    float* o = out + (size_t)t * stride;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
        // magnitude and sign (no cancellation between the two halves), then 2^-E
        const bool neg = hi[ch] < 0;
        unsigned long long ml = lo[ch], mh = (unsigned long long)hi[ch];
        if (neg) {
            ml = ~ml + 1ull;
            mh = ~mh + (ml == 0ull ? 1ull : 0ull);
        }
        const double m = ((double)mh * 0x1p64 + (double)ml) * down;
        const float v = nan ? __builtin_nanf("") : (float)(neg ? -m : m);
        if (v != 0.f) o[ch] += v;
    }
}
template <int CA, int CB>
__global__ void __launch_bounds__(256) k_bin_gather(MapBins a, float* __restrict__ oa, int sa, MapBins b,
                                                    float* __restrict__ ob, int sb, uint32_t ga) {
    if (blockIdx.x < ga) bin_gather<CA>(a, oa, sa, (int64_t)blockIdx.x * 256 + threadIdx.x);
    else bin_gather<CB>(b, ob, sb, (int64_t)(blockIdx.x - ga) * 256 + threadIdx.x);
}

// ---------------------------------------------------------------- replay from records
// The replay's queue sizes rotate over three slots, q.cnt[REPLAY_CNT + (depth mod 3)]:
// a launch reads its own, appends to the next and empties the one after (read by the
// launch before, untouched by this one; replay_count_clear), so no launch between depths
// resets a count.  The caller starts depth 0 with its slot = queue size, the next = 0.
__device__ __forceinline__ uint32_t* replay_count(const Queues& q, int depth) {
    return q.cnt + REPLAY_CNT + depth % 3;
}
// Called by workgroup 0 after its last read of the counts: a store ahead of the size's
// read turns that read from a scalar load into a vector load per wave, which made the
// whole launch several times slower.
__device__ __forceinline__ void replay_count_clear(const Queues& q, int depth) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(replay_count(q, depth + 2), 0u);
}
// One bounce of the replay when the forward kept its path records: the vertex's leaf and
// the visibility of its shadow rays are read instead of traced.  Shading, the
// next-event terms and the bounce are re-evaluated with the forward's Philox counters.
// The next-event cotangents on the BRDF maps at this vertex travel with the path and
// are added to its bounce derivative when that is settled at the next vertex, so each
// vertex scatters into the maps once (twice where the path ends).
template <bool UNI>
__global__ void __launch_bounds__(BLOCK) k_adj_replay(Queues q, AdjQueues aq, int cur, int depth, ReqDesc uni,
                                                      const ReqDesc* __restrict__ table) {
    const int nxt = cur ^ 1;
    const uint32_t n = *replay_count(q, depth);
    // one path per thread (the grid covers the queue): with no grid-stride loop no
    // descriptor field is held across iterations, which saves ~60 VGPRs
    const uint32_t base = blockIdx.x * BLOCK;
    if (base >= n) {   // uniform per workgroup
        replay_count_clear(q, depth);
        return;
    }
    {
        const uint32_t i = base + threadIdx.x;
        bool cont = false;
        PathO no{};
        PathD nd{};
        float4 nb = {}, nrl = {}, npenda = {}, npn = {};
        float2 npend = {};
        double2 npuv = {};
        float npns = 0.f;
        // map cotangents of the previous vertex (a) and of this one when the path ends here (b)
        bool a_on = false, b_on = false, e_on = false;
        double a_u = 0.0, a_v = 0.0, b_u = 0.0, b_v = 0.0;
        float ag[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, bg[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        // E_p cotangent of this vertex's projector term
        double e_pu = 0.0, e_pv = 0.0;
        float eg[3] = {0.f, 0.f, 0.f};
        int lslot = -1;   // request slot of this lane's path (-1: no path)
        const ReqDesc* rp = &sel<UNI>(uni, table, 0);
        if (i < n) {
            PathO o;
            PathD dd;
            float4 b, rl, penda;
            // the previous vertex's pending cotangents (read when penda.w >= 0)
            float2 pend = {};
            double2 puv = {};
            float4 pn = {};
            float pns = 0.f;
            if (UNI && depth == 0) {
                // the dense camera wave (queue index = batch sample index): the ray is
                // regenerated as the forward's raygen made it instead of read back
                const uint32_t g = i - uni.sid_base + uni.g_base;
                const D3 cd = camera_dir(uni, g);
                o = PathO{uni.cam_o[0], uni.cam_o[1], uni.cam_o[2], 0, -1};
                dd = PathD{cd.x, cd.y, cd.z, g, 0u};
                b = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
                rl = q.L[i];                                  // remaining radiance = the sample's total
                penda = make_float4(0.f, 0.f, 0.f, -1.f);     // no pending bounce
            } else {
                o = nt_ld(&q.po[cur][i]);
                dd = nt_ld(&q.pd[cur][i]);
                b = nt_ld(&q.pb[cur][i]);
                if (depth == 0) {   // camera wave of several requests: as above, from the queue's rays
                    rl = q.L[i];
                    penda = make_float4(0.f, 0.f, 0.f, -1.f);
                } else {
                    rl = nt_ld(&aq.rl[cur][i]);
                    penda = nt_ld(&aq.penda[cur][i]);
                    // loaded with the path state (every path past depth 0 bounced, so
                    // they are nearly always used): behind the penda.w test they cost a
                    // further trip to memory
                    pend = nt_ld(&aq.pend[cur][i]);
                    puv = nt_ld(&aq.puv[cur][i]);
                    pn = nt_ld(&aq.pn[cur][i]);
                    pns = nt_ld(&aq.pns[cur][i]);
                }
            }
            const ReqDesc& r = sel<UNI>(uni, table, o.slot);
            rp = &r;
            lslot = o.slot;
            const uint32_t g = dd.g;
            const uint32_t sid = g - r.g_base + r.sid_base;
            const uint32_t rec = __builtin_nontemporal_load(&r.rec[(size_t)(g - r.rec_g0) * r.max_depth + depth]);
            const int leaf = (int)(rec & REC_LEAF) - 1;
            const float4 dl = aq.delta[sid];
            const D3 delta = d3(dl.x, dl.y, dl.z);
            const D3 beta = d3(b.x, b.y, b.z);
            if (penda.w >= 0.f) {
                // previous vertex: its next-event cotangents plus d/df of its bounce,
                // beta_k f cos/pdf R_{k+1} -> R_{k+1} / f (zero when this ray escaped)
                a_on = true;
                a_u = puv.x;
                a_v = puv.y;
                double ga0 = pn.x, ga1 = pn.y, ga2 = pn.z, gr = pn.w, gs = pns;
                if (leaf >= 0) {
                    const D3 t = delta * d3(rl.x, rl.y, rl.z) * d3(penda.x, penda.y, penda.z);
                    const double sum = t.x + t.y + t.z;
                    ga0 += t.x * (1.0 / PI);
                    ga1 += t.y * (1.0 / PI);
                    ga2 += t.z * (1.0 / PI);
                    gr += sum * pend.x;
                    gs += sum * pend.y;
                }
                ag[0] = (float)ga0;
                ag[1] = (float)ga1;
                ag[2] = (float)ga2;
                ag[3] = (float)gr;
                ag[4] = (float)gs;
            }
            if (leaf >= 0) {
                const Surf s = surface(r, leaf, d3(o.x, o.y, o.z), d3(dd.x, dd.y, dd.z));
                if (r.emission) {
                    const float4 e = r.emission[leaf];
                    rl.x -= (float)(beta.x * e.x);
                    rl.y -= (float)(beta.y * e.y);
                    rl.z -= (float)(beta.z * e.z);
                }
                const D3 db = delta * beta;
                D3 nga = d3(0., 0., 0.);
                double ngr = 0.0, ngs = 0.0;
                ProjNee p;
                if ((rec & REC_PRJ) && projector_nee(r, s, p)) {
                    const D4 E = fetch4(r.Ep, p.pb);
                    const Brdf f = brdf_eval<true>(r.brdf, s.n, s.wo, p.wp, s.alb, s.rough, s.spec);
                    const D3 Ex = d3(E.x, E.y, E.z) * p.geom;
                    const D3 C = beta * f.f * Ex;
                    const D3 gE = db * f.f * p.geom;   // d/dE_p before the bilinear weights
                    const double sx = db.x * Ex.x + db.y * Ex.y + db.z * Ex.z;
                    e_on = r.dEp != nullptr;
                    e_pu = p.pu;
                    e_pv = p.pv;
                    eg[0] = (float)gE.x;
                    eg[1] = (float)gE.y;
                    eg[2] = (float)gE.z;
                    nga = nga + db * Ex * (1.0 / PI);
                    ngr += sx * f.ds_dr;
                    ngs += sx * f.ds_dsp;
                    rl.x -= (float)C.x;
                    rl.y -= (float)C.y;
                    rl.z -= (float)C.z;
                }
                if (r.env_on && (rec & REC_ENV)) {
                    const U4 x = vertex_rng(r, g, 2u + 2u * depth);
                    const D3 we = sample_cosine(s.n, u24(x.x), u24(x.y));
                    const Brdf f = brdf_eval<true>(r.brdf, s.n, s.wo, we, s.alb, s.rough, s.spec);
                    const D3 Ee = d3(r.env[0], r.env[1], r.env[2]) * PI;
                    const D3 C = beta * f.f * Ee;
                    const double sx = db.x * Ee.x + db.y * Ee.y + db.z * Ee.z;
                    nga = nga + db * Ee * (1.0 / PI);
                    ngr += sx * f.ds_dr;
                    ngs += sx * f.ds_dsp;
                    rl.x -= (float)C.x;
                    rl.y -= (float)C.y;
                    rl.z -= (float)C.z;
                }
                if (depth < r.max_depth - 1) {
                    const U4 x = vertex_rng(r, g, 1u + 2u * depth);
                    const D3 wi = sample_bounce(r.brdf, s.n, s.wo, s.rough, u24(x.x), u24(x.y), u24(x.z));
                    const double ci = dot(s.n, wi);
                    const double pdf = bounce_pdf(r.brdf, s.n, s.wo, wi, s.rough);
                    if (ci > 0.0 && pdf > 0.0) {
                        const Brdf f = brdf_eval<true>(r.brdf, s.n, s.wo, wi, s.alb, s.rough, s.spec);
                        const D3 nbeta = beta * (f.f * (ci / pdf));
                        cont = true;
                        no = PathO{s.x.x, s.x.y, s.x.z, o.slot, s.prim};
                        nd = PathD{wi.x, wi.y, wi.z, g, 0u};
                        nb = make_float4((float)nbeta.x, (float)nbeta.y, (float)nbeta.z, 0.0f);
                        nrl = rl;
                        npuv = make_double2(s.u, s.v);
                        npend = make_float2((float)f.ds_dr, (float)f.ds_dsp);
                        npenda = make_float4(f.f.x > 0.0 ? (float)(1.0 / f.f.x) : 0.f,
                                             f.f.y > 0.0 ? (float)(1.0 / f.f.y) : 0.f,
                                             f.f.z > 0.0 ? (float)(1.0 / f.f.z) : 0.f, 1.f);
                        npn = make_float4((float)nga.x, (float)nga.y, (float)nga.z, (float)ngr);
                        npns = (float)ngs;
                    }
                }
                if (!cont) {   // the path ends here: its next-event cotangents go out now
                    b_on = true;
                    b_u = s.u;
                    b_v = s.v;
                    bg[0] = (float)nga.x;
                    bg[1] = (float)nga.y;
                    bg[2] = (float)nga.z;
                    bg[3] = (float)ngr;
                    bg[4] = (float)ngs;
                }
            }
        }
        if (UNI && aq.tb.rec) {   // records for the binned flush (direct atomics if full)
            const bool to_e = e_on && aq.eb.rec;
            const bool pred[3] = {a_on, b_on, to_e};
            uint32_t* const ctr[3] = {aq.tb.count, aq.tb.count, aq.eb.count};
            uint32_t at[3];
            block_append<3>(pred, ctr, at);
            if (a_on && !put_tex_rec(aq.tb, at[0], a_u, a_v, ag)) scatter_tex_lane(*rp, a_u, a_v, ag);
            if (b_on && !put_tex_rec(aq.tb, at[1], b_u, b_v, bg)) scatter_tex_lane(*rp, b_u, b_v, bg);
            if (e_on && !(to_e && put_ep_rec(aq.eb, at[2], e_pu, e_pv, eg))) scatter_ep_lane(*rp, e_pu, e_pv, eg);
        } else if (UNI) {
            scatter_tex(*rp, a_on, a_u, a_v, ag);
            scatter_tex(*rp, b_on, b_u, b_v, bg);
            if (rp->dEp) scatter_ep(*rp, e_on, e_pu, e_pv, eg);
        } else {
            // several requests: when every path of this wave belongs to one of them (the
            // usual case, segments are contiguous) the wave still sums shared texels
            const unsigned long long vm = __ballot(lslot >= 0);
            const int s0 = vm ? __shfl(lslot, __ffsll(vm) - 1) : -1;
            if (s0 >= 0 && __ballot(lslot >= 0 && lslot != s0) == 0ull) {
                const ReqDesc& rr = table[s0];
                scatter_tex(rr, a_on, a_u, a_v, ag);
                scatter_tex(rr, b_on, b_u, b_v, bg);
                if (rr.dEp) scatter_ep(rr, e_on, e_pu, e_pv, eg);
            } else {
                if (a_on) scatter_tex_lane(*rp, a_u, a_v, ag);
                if (b_on) scatter_tex_lane(*rp, b_u, b_v, bg);
                if (e_on) scatter_ep_lane(*rp, e_pu, e_pv, eg);
            }
        }
        const bool pred[1] = {cont};
        uint32_t* const ctr[1] = {replay_count(q, depth + 1)};
        uint32_t jn;
        block_append<1>(pred, ctr, &jn);
        replay_count_clear(q, depth);
        if (cont) {
            nt_st(&q.po[nxt][jn], no);
            nt_st(&q.pd[nxt][jn], nd);
            nt_st(&q.pb[nxt][jn], nb);
            nt_st(&aq.rl[nxt][jn], nrl);
            nt_st(&aq.pend[nxt][jn], npend);
            nt_st(&aq.puv[nxt][jn], npuv);
            nt_st(&aq.penda[nxt][jn], npenda);
            nt_st(&aq.pn[nxt][jn], npn);
            nt_st(&aq.pns[nxt][jn], npns);
        }
    }
}

// ---------------------------------------------------------------- replay, metallic and normal maps
// k_adj_replay for a request with the metallic and normal maps (one request per launch).
// Every term of a vertex is beta_c f_c c S_c with c the cosine about the shading normal
// and S_c its remaining factor: E_c / (cos^3 alpha d^2) for the projector, L_env pi / c
// for the environment (the sampling pdf c / pi held fixed), R_{k+1} / pdf for the bounce;
// its derivative w.r.t. a map value is beta_c d(f_c c) S_c.  For the bounce S_c is only
// known at the next vertex, where beta_c f_c c S_c = its remaining radiance rl_c: the
// vertex leaves the coefficients d(f_c c)/d theta / (f_c c) (PendX), the next one
// multiplies them by delta_c rl_c.  Normal cotangents are carried in the stored map
// values (through the vertex's frame), so the records hold 9 channels.
__global__ void __launch_bounds__(BLOCK) k_adj_replay_ext(Queues q, AdjQueues aq, int cur, int depth, ReqDesc r) {
    const int nxt = cur ^ 1;
    const uint32_t n = *replay_count(q, depth);
    const uint32_t base = blockIdx.x * BLOCK;
    if (base >= n) {   // uniform per workgroup
        replay_count_clear(q, depth);
        return;
    }
    const uint32_t i = base + threadIdx.x;
    bool cont = false;
    PathO no{};
    PathD nd{};
    float4 nb = {}, nrl = {}, npn = {}, npnx = {};
    PendX npx{};
    double2 npuv = {};
    float npns = 0.f;
    bool a_on = false, b_on = false, e_on = false;
    double a_u = 0.0, a_v = 0.0, b_u = 0.0, b_v = 0.0;
    float ag[9] = {}, bg[9] = {};
    double e_pu = 0.0, e_pv = 0.0;
    float eg[3] = {0.f, 0.f, 0.f};
    if (i < n) {
        PathO o;
        PathD dd;
        float4 b, rl, penda;
        if (depth == 0) {   // the dense camera wave, regenerated as the forward's raygen made it
            const uint32_t g = i - r.sid_base + r.g_base;
            const D3 cd = camera_dir(r, g);
            o = PathO{r.cam_o[0], r.cam_o[1], r.cam_o[2], 0, -1};
            dd = PathD{cd.x, cd.y, cd.z, g, 0u};
            b = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
            rl = q.L[i];
            penda = make_float4(0.f, 0.f, 0.f, -1.f);
        } else {
            o = nt_ld(&q.po[cur][i]);
            dd = nt_ld(&q.pd[cur][i]);
            b = nt_ld(&q.pb[cur][i]);
            rl = nt_ld(&aq.rl[cur][i]);
            penda = nt_ld(&aq.penda[cur][i]);
        }
        const uint32_t g = dd.g;
        const uint32_t sid = g - r.g_base + r.sid_base;
        const uint32_t rec = __builtin_nontemporal_load(&r.rec[(size_t)(g - r.rec_g0) * r.max_depth + depth]);
        const int leaf = (int)(rec & REC_LEAF) - 1;
        const float4 dl = aq.delta[sid];
        const D3 delta = d3(dl.x, dl.y, dl.z);
        const D3 beta = d3(b.x, b.y, b.z);
        if (penda.w >= 0.f) {   // settle the previous vertex: its next-event cotangents and its bounce
            const double2 puv = nt_ld(&aq.puv[cur][i]);
            const float4 pn = nt_ld(&aq.pn[cur][i]);
            const float pns = nt_ld(&aq.pns[cur][i]);
            const float4 pnx = nt_ld(&aq.pnx[cur][i]);
            a_on = true;
            a_u = puv.x;
            a_v = puv.y;
            double ga[9] = {pn.x, pn.y, pn.z, pn.w, pns, pnx.x, pnx.y, pnx.z, pnx.w};
            if (leaf >= 0) {
                const PendX P = nt_ld(&aq.px[cur][i]);
                const double w[3] = {delta.x * rl.x, delta.y * rl.y, delta.z * rl.z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ga[c] += w[c] * P.a[c];
                    ga[3] += w[c] * P.r[c];
                    ga[4] += w[c] * P.s[c];
                    ga[5] += w[c] * P.m[c];
                    ga[6] += w[c] * P.n[3 * c];
                    ga[7] += w[c] * P.n[3 * c + 1];
                    ga[8] += w[c] * P.n[3 * c + 2];
                }
            }
#pragma unroll
            for (int j = 0; j < 9; ++j) ag[j] = (float)ga[j];
        }
        if (leaf >= 0) {
            const Surf s = surface(r, leaf, d3(o.x, o.y, o.z), d3(dd.x, dd.y, dd.z));
            const Shading sh = shading(r, leaf, s);
            if (r.emission) {
                const float4 e = r.emission[leaf];
                rl.x -= (float)(beta.x * e.x);
                rl.y -= (float)(beta.y * e.y);
                rl.z -= (float)(beta.z * e.z);
            }
            const D3 db = delta * beta;
            double ng[6] = {0., 0., 0., 0., 0., 0.};   // albedo rgb, roughness, specular, metallic
            D3 gnv = d3(0., 0., 0.);                   // cotangent of the shading normal
            auto term = [&](const BrdfX& f, D3 S) {    // cotangents of beta_c f_c c S_c
                const D3 cs = S * f.c;
                ng[0] += db.x * f.dfa * cs.x;
                ng[1] += db.y * f.dfa * cs.y;
                ng[2] += db.z * f.dfa * cs.z;
                ng[3] += db.x * f.dfr.x * cs.x + db.y * f.dfr.y * cs.y + db.z * f.dfr.z * cs.z;
                ng[4] += (db.x * cs.x + db.y * cs.y + db.z * cs.z) * f.dfs;
                ng[5] += db.x * f.dfm.x * cs.x + db.y * f.dfm.y * cs.y + db.z * f.dfm.z * cs.z;
                gnv = gnv + f.dn[0] * (db.x * S.x) + f.dn[1] * (db.y * S.y) + f.dn[2] * (db.z * S.z);
            };
            ProjNee p;
            if ((rec & REC_PRJ) && projector_nee(r, s, p)) {
                const D4 E = fetch4(r.Ep, p.pb);
                const BrdfX f = brdf_x<true>(r.brdf, s.n, sh.ns, s.wo, p.wp, s.alb, s.rough, s.spec, sh.metal);
                const D3 S = d3(E.x, E.y, E.z) * p.g0;
                const D3 C = beta * f.f * S * f.c;
                const D3 gE = db * f.f * (f.c * p.g0);   // d/dE_p before the bilinear weights
                e_on = r.dEp != nullptr;
                e_pu = p.pu;
                e_pv = p.pv;
                eg[0] = (float)gE.x;
                eg[1] = (float)gE.y;
                eg[2] = (float)gE.z;
                term(f, S);
                rl.x -= (float)C.x;
                rl.y -= (float)C.y;
                rl.z -= (float)C.z;
            }
            if (r.env_on && (rec & REC_ENV)) {
                const U4 x = vertex_rng(r, g, 2u + 2u * depth);
                const D3 we = sample_cosine(sh.ns, u24(x.x), u24(x.y));
                const BrdfX f = brdf_x<true>(r.brdf, s.n, sh.ns, s.wo, we, s.alb, s.rough, s.spec, sh.metal);
                const D3 Le = d3(r.env[0], r.env[1], r.env[2]);
                const D3 C = beta * f.f * Le * PI;
                if (f.c > 0.0) term(f, Le * (PI / f.c));
                rl.x -= (float)C.x;
                rl.y -= (float)C.y;
                rl.z -= (float)C.z;
            }
            const D3 gnm = nmap_cotangent(sh, s.n, gnv);
            if (depth < r.max_depth - 1) {
                const U4 x = vertex_rng(r, g, 1u + 2u * depth);
                const D3 wi = sample_bounce(r.brdf, sh.ns, s.wo, s.rough, u24(x.x), u24(x.y), u24(x.z));
                const double ci = dot(s.n, wi);
                const double pdf = bounce_pdf(r.brdf, sh.ns, s.wo, wi, s.rough);
                if (ci > 0.0 && pdf > 0.0) {
                    const BrdfX f = brdf_x<true>(r.brdf, s.n, sh.ns, s.wo, wi, s.alb, s.rough, s.spec, sh.metal);
                    const D3 nbeta = beta * (f.f * (f.c / pdf));
                    cont = true;
                    no = PathO{s.x.x, s.x.y, s.x.z, o.slot, s.prim};
                    nd = PathD{wi.x, wi.y, wi.z, g, 0u};
                    nb = make_float4((float)nbeta.x, (float)nbeta.y, (float)nbeta.z, 0.0f);
                    nrl = rl;
                    npuv = make_double2(s.u, s.v);
                    const double fv[3] = {f.f.x, f.f.y, f.f.z};
                    const double dfr[3] = {f.dfr.x, f.dfr.y, f.dfr.z}, dfm[3] = {f.dfm.x, f.dfm.y, f.dfm.z};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double inv = fv[c] > 0.0 ? 1.0 / fv[c] : 0.0;
                        npx.a[c] = (float)(f.dfa * inv);
                        npx.r[c] = (float)(dfr[c] * inv);
                        npx.s[c] = (float)(f.dfs * inv);
                        npx.m[c] = (float)(dfm[c] * inv);
                        const D3 pn = nmap_cotangent(sh, s.n, f.dn[c]) * (inv / f.c);
                        npx.n[3 * c] = (float)pn.x;
                        npx.n[3 * c + 1] = (float)pn.y;
                        npx.n[3 * c + 2] = (float)pn.z;
                    }
                    npn = make_float4((float)ng[0], (float)ng[1], (float)ng[2], (float)ng[3]);
                    npns = (float)ng[4];
                    npnx = make_float4((float)ng[5], (float)gnm.x, (float)gnm.y, (float)gnm.z);
                }
            }
            if (!cont) {   // the path ends here: its next-event cotangents go out now
                b_on = true;
                b_u = s.u;
                b_v = s.v;
#pragma unroll
                for (int j = 0; j < 6; ++j) bg[j] = (float)ng[j];
                bg[6] = (float)gnm.x;
                bg[7] = (float)gnm.y;
                bg[8] = (float)gnm.z;
            }
        }
    }
    if (aq.tb.rec) {   // records for the binned flush (direct atomics if full)
        const bool to_e = e_on && aq.eb.rec;
        const bool pred[3] = {a_on, b_on, to_e};
        uint32_t* const ctr[3] = {aq.tb.count, aq.tb.count, aq.eb.count};
        uint32_t at[3];
        block_append<3>(pred, ctr, at);
        if (a_on && !put_tex9_rec(aq.tb, at[0], a_u, a_v, ag)) scatter_tex9_lane(r, a_u, a_v, ag);
        if (b_on && !put_tex9_rec(aq.tb, at[1], b_u, b_v, bg)) scatter_tex9_lane(r, b_u, b_v, bg);
        if (e_on && !(to_e && put_ep_rec(aq.eb, at[2], e_pu, e_pv, eg))) scatter_ep_lane(r, e_pu, e_pv, eg);
    } else {
        scatter_tex9(r, a_on, a_u, a_v, ag);
        scatter_tex9(r, b_on, b_u, b_v, bg);
        if (r.dEp) scatter_ep(r, e_on, e_pu, e_pv, eg);
    }
    const bool pred[1] = {cont};
    uint32_t* const ctr[1] = {replay_count(q, depth + 1)};
    uint32_t jn;
    block_append<1>(pred, ctr, &jn);
    replay_count_clear(q, depth);
    if (cont) {
        nt_st(&q.po[nxt][jn], no);
        nt_st(&q.pd[nxt][jn], nd);
        nt_st(&q.pb[nxt][jn], nb);
        nt_st(&aq.rl[nxt][jn], nrl);
        nt_st(&aq.puv[nxt][jn], npuv);
        nt_st(&aq.penda[nxt][jn], make_float4(0.f, 0.f, 0.f, 1.f));
        nt_st(&aq.pn[nxt][jn], npn);
        nt_st(&aq.pns[nxt][jn], npns);
        nt_st(&aq.pnx[nxt][jn], npnx);
        nt_st(&aq.px[nxt][jn], npx);
    }
}

// ---------------------------------------------------------------- finish
// Eq. 1 backward per texel: z = g_p M y, y = I_p^gamma_p, E_p = max(0, z)
__device__ __forceinline__ void adj_maps(const ReqDesc& r, int t, float* d_albedo, float* d_rough, float* d_spec,
                                         float* d_metal, float* d_nmap);
// workgroups [0, gp): the PRF backward per projector texel (per-block partials of the
// 12 scalars); the rest: the map cotangents copied out per texel (adj_maps)
__global__ void __launch_bounds__(BLOCK) k_adj_prf(ReqDesc r, float* __restrict__ d_proj, float* __restrict__ acc,
                                                   int gp, float* d_albedo, float* d_rough, float* d_spec,
                                                   float* d_metal, float* d_nmap) {
    if ((int)blockIdx.x >= gp) {   // uniform per workgroup
        adj_maps(r, (blockIdx.x - gp) * BLOCK + threadIdx.x, d_albedo, d_rough, d_spec, d_metal, d_nmap);
        return;
    }
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float part[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // d gamma_p[3], d M[9]
    if (t < r.Wp * r.Hp) {
        float x[3], y[3], z[3], dz[3];
        for (int c = 0; c < 3; ++c) {
            x[c] = r.proj_image[3 * (size_t)t + c];
            y[c] = x[c] > 0.f ? powf(x[c], scalar(r, c)) : 0.f;
        }
        for (int c = 0; c < 3; ++c) {
            z[c] = r.prf_gain * (scalar(r, 3 + 3 * c) * y[0] + scalar(r, 4 + 3 * c) * y[1] + scalar(r, 5 + 3 * c) * y[2]);
            dz[c] = z[c] > 0.f ? r.dEp[4 * (size_t)t + c] : 0.f;
        }
        for (int c = 0; c < 3; ++c) {
            const float dy = r.prf_gain * (scalar(r, 3 + c) * dz[0] + scalar(r, 6 + c) * dz[1] + scalar(r, 9 + c) * dz[2]);
            float di = 0.f;
            if (x[c] > 0.f) {
                const float gp = scalar(r, c);
                di = dy * gp * powf(x[c], gp - 1.f);
                part[c] = dy * y[c] * logf(x[c]);
            }
            if (d_proj) d_proj[3 * (size_t)t + c] = di;
            for (int k = 0; k < 3; ++k) part[3 + 3 * c + k] = r.prf_gain * dz[c] * y[k];
        }
    }
    __shared__ float red[12][BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 12; ++k) {
        float v = part[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        float v = 0.f;
        for (int k = 0; k < BLOCK / 64; ++k) v += red[threadIdx.x][k];
        if (r.d_part) r.d_part[12 * (size_t)blockIdx.x + threadIdx.x] = v;
        else if (v != 0.f) atomicAdd(&acc[8 + threadIdx.x], v);
    }
}

// scalar gradients and the de-interleaving of the map cotangents
__device__ __forceinline__ void adj_maps(const ReqDesc& r, int t, float* d_albedo, float* d_rough, float* d_spec,
                                         float* d_metal, float* d_nmap) {
    if (t >= r.tw * r.th) return;
    const float* s = r.d_tex + (size_t)r.dtex_c * t;
    if (r.dtex_c == 9) {
        if (d_metal) d_metal[t] = r.brdf ? s[5] : 0.f;
        if (d_nmap) {
            d_nmap[3 * (size_t)t] = s[6];
            d_nmap[3 * (size_t)t + 1] = s[7];
            d_nmap[3 * (size_t)t + 2] = s[8];
        }
    } else {
        if (d_metal) d_metal[t] = 0.f;
        if (d_nmap) {
            d_nmap[3 * (size_t)t] = 0.f;
            d_nmap[3 * (size_t)t + 1] = 0.f;
            d_nmap[3 * (size_t)t + 2] = 0.f;
        }
    }
    if (d_albedo) {
        d_albedo[3 * (size_t)t] = s[0];
        d_albedo[3 * (size_t)t + 1] = s[1];
        d_albedo[3 * (size_t)t + 2] = s[2];
    }
    if (d_rough) d_rough[t] = r.brdf ? s[3] : 0.f;
    if (d_spec) d_spec[t] = r.brdf ? s[4] : 0.f;
}

// one 256-thread workgroup: the PRF backward's partials (nb blocks) into acc[8..20), then
// the scalar gradients
__global__ void __launch_bounds__(256) k_adj_scalars(ReqDesc r, float* __restrict__ acc, float* d_scalars, int nb) {
    __shared__ double red[256];
    if (r.d_part)
        for (int k = 0; k < 12; ++k) sum_partial(r.d_part, nb, 12, k, acc + 8, red);
    if (threadIdx.x != 0 || !d_scalars) return;
    for (int k = 0; k < 12; ++k) d_scalars[k] = acc[8 + k];           // gamma_p, M
    for (int c = 0; c < 3; ++c) {
        d_scalars[12 + c] = acc[c];                                    // gamma_c
        d_scalars[15 + c] = acc[3 + c];                                // w through the CRF
    }
    if (r.clip) {   // threshold k / min(w): the lowest index wins a tie
        int a = 0;
        for (int c = 1; c < 3; ++c)
            if (scalar(r, 15 + c) < scalar(r, 15 + a)) a = c;
        const float wa = scalar(r, 15 + a);
        d_scalars[15 + a] += -acc[6] * r.clip_k / (wa * wa);
    }
}

// ---------------------------------------------------------------- launchers
static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline unsigned grid_cap(const Launch& l, int64_t n, int b) {
    const int64_t g = (n + b - 1) / b;
    return (unsigned)(g < 1 ? 1 : (g > l.grid_cap ? l.grid_cap : g));
}

void launch_adj_pixel(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, uint32_t p0,
                      uint32_t p1, const float* sample_L, float4* pix_dE) {
    if (p1 <= p0) return;
    const unsigned g = grid_of((int64_t)(p1 - p0) * PIX_LANES, BLOCK);
    hipLaunchKernelGGL(k_adj_pixel, dim3(g), dim3(BLOCK), 0, l.st, q, aq, r, p0, p1, sample_L, pix_dE);
    if (r.d_part) hipLaunchKernelGGL(k_sum_partials, dim3(7), dim3(256), 0, l.st, r.d_part, (int)g, 8, 7, r.d_acc);
}
size_t partial_floats(int64_t pixels_per_wave, int64_t proj_pixels) {
    return std::max<size_t>(8 * (size_t)grid_of(pixels_per_wave * PIX_LANES, BLOCK), 12 * (size_t)grid_of(proj_pixels, BLOCK));
}
void launch_adj_raygen(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, int slot, uint32_t g0,
                       uint32_t n) {
    if (n) hipLaunchKernelGGL(k_adj_raygen, dim3(grid_of(n, 256)), dim3(256), 0, l.st, q, aq, r, slot, g0, n);
}
void launch_adj_shade(const Launch& l, const Queues& q, const AdjQueues& aq, int cur, int depth, const ReqDesc& uni,
                      const ReqDesc* table, int64_t n_upper) {
    const dim3 g(grid_of(n_upper, BLOCK)), b(BLOCK);
    if (table) hipLaunchKernelGGL((k_adj_shade<false>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
    else hipLaunchKernelGGL((k_adj_shade<true>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
}
void launch_adj_shadow(const Launch& l, const Queues& q, const AdjQueues& aq, int which, int nxt, const ReqDesc& uni,
                       const ReqDesc* table, int64_t n_upper) {
    const dim3 g(grid_cap(Launch{l.st, q.trace_blocks}, n_upper, TB)), b(TB);
    if (q.stats) {
        if (table) hipLaunchKernelGGL((k_adj_shadow<false, true>), g, b, 0, l.st, q, aq, which, nxt, uni, table);
        else hipLaunchKernelGGL((k_adj_shadow<true, true>), g, b, 0, l.st, q, aq, which, nxt, uni, table);
    } else {
        if (table) hipLaunchKernelGGL((k_adj_shadow<false, false>), g, b, 0, l.st, q, aq, which, nxt, uni, table);
        else hipLaunchKernelGGL((k_adj_shadow<true, false>), g, b, 0, l.st, q, aq, which, nxt, uni, table);
    }
}
void launch_adj_replay(const Launch& l, const Queues& q, const AdjQueues& aq, int cur, int depth, const ReqDesc& uni,
                       const ReqDesc* table, int64_t n_upper) {
    const dim3 g(grid_of(n_upper, BLOCK)), b(BLOCK);
    if (!table && uni.tex4b) {
        hipLaunchKernelGGL(k_adj_replay_ext, g, b, 0, l.st, q, aq, cur, depth, uni);
        return;
    }
    if (table) hipLaunchKernelGGL((k_adj_replay<false>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
    else hipLaunchKernelGGL((k_adj_replay<true>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
}
bool map_tiling(int W, int H, int& T, int& nbx, int& nby) {
    for (int t = 8; t <= MAP_MAX_T; t *= 2) {
        T = t;
        nbx = (W + t - 1) / t;
        nby = (H + t - 1) / t;
        if ((int64_t)nbx * nby <= 1024) return true;
    }
    return (int64_t)nbx * nby <= MAP_MAX_BINS;
}
// map a alone (b null) or maps a and b together; hist, scan, place, accumulate, gather
template <int CA, int RSA, int CB, int RSB>
static void flush_maps(const Launch& l, const MapBins& a, float* oa, int sa, const MapBins* b, float* ob, int sb) {
    const MapBins& bb = b ? *b : a;
    const uint32_t ha = (uint32_t)((a.cap + BIN_CHUNK - 1) / BIN_CHUNK), hb = b ? (uint32_t)((b->cap + BIN_CHUNK - 1) / BIN_CHUNK) : 0u;
    const uint32_t aa = (uint32_t)((a.cap + ACC_CHUNK - 1) / ACC_CHUNK), ab = b ? (uint32_t)((b->cap + ACC_CHUNK - 1) / ACC_CHUNK) : 0u;
    const uint32_t ta = grid_of((int64_t)a.W * a.H, 256), tb = b ? grid_of((int64_t)b->W * b->H, 256) : 0u;
    hipLaunchKernelGGL((k_bin_hist<CA, RSA, CB, RSB>), dim3(ha + hb), dim3(BIN_TB), 0, l.st, a, bb, ha);
    hipLaunchKernelGGL(k_bin_scan, dim3(b ? 2 : 1), dim3(1024), 0, l.st, a, bb);
    hipLaunchKernelGGL((k_bin_place<RSA, RSB>), dim3(ha + hb), dim3(BIN_TB), 0, l.st, a, bb, ha);
    hipLaunchKernelGGL((k_bin_accum<CA, RSA, CB, RSB>), dim3(aa + ab), dim3(ACC_TB), 0, l.st, a, bb, aa);
    hipLaunchKernelGGL((k_bin_gather<CA, CB>), dim3(ta + tb), dim3(256), 0, l.st, a, oa, sa, bb, b ? ob : oa,
                       b ? sb : sa, ta);
}
void launch_sum_partials(const Launch& l, const float* part, int nb, int stride, int nv, float* dst) {
    hipLaunchKernelGGL(k_sum_partials, dim3(nv), dim3(256), 0, l.st, part, nb, stride, nv, dst);
}
void launch_map_flush(const Launch& l, const AdjQueues& aq, const ReqDesc& r) {
    const bool tex = aq.tb.rec && r.d_tex, ep = aq.eb.rec && r.dEp;
    const MapBins* e = ep ? &aq.eb : nullptr;
    if (tex && r.dtex_c == 9) flush_maps<9, TEX9_RS, 3, EP_RS>(l, aq.tb, r.d_tex, 9, e, r.dEp, 4);
    else if (tex) flush_maps<5, TEX_RS, 3, EP_RS>(l, aq.tb, r.d_tex, 5, e, r.dEp, 4);
    else if (ep) flush_maps<3, EP_RS, 3, EP_RS>(l, aq.eb, r.dEp, 4, nullptr, nullptr, 0);
}
void launch_adj_finish(const Launch& l, const ReqDesc& r, float* d_proj, float* d_albedo, float* d_rough,
                       float* d_spec, float* d_scalars, float* acc, float* d_metal, float* d_nmap) {
    const unsigned g = grid_of((int64_t)r.Wp * r.Hp, BLOCK);
    const bool maps = d_albedo || d_rough || d_spec || d_metal || d_nmap;
    const unsigned gm = maps ? grid_of((int64_t)r.tw * r.th, BLOCK) : 0u;
    hipLaunchKernelGGL(k_adj_prf, dim3(g + gm), dim3(BLOCK), 0, l.st, r, d_proj, acc, (int)g, d_albedo, d_rough,
                       d_spec, d_metal, d_nmap);
    hipLaunchKernelGGL(k_adj_scalars, dim3(1), dim3(256), 0, l.st, r, acc, d_scalars, (int)g);
}

}  // namespace dpcs
