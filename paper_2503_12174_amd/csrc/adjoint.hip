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

// ---------------------------------------------------------------- per pixel
// Eq. 5 backward: y = g_c w E_c, I_c = y^gamma_c;  Eq. 12 backward per sample
__global__ void k_adj_pixel(Queues q, AdjQueues aq, ReqDesc r, uint32_t p0, uint32_t p1, const float* sample_L) {
    const uint32_t p = p0 + blockIdx.x * blockDim.x + threadIdx.x;
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};   // d gamma_c[3], d w[3], d threshold
    if (p < p1) {
        const float thr = clip_threshold(r);
        float Ls[3] = {0.f, 0.f, 0.f};
        for (int s = 0; s < r.spp; ++s) {
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
                acc[c] += G * powf(y, gc) * logf(y);
                acc[3 + c] += dy * r.crf_gain * Ec;
            }
        }
        for (int s = 0; s < r.spp; ++s) {
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
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 7; ++k) {
        float v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        float v = 0.f;
        for (int k = 0; k < BLOCK / 64; ++k) v += red[threadIdx.x][k];
        if (v != 0.f) atomicAdd(&r.d_acc[threadIdx.x], v);
    }
}

// replay camera rays; the remaining radiance starts at the sample's total
__global__ void k_adj_raygen(Queues q, AdjQueues aq, ReqDesc r, int slot, uint32_t g0, uint32_t n) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t g = g0 + k;
    const uint32_t sid = g - r.g_base + r.sid_base;
    const D3 d = camera_dir(r, g);
    q.po[0][sid] = PathO{r.cam_o[0], r.cam_o[1], r.cam_o[2], slot, -1};
    q.pd[0][sid] = PathD{d.x, d.y, d.z, g, 0u};
    q.pb[0][sid] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    aq.rl[0][sid] = q.L[sid];
    aq.pend[0][sid] = make_float4(0.f, 0.f, 0.f, 0.f);
    aq.penda[0][sid] = make_float4(0.f, 0.f, 0.f, -1.f);   // w < 0: no pending bounce
    aq.pn[0][sid] = make_float4(0.f, 0.f, 0.f, 0.f);
    aq.pns[0][sid] = 0.f;
}

// ---------------------------------------------------------------- shading
template <bool UNI>
__global__ void __launch_bounds__(BLOCK) k_adj_shade(Queues q, AdjQueues aq, int cur, int depth, ReqDesc uni,
                                                     const ReqDesc* __restrict__ table) {
    const int nxt = cur ^ 1;
    const uint32_t n = q.cnt[cur];
    for (uint32_t base = blockIdx.x * BLOCK; base < n; base += gridDim.x * BLOCK) {
        const uint32_t i = base + threadIdx.x;
        bool cont = false, shp = false, she = false;
        PathO no{};
        PathD nd{};
        float4 nb = {}, nrl = {}, npend = {}, npenda = {};
        float4 po = {}, pd = {}, pc = {}, px = {}, pg = {}, pa = {};
        float4 eo = {}, ed = {}, ec = {}, ex = {}, ea = {};
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
            float4 rl = aq.rl[cur][i];
            const float4 pend = aq.pend[cur][i], penda = aq.penda[cur][i];
            if (leaf >= 0) {
                const Surf s = surface(r, leaf, d3(o.x, o.y, o.z), d3(dd.x, dd.y, dd.z));
                // the previous vertex's bounce: d/df of beta_k f cos/pdf R_{k+1} = L_r / f
                if (penda.w >= 0.f) {
                    const D3 t = delta * d3(rl.x, rl.y, rl.z) * d3(penda.x, penda.y, penda.z);
                    const double sum = t.x + t.y + t.z;
                    pend_on = true;
                    pend_u = pend.x;
                    pend_v = pend.y;
                    pend_g[0] = (float)(t.x * (1.0 / PI));
                    pend_g[1] = (float)(t.y * (1.0 / PI));
                    pend_g[2] = (float)(t.z * (1.0 / PI));
                    pend_g[3] = (float)(sum * pend.z);
                    pend_g[4] = (float)(sum * pend.w);
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
                    px = make_float4((float)p.pu, (float)p.pv, (float)s.u, (float)s.v);
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
                    ex = make_float4(0.f, 0.f, (float)s.u, (float)s.v);
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
                        npend = make_float4((float)s.u, (float)s.v, (float)f.ds_dr, (float)f.ds_dsp);
                        npenda = make_float4(f.f.x > 0.0 ? (float)(1.0 / f.f.x) : 0.f,
                                             f.f.y > 0.0 ? (float)(1.0 / f.f.y) : 0.f,
                                             f.f.z > 0.0 ? (float)(1.0 / f.f.z) : 0.f, 1.f);
                    }
                }
            }
        }
        if (UNI) scatter_tex(*rp, pend_on, pend_u, pend_v, pend_g);
        else if (pend_on) scatter_tex_lane(*rp, pend_u, pend_v, pend_g);
        const uint32_t jn = wave_append(cont, &q.cnt[nxt]);
        if (cont) {
            q.po[nxt][jn] = no;
            q.pd[nxt][jn] = nd;
            q.pb[nxt][jn] = nb;
            aq.rl[nxt][jn] = nrl;
            aq.pend[nxt][jn] = npend;
            aq.penda[nxt][jn] = npenda;
        }
        const int next_idx = cont ? (int)jn : -1;
        const uint32_t jp = wave_append(shp, &q.cnt[2]);
        if (shp) {
            pc.w = __int_as_float(next_idx);
            q.so[0][jp] = po;
            q.sd[0][jp] = pd;
            q.sc[0][jp] = pc;
            q.st[0][jp] = ptmax;
            aq.sx[0][jp] = px;
            aq.sg[0][jp] = pg;
            aq.sa[0][jp] = pa;
            aq.ss[0][jp] = ps;
        }
        const uint32_t je = wave_append(she, &q.cnt[3]);
        if (she) {
            ec.w = __int_as_float(next_idx);
            q.so[1][je] = eo;
            q.sd[1][je] = ed;
            q.sc[1][je] = ec;
            q.st[1][je] = __builtin_inff();
            aq.sx[1][je] = ex;
            aq.sg[1][je] = make_float4(0.f, 0.f, 0.f, 0.f);
            aq.sa[1][je] = ea;
            aq.ss[1][je] = es;
        }
    }
}

// ---------------------------------------------------------------- shadows
template <bool UNI>
__global__ void __launch_bounds__(TB) k_adj_shadow(Queues q, AdjQueues aq, int which, int nxt, ReqDesc uni,
                                                   const ReqDesc* __restrict__ table) {
    __shared__ int stack[SHORT_STACK * TB];
    int* spill = q.spill + (size_t)blockIdx.x * TB * SPILL + threadIdx.x;
    const uint32_t n = q.cnt[2 + which];
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
            Visits vis;
            occ = traverse<true, SHORT_STACK, TB>(r.nodes, r.tris, xyz(o), xyz(d), r.tmin, q.st[which][i],
                                                  __float_as_int(d.w), h, stack + threadIdx.x, spill, vis);
            if (q.stats) {
                atomicAdd(&q.stats[0], (unsigned long long)vis.nodes);
                atomicAdd(&q.stats[1], (unsigned long long)vis.tris);
            }
        }
        const float4 c = q.sc[which][ii], x = aq.sx[which][ii], a = aq.sa[which][ii];
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
                    scatter_ep_lane(r, x.x, x.y, ge);
                }
                scatter_tex_lane(r, x.z, x.w, gt);
            }
            continue;
        }
        // one request: lanes of one wave sum shared texels before the atomics
        if (which == 0 && r.dEp) {   // d/dE_p at the four projector texels
            const float4 gE = aq.sg[which][ii];
            const float ge[3] = {gE.x, gE.y, gE.z};
            scatter_ep(r, !occ, x.x, x.y, ge);
        }
        scatter_tex(r, !occ, x.z, x.w, gt);
    }
}

// ---------------------------------------------------------------- replay from records
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
    const uint32_t n = q.cnt[cur];
    for (uint32_t base = blockIdx.x * BLOCK; base < n; base += gridDim.x * BLOCK) {
        const uint32_t i = base + threadIdx.x;
        bool cont = false;
        PathO no{};
        PathD nd{};
        float4 nb = {}, nrl = {}, npend = {}, npenda = {}, npn = {};
        float npns = 0.f;
        // map cotangents of the previous vertex (a) and of this one when the path ends here (b)
        bool a_on = false, b_on = false, e_on = false;
        float a_u = 0.f, a_v = 0.f, b_u = 0.f, b_v = 0.f;
        float ag[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, bg[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        // E_p cotangent of this vertex's projector term
        double e_pu = 0.0, e_pv = 0.0;
        float eg[3] = {0.f, 0.f, 0.f};
        const ReqDesc* rp = &sel<UNI>(uni, table, 0);
        if (i < n) {
            const PathO o = q.po[cur][i];
            const PathD dd = q.pd[cur][i];
            const float4 b = q.pb[cur][i];
            const ReqDesc& r = sel<UNI>(uni, table, o.slot);
            rp = &r;
            const uint32_t g = dd.g;
            const uint32_t sid = g - r.g_base + r.sid_base;
            const uint32_t rec = r.rec[(size_t)(g - r.rec_g0) * r.max_depth + depth];
            const int leaf = (int)(rec & REC_LEAF) - 1;
            const float4 dl = aq.delta[sid];
            const D3 delta = d3(dl.x, dl.y, dl.z);
            const D3 beta = d3(b.x, b.y, b.z);
            float4 rl = aq.rl[cur][i];
            const float4 penda = aq.penda[cur][i];
            if (penda.w >= 0.f) {
                // previous vertex: its next-event cotangents plus d/df of its bounce,
                // beta_k f cos/pdf R_{k+1} -> R_{k+1} / f (zero when this ray escaped)
                const float4 pend = aq.pend[cur][i], pn = aq.pn[cur][i];
                const float pns = aq.pns[cur][i];
                a_on = true;
                a_u = pend.x;
                a_v = pend.y;
                double ga0 = pn.x, ga1 = pn.y, ga2 = pn.z, gr = pn.w, gs = pns;
                if (leaf >= 0) {
                    const D3 t = delta * d3(rl.x, rl.y, rl.z) * d3(penda.x, penda.y, penda.z);
                    const double sum = t.x + t.y + t.z;
                    ga0 += t.x * (1.0 / PI);
                    ga1 += t.y * (1.0 / PI);
                    ga2 += t.z * (1.0 / PI);
                    gr += sum * pend.z;
                    gs += sum * pend.w;
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
                        npend = make_float4((float)s.u, (float)s.v, (float)f.ds_dr, (float)f.ds_dsp);
                        npenda = make_float4(f.f.x > 0.0 ? (float)(1.0 / f.f.x) : 0.f,
                                             f.f.y > 0.0 ? (float)(1.0 / f.f.y) : 0.f,
                                             f.f.z > 0.0 ? (float)(1.0 / f.f.z) : 0.f, 1.f);
                        npn = make_float4((float)nga.x, (float)nga.y, (float)nga.z, (float)ngr);
                        npns = (float)ngs;
                    }
                }
                if (!cont) {   // the path ends here: its next-event cotangents go out now
                    b_on = true;
                    b_u = (float)s.u;
                    b_v = (float)s.v;
                    bg[0] = (float)nga.x;
                    bg[1] = (float)nga.y;
                    bg[2] = (float)nga.z;
                    bg[3] = (float)ngr;
                    bg[4] = (float)ngs;
                }
            }
        }
        if (UNI) {
            scatter_tex(*rp, a_on, a_u, a_v, ag);
            scatter_tex(*rp, b_on, b_u, b_v, bg);
            if (rp->dEp) scatter_ep(*rp, e_on, e_pu, e_pv, eg);
        } else {
            if (a_on) scatter_tex_lane(*rp, a_u, a_v, ag);
            if (b_on) scatter_tex_lane(*rp, b_u, b_v, bg);
            if (e_on) scatter_ep_lane(*rp, e_pu, e_pv, eg);
        }
        const bool pred[1] = {cont};
        uint32_t* const ctr[1] = {&q.cnt[nxt]};
        uint32_t jn;
        block_append<1>(pred, ctr, &jn);
        if (cont) {
            q.po[nxt][jn] = no;
            q.pd[nxt][jn] = nd;
            q.pb[nxt][jn] = nb;
            aq.rl[nxt][jn] = nrl;
            aq.pend[nxt][jn] = npend;
            aq.penda[nxt][jn] = npenda;
            aq.pn[nxt][jn] = npn;
            aq.pns[nxt][jn] = npns;
        }
    }
}

// ---------------------------------------------------------------- finish
// Eq. 1 backward per texel: z = g_p M y, y = I_p^gamma_p, E_p = max(0, z)
__global__ void k_adj_prf(ReqDesc r, float* __restrict__ d_proj, float* __restrict__ acc) {
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
        if (v != 0.f) atomicAdd(&acc[8 + threadIdx.x], v);
    }
}

// scalar gradients and the de-interleaving of the map cotangents
__global__ void k_adj_maps(ReqDesc r, float* d_albedo, float* d_rough, float* d_spec) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r.tw * r.th) return;
    const float* s = r.d_tex + 5 * (size_t)t;
    if (d_albedo) {
        d_albedo[3 * (size_t)t] = s[0];
        d_albedo[3 * (size_t)t + 1] = s[1];
        d_albedo[3 * (size_t)t + 2] = s[2];
    }
    if (d_rough) d_rough[t] = r.brdf ? s[3] : 0.f;
    if (d_spec) d_spec[t] = r.brdf ? s[4] : 0.f;
}

__global__ void k_adj_scalars(ReqDesc r, const float* __restrict__ acc, float* d_scalars) {
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
                      uint32_t p1, const float* sample_L) {
    if (p1 > p0)
        hipLaunchKernelGGL(k_adj_pixel, dim3(grid_of(p1 - p0, BLOCK)), dim3(BLOCK), 0, l.st, q, aq, r, p0, p1,
                           sample_L);
}
void launch_adj_raygen(const Launch& l, const Queues& q, const AdjQueues& aq, const ReqDesc& r, int slot, uint32_t g0,
                       uint32_t n) {
    if (n) hipLaunchKernelGGL(k_adj_raygen, dim3(grid_of(n, 256)), dim3(256), 0, l.st, q, aq, r, slot, g0, n);
}
void launch_adj_shade(const Launch& l, const Queues& q, const AdjQueues& aq, int cur, int depth, const ReqDesc& uni,
                      const ReqDesc* table, int64_t n_upper) {
    const dim3 g(grid_cap(l, n_upper, BLOCK)), b(BLOCK);
    if (table) hipLaunchKernelGGL((k_adj_shade<false>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
    else hipLaunchKernelGGL((k_adj_shade<true>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
}
void launch_adj_shadow(const Launch& l, const Queues& q, const AdjQueues& aq, int which, int nxt, const ReqDesc& uni,
                       const ReqDesc* table, int64_t n_upper, int) {
    const dim3 g(grid_cap(l, n_upper, TB)), b(TB);
    if (table) hipLaunchKernelGGL((k_adj_shadow<false>), g, b, 0, l.st, q, aq, which, nxt, uni, table);
    else hipLaunchKernelGGL((k_adj_shadow<true>), g, b, 0, l.st, q, aq, which, nxt, uni, table);
}
void launch_adj_replay(const Launch& l, const Queues& q, const AdjQueues& aq, int cur, int depth, const ReqDesc& uni,
                       const ReqDesc* table, int64_t n_upper) {
    const dim3 g(grid_cap(l, n_upper, BLOCK)), b(BLOCK);
    if (table) hipLaunchKernelGGL((k_adj_replay<false>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
    else hipLaunchKernelGGL((k_adj_replay<true>), g, b, 0, l.st, q, aq, cur, depth, uni, table);
}
void launch_adj_finish(const Launch& l, const ReqDesc& r, float* d_proj, float* d_albedo, float* d_rough,
                       float* d_spec, float* d_scalars, float* acc) {
    hipLaunchKernelGGL(k_adj_prf, dim3(grid_of((int64_t)r.Wp * r.Hp, BLOCK)), dim3(BLOCK), 0, l.st, r, d_proj, acc);
    if (d_albedo || d_rough || d_spec)
        hipLaunchKernelGGL(k_adj_maps, dim3(grid_of((int64_t)r.tw * r.th, 256)), dim3(256), 0, l.st, r, d_albedo,
                           d_rough, d_spec);
    hipLaunchKernelGGL(k_adj_scalars, dim3(1), dim3(64), 0, l.st, r, (const float*)acc, d_scalars);
}

}  // namespace dpcs
