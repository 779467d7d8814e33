// render.hip -- forward wavefront path tracer of the project-and-capture process.
//
// One launch wave traces a batch of camera samples through structure-of-arrays
// queues in HBM:
//   raygen   camera ray of every sample (Philox jitter, Eq. 6 inverted)
//   trace    closest hit of every queued path (BVH)
//   shade    hit point, BRDF maps, projector next-event estimation (Eq. 1-3, 6),
//            environment next-event estimation, bounce sampling (Eq. 10); emits
//            shadow rays and the surviving paths, compacted with wave64 ballots
//   shadow   any-hit visibility of each shadow ray; visible contributions are added
//            to the sample's radiance slot (one writer per slot per launch)
//   finalize clip per sample (Eq. 12), ordered mean over the pixel's samples (Eq. 4),
//            camera response and white balance (Eq. 5)
#include "kernels.hpp"
#include "shade.hpp"

namespace dpcs {

constexpr int TB = TRACE_TB;

// ---------------------------------------------------------------- per texel
// Eq. 1 with colour mixing: E_p = max(0, g_p M max(I_p, 0)^gamma_p)
__global__ void k_prf(ReqDesc r, float4* __restrict__ Ep) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r.Wp * r.Hp) return;
    float y[3];
    for (int c = 0; c < 3; ++c) {
        const float x = r.proj_image[3 * t + c];
        y[c] = x > 0.0f ? powf(x, scalar(r, c)) : 0.0f;
    }
    float e[3];
    for (int c = 0; c < 3; ++c) {
        const float z = r.prf_gain * (scalar(r, 3 + 3 * c) * y[0] + scalar(r, 4 + 3 * c) * y[1] +
                                      scalar(r, 5 + 3 * c) * y[2]);
        e[c] = fmaxf(z, 0.0f);
    }
    Ep[t] = make_float4(e[0], e[1], e[2], 0.0f);
}

__global__ void k_pack_tex(int n, const float* __restrict__ albedo, const float* __restrict__ rough,
                           float4* __restrict__ tex4) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    tex4[t] = make_float4(albedo[3 * t], albedo[3 * t + 1], albedo[3 * t + 2], rough ? rough[t] : 0.0f);
}

// (normal map rgb, metallic) per texel; absent maps stand for no change / metallic 0
__global__ void k_pack_tex_b(int n, const float* __restrict__ nmap, const float* __restrict__ metal,
                             float4* __restrict__ tex4b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    tex4b[t] = make_float4(nmap ? nmap[3 * t] : 0.5f, nmap ? nmap[3 * t + 1] : 0.5f, nmap ? nmap[3 * t + 2] : 1.0f,
                           metal ? metal[t] : 0.0f);
}

__global__ void k_set_count(uint32_t* cnt, int idx, uint32_t value, int zero_from, int zero_to) {
    if (threadIdx.x == 0) {
        if (idx >= 0) cnt[idx] = value;
        for (int k = zero_from; k < zero_to; ++k) cnt[k] = 0u;
    }
}

__global__ void k_zero(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// several buffers cleared by one launch: blockIdx.y picks the buffer
__global__ void k_zero_list(ZeroArgs z) {
    float* const p = z.p[blockIdx.y];
    const int64_t n = z.n[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_set_desc(ReqDesc r, ReqDesc* table, int slot) {
    if (threadIdx.x == 0) table[slot] = r;
}

// ---------------------------------------------------------------- raygen
__global__ void k_raygen(Queues q, ReqDesc r, int slot, uint32_t g0, uint32_t n) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t g = g0 + k;
    const uint32_t sid = g - r.g_base + r.sid_base;
    const D3 d = camera_dir(r, g);
    q.po[0][sid] = PathO{r.cam_o[0], r.cam_o[1], r.cam_o[2], slot, -1};
    q.pd[0][sid] = PathD{d.x, d.y, d.z, g, 0u};
    q.pb[0][sid] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    q.L[sid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (r.out_hits)
        for (int dd = 0; dd < r.max_depth; ++dd) r.out_hits[(size_t)g * r.max_depth + dd] = -2;
}

// ---------------------------------------------------------------- closest hit
// PROF: the counting pass's instantiation (node and triangle visit counters, summed
// into q.stats), which a profiler reports apart from the timed launches.
// CAM: the queue is one request's camera rays, entry i being sample g_base + i: each is
// generated here (Eq. 6 inverted) instead of being read back from the path queue.
template <bool UNI, bool PROF, bool CAM = false>
__global__ void __launch_bounds__(TB) TRAVERSAL_OCCUPANCY k_trace(Queues q, int cur, ReqDesc uni, const ReqDesc* __restrict__ table) {
    __shared__ int stack[(SHORT_STACK + 1) * TB];
    __shared__ float4 ltop[UNI ? 8 * TOP_NODES : 1];
    int* spill = q.spill + (size_t)blockIdx.x * TB * SPILL;
    const uint32_t n = q.cnt[cur];
    // the queues the shading after this launch appends to start empty (this kernel reads
    // only its own queue's count, and whatever read the others ran before it)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        q.cnt[cur ^ 1] = 0u;
        q.cnt[shadow_slot(cur, 0)] = 0u;
        q.cnt[shadow_slot(cur, 1)] = 0u;
    }
    TopNodes top{nullptr, 0u};
    if constexpr (UNI)   // one tree for the whole launch: stage its top levels
        if (uni.nodes4) top = stage_top<TB>(ltop, uni.nodes4, uni.top_nodes);
    for (uint32_t i = blockIdx.x * TB + threadIdx.x; i < n; i += gridDim.x * TB) {
        PathO o;
        PathD d;
        if constexpr (CAM) {
            const uint32_t g = uni.g_base + i;
            const D3 cd = camera_dir(uni, g);
            o = PathO{uni.cam_o[0], uni.cam_o[1], uni.cam_o[2], 0, -1};
            d = PathD{cd.x, cd.y, cd.z, g, 0u};
        } else {
            o = nt_ld(&q.po[cur][i]);
            d = nt_ld(&q.pd[cur][i]);
        }
        const ReqDesc& r = sel<UNI>(uni, table, o.slot);
        Hit h;
        Visits<PROF> vis;
        trace_ray<false, SHORT_STACK, TB>(r.nodes4, r.nodes, r.tris, v3((float)o.x, (float)o.y, (float)o.z),
                                         v3((float)d.x, (float)d.y, (float)d.z), r.tmin, __builtin_inff(), o.skip,
                                         h, stack, spill, threadIdx.x, vis, top);
        __builtin_nontemporal_store(h.leaf, &q.hit[i]);
        if constexpr (PROF)
            if (q.stats) {
                atomicAdd(&q.stats[0], (unsigned long long)vis.nodes);
                atomicAdd(&q.stats[1], (unsigned long long)vis.tris);
            }
    }
}

// ---------------------------------------------------------------- shading
// EXT: the request has the metallic and normal maps (tex4b): BRDF, cosines and sampling
// about the shading normal (one request per launch).  CAM: depth 0 of one request, its
// camera rays generated here as in k_trace (throughput 1, the sample's radiance started
// at zero here)
template <bool UNI, bool EXT, bool CAM = false>
__global__ void __launch_bounds__(BLOCK) k_shade(Queues q, int cur, int depth, ReqDesc uni,
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
        float4 nb = {}, po = {}, pd = {}, pc = {}, eo = {}, ed = {}, ec = {};
        float ptmax = 0.0f;
        if (i < n) {
            PathO o;
            PathD dd;
            float4 b;
            if constexpr (CAM) {
                const uint32_t gc = uni.g_base + i;
                const D3 cd = camera_dir(uni, gc);
                o = PathO{uni.cam_o[0], uni.cam_o[1], uni.cam_o[2], 0, -1};
                dd = PathD{cd.x, cd.y, cd.z, gc, 0u};
                b = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
            } else {
                o = nt_ld(&q.po[cur][i]);
                dd = nt_ld(&q.pd[cur][i]);
                b = nt_ld(&q.pb[cur][i]);
            }
            const int leaf = __builtin_nontemporal_load(&q.hit[i]);
            const ReqDesc& r = sel<UNI>(uni, table, o.slot);
            const uint32_t g = dd.g;
            const uint32_t sid = g - r.g_base + r.sid_base;
            const D3 beta = d3(b.x, b.y, b.z);
            if constexpr (CAM) {
                q.L[sid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (r.out_hits)
                    for (int k = 1; k < r.max_depth; ++k) r.out_hits[(size_t)g * r.max_depth + k] = -2;
            }
            if (r.rec) __builtin_nontemporal_store((uint32_t)(leaf + 1), &r.rec[(size_t)(g - r.rec_g0) * r.max_depth + depth]);
            if (leaf < 0) {
                if (r.out_hits) r.out_hits[(size_t)g * r.max_depth + depth] = -1;
                if (depth == 0 && r.env_on) {   // a camera ray that escapes sees the environment
                    float4 L = q.L[sid];
                    L.x += (float)(beta.x * r.env[0]);
                    L.y += (float)(beta.y * r.env[1]);
                    L.z += (float)(beta.z * r.env[2]);
                    q.L[sid] = L;
                }
            } else {
                // the projector lookup needs only the point and normal: its texels load
                // together with the maps' instead of after them
                Surf s = surface_geo(r, leaf, d3(o.x, o.y, o.z), d3(dd.x, dd.y, dd.z));
                ProjNee p;
                const bool prj = projector_nee(r, s, p);
                D4 E{};
                if (prj) E = fetch4(r.Ep, p.pb);
                surface_maps(r, s);
                if (r.out_hits) r.out_hits[(size_t)g * r.max_depth + depth] = s.prim;
                if (r.emission) {   // test scenes: surface emission
                    const float4 e = r.emission[leaf];
                    float4 L = q.L[sid];
                    L.x += (float)(beta.x * e.x);
                    L.y += (float)(beta.y * e.y);
                    L.z += (float)(beta.z * e.z);
                    q.L[sid] = L;
                }
                Shading sh{};
                if constexpr (EXT) sh = shading(r, leaf, s);
                const D3 ns = EXT ? sh.ns : s.n;
                if (prj) {
                    D3 C;
                    if constexpr (EXT) {
                        const BrdfX f = brdf_x<false>(r.brdf, s.n, ns, s.wo, p.wp, s.alb, s.rough, s.spec, sh.metal);
                        C = beta * f.f * d3(E.x, E.y, E.z) * (f.c * p.g0);
                    } else {
                        const Brdf f = brdf_eval<false>(r.brdf, s.n, s.wo, p.wp, s.alb, s.rough, s.spec);
                        C = beta * f.f * d3(E.x, E.y, E.z) * p.geom;
                    }
                    if (r.rec || C.x > 0.0 || C.y > 0.0 || C.z > 0.0) {
                        shp = true;
                        po = f4(to_f(s.x), __int_as_float(o.slot));
                        pd = f4(to_f(p.wp), __int_as_float(s.prim));
                        pc = f4(to_f(C), __uint_as_float(sid));
                        ptmax = (float)(p.dist - r.tmin);
                    }
                }
                if (r.env_on) {
                    const U4 x = vertex_rng(r, g, 2u + 2u * depth);
                    const D3 we = sample_cosine(ns, u24(x.x), u24(x.y));
                    D3 fv;
                    if constexpr (EXT) fv = brdf_x<false>(r.brdf, s.n, ns, s.wo, we, s.alb, s.rough, s.spec, sh.metal).f;
                    else fv = brdf_eval<false>(r.brdf, s.n, s.wo, we, s.alb, s.rough, s.spec).f;
                    const D3 C = beta * fv * d3(r.env[0], r.env[1], r.env[2]) * PI;
                    if (r.rec || C.x > 0.0 || C.y > 0.0 || C.z > 0.0) {
                        she = true;
                        eo = f4(to_f(s.x), __int_as_float(o.slot));
                        ed = f4(to_f(we), __int_as_float(s.prim));
                        ec = f4(to_f(C), __uint_as_float(sid));
                    }
                }
                if (depth < r.max_depth - 1) {
                    const U4 x = vertex_rng(r, g, 1u + 2u * depth);
                    const D3 wi = sample_bounce(r.brdf, ns, s.wo, s.rough, u24(x.x), u24(x.y), u24(x.z));
                    const double ci = dot(s.n, wi);   // the path goes on above the geometric surface
                    const double pdf = bounce_pdf(r.brdf, ns, s.wo, wi, s.rough);
                    if (ci > 0.0 && pdf > 0.0) {
                        D3 nbeta;
                        if constexpr (EXT) {
                            const BrdfX f = brdf_x<false>(r.brdf, s.n, ns, s.wo, wi, s.alb, s.rough, s.spec, sh.metal);
                            nbeta = beta * (f.f * (f.c / pdf));
                        } else {
                            const Brdf f = brdf_eval<false>(r.brdf, s.n, s.wo, wi, s.alb, s.rough, s.spec);
                            nbeta = beta * (f.f * (ci / pdf));
                        }
                        cont = true;
                        no = PathO{s.x.x, s.x.y, s.x.z, o.slot, s.prim};
                        nd = PathD{wi.x, wi.y, wi.z, g, 0u};
                        nb = make_float4((float)nbeta.x, (float)nbeta.y, (float)nbeta.z, 0.0f);
                    }
                }
            }
        }
        const bool pred[3] = {cont, shp, she};
        const int key[3] = {octant(nd.x, nd.y, nd.z), 0, octant(ed.x, ed.y, ed.z)};
        uint32_t* const ctr[3] = {&q.cnt[nxt], &q.cnt[shadow_slot(cur, 0)], &q.cnt[shadow_slot(cur, 1)]};
        uint32_t at[3];
        block_append_keyed<3, 8>(pred, key, ctr, at);
        const uint32_t jn = at[0], jp = at[1], je = at[2];
        if (cont) {
            nt_st(&q.po[nxt][jn], no);
            nt_st(&q.pd[nxt][jn], nd);
            nt_st(&q.pb[nxt][jn], nb);
        }
        if (shp) {
            nt_st(&q.so[0][jp], po);
            nt_st(&q.sd[0][jp], pd);
            nt_st(&q.sc[0][jp], pc);
            __builtin_nontemporal_store(ptmax, &q.st[0][jp]);
        }
        if (she) {
            nt_st(&q.so[1][je], eo);
            nt_st(&q.sd[1][je], ed);
            nt_st(&q.sc[1][je], ec);
            __builtin_nontemporal_store(__builtin_inff(), &q.st[1][je]);
        }
    }
}

// ---------------------------------------------------------------- shadows
// PROF: the counting pass's instantiation (node and triangle visit counters, summed
// into q.stats), which a profiler reports apart from the timed launches
// TREE: every ray of the launch is on the tree of `uni` (several requests of one scene):
// the tree's top is staged and its pointers come from `uni`, the rest from the table
template <bool UNI, bool PROF, bool TREE = UNI>
__global__ void __launch_bounds__(TB) SHADOW_OCCUPANCY k_shadow(Queues q, int which, int depth, ReqDesc uni,
                                               const ReqDesc* __restrict__ table) {
    __shared__ int stack[(SHORT_STACK + 1) * TB];
    __shared__ float4 ltop[TREE ? 8 * TOP_NODES : 1];
    int* spill = q.spill + (size_t)blockIdx.x * TB * SPILL;
    const uint32_t n = q.cnt[shadow_slot(depth & 1, which)];
    TopNodes top{nullptr, 0u};
    if constexpr (TREE)
        if (uni.nodes4) top = stage_top<TB>(ltop, uni.nodes4, uni.top_nodes);
    for (uint32_t i = blockIdx.x * TB + threadIdx.x; i < n; i += gridDim.x * TB) {
        const float4 o = nt_ld(&q.so[which][i]), d = nt_ld(&q.sd[which][i]);
        const ReqDesc& r = sel<UNI>(uni, table, __float_as_int(o.w));
        const ReqDesc& tr = TREE ? uni : r;
        Hit h;
        Visits<PROF> vis;
        const bool occ = trace_ray<true, SHORT_STACK, TB>(tr.nodes4, tr.nodes, tr.tris, xyz(o), xyz(d), tr.tmin,
                                                         nt_ld(&q.st[which][i]), __float_as_int(d.w), h, stack,
                                                         spill, threadIdx.x, vis, top);
        if constexpr (PROF)
            if (q.stats) {
                atomicAdd(&q.stats[0], (unsigned long long)vis.nodes);
                atomicAdd(&q.stats[1], (unsigned long long)vis.tris);
            }
        if (!occ) {
            const float4 c = nt_ld(&q.sc[which][i]);
            const uint32_t sid = __float_as_uint(c.w);
            float4 L = q.L[sid];
            L.x += c.x;
            L.y += c.y;
            L.z += c.z;
            q.L[sid] = L;
            if (r.rec) {
                const uint32_t g = sid - r.sid_base + r.g_base;
                atomicOr(&r.rec[(size_t)(g - r.rec_g0) * r.max_depth + depth], which == 0 ? REC_PRJ : REC_ENV);
            }
        }
    }
}

// ---------------------------------------------------------------- finalize
__device__ __forceinline__ float crf(const ReqDesc& r, int c, float Ec) {
    const float y = r.crf_gain * scalar(r, 15 + c) * Ec;
    return y > 0.0f ? powf(y, scalar(r, 12 + c)) : 0.0f;
}

// PIX_LANES lanes per pixel stride over its samples (neighbouring lanes read neighbouring
// samples), then a reduction inside the lane group; the per-pixel math stays spread
// over 64 / PIX_LANES pixels per wave.
__global__ void __launch_bounds__(256) k_finalize(Queues q, ReqDesc r, uint32_t p0, uint32_t p1) {
    const uint32_t p = p0 + (blockIdx.x * 256u + threadIdx.x) / PIX_LANES;
    if (p >= p1) return;   // uniform per lane group
    const int lane = threadIdx.x & (PIX_LANES - 1);
    const float thr = clip_threshold(r);
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int s = lane; s < r.spp; s += PIX_LANES) {
        const uint32_t g = p * (uint32_t)r.spp + (uint32_t)s;
        const float4 L = q.L[g - r.g_base + r.sid_base];
        const float l[3] = {L.x, L.y, L.z};
        for (int c = 0; c < 3; ++c) {
            if (r.out_L) r.out_L[3 * (size_t)g + c] = l[c];
            acc[c] += r.clip ? fminf(l[c], thr) : l[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int off = PIX_LANES / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off);
    if (lane == 0)
        for (int c = 0; c < 3; ++c) {
            const float Ec = acc[c] / (float)r.spp;
            if (r.out_linear) r.out_linear[3 * (size_t)p + c] = Ec;
            if (r.out_image) r.out_image[3 * (size_t)p + c] = crf(r, c, Ec);
        }
}

// ---------------------------------------------------------------- guide features
// One camera ray through each pixel centre; closest hit through the renderer's BVH with
// a full LDS stack (no spill region), hit attributes in FP64 as the shading uses them.
// Per pixel two float4: (albedo rgb, n.x), (n.y, n.z, t, 1); zeros on a miss.
__global__ void __launch_bounds__(TB) k_gbuffer(ReqDesc r, float4* __restrict__ out) {
    __shared__ int stack[(MAX_STACK + 1) * TB];
    const int64_t npix = (int64_t)r.Wc * r.Hc;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < npix; i += (int64_t)gridDim.x * TB) {
        const int px = (int)(i % r.Wc), py = (int)(i / r.Wc);
        const D3 o = d3(r.cam_o[0], r.cam_o[1], r.cam_o[2]);
        const D3 d = normalize(mat3(r.cam_M, d3(px + 0.5, py + 0.5, 1.0)));
        Hit h;
        Visits<false> vis;
        trace_ray<false, MAX_STACK, TB>(r.nodes4, r.nodes, r.tris, v3((float)o.x, (float)o.y, (float)o.z),
                                        v3((float)d.x, (float)d.y, (float)d.z), r.tmin, __builtin_inff(), -1, h,
                                        stack, nullptr, threadIdx.x, vis);
        float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
        if (h.leaf >= 0) {
            const Surf s = surface(r, h.leaf, o, d);
            const double t = dot(s.x - o, d);
            a = make_float4((float)s.alb.x, (float)s.alb.y, (float)s.alb.z, (float)s.n.x);
            b = make_float4((float)s.n.y, (float)s.n.z, (float)t, 1.0f);
        }
        out[2 * i] = a;
        out[2 * i + 1] = b;
    }
}

// ---------------------------------------------------------------- debug
// BRDF value and derivatives, bounce density and a bounce sample, on rows of FP64 input
// (17 per row in, 11 per row out; the layout is the C ABI's)
__global__ void k_debug_brdf(int kind, const double* __restrict__ in, int64_t n, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* x = in + 17 * i;
    const D3 nn = d3(x[0], x[1], x[2]), wo = d3(x[3], x[4], x[5]), wi = d3(x[6], x[7], x[8]);
    const D3 alb = d3(x[9], x[10], x[11]);
    const double r = x[12], sp = x[13];
    const Brdf f = brdf_eval<true>(kind, nn, wo, wi, alb, r, sp);
    const Brdf f0 = brdf_eval<false>(kind, nn, wo, wi, alb, r, sp);
    const D3 ws = sample_bounce(kind, nn, wo, r, x[14], x[15], x[16]);
    double* y = out + 11 * i;
    y[0] = f.f.x;
    y[1] = f.f.y;
    y[2] = f.f.z;
    y[3] = f.ds_dr;
    y[4] = f.ds_dsp;
    y[5] = bounce_pdf(kind, nn, wo, wi, r);
    y[6] = ws.x;
    y[7] = ws.y;
    y[8] = ws.z;
    y[9] = bounce_pdf(kind, nn, wo, ws, r);
    y[10] = f0.f.x;
}

// full 64-entry LDS stack (no spill region needed: the host checks the stack bound).
// mode: 0 brute force, 1 the BVH the renderer uses (4-wide when built), 2 the binary
// BVH, 3 any hit on the renderer's BVH, 4 any hit by brute force
__global__ void __launch_bounds__(TB) k_debug_intersect(const float4* __restrict__ nodes4,
                                                        const float4* __restrict__ nodes,
                                                        const float4* __restrict__ tris,
                                                        const int* __restrict__ leaf_of_prim, int nt, float tmin,
                                                        const float* __restrict__ rays, int64_t n, int mode,
                                                        int32_t* prim, float* t, float* b1, float* b2) {
    __shared__ int stack[(MAX_STACK + 1) * TB];
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const float* ry = rays + 8 * i;
    const V3 o = v3(ry[0], ry[1], ry[2]), d = v3(ry[3], ry[4], ry[5]);
    Hit h;
    Visits<false> vis;
    int* st = stack;
    const int lane = threadIdx.x;
    if (mode == 1)
        trace_ray<false, MAX_STACK, TB>(nodes4, nodes, tris, o, d, tmin, ry[6], (int)ry[7], h, st, nullptr, lane, vis);
    else if (mode == 2)
        traverse<false, MAX_STACK, TB>(nodes, tris, o, d, tmin, ry[6], (int)ry[7], h, st, nullptr, lane, vis);
    else if (mode == 3)
        trace_ray<true, MAX_STACK, TB>(nodes4, nodes, tris, o, d, tmin, ry[6], (int)ry[7], h, st, nullptr, lane, vis);
    else if (mode == 4)
        brute_force<true>(tris, leaf_of_prim, nt, o, d, tmin, ry[6], (int)ry[7], h);
    else
        brute_force<false>(tris, leaf_of_prim, nt, o, d, tmin, ry[6], (int)ry[7], h);
    prim[i] = h.prim;
    if (t) t[i] = h.t;
    if (b1) b1[i] = h.b1;
    if (b2) b2[i] = h.b2;
}

__global__ void k_debug_philox(uint32_t klo, uint32_t khi, const uint32_t* __restrict__ ctr, int64_t n,
                               uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 x = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], klo, khi);
    out[4 * i] = x.x;
    out[4 * i + 1] = x.y;
    out[4 * i + 2] = x.z;
    out[4 * i + 3] = x.w;
}

// ---------------------------------------------------------------- launchers
static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline unsigned grid_cap(const Launch& l, int64_t n, int b) {
    const int64_t g = (n + b - 1) / b;
    return (unsigned)(g < 1 ? 1 : (g > l.grid_cap ? l.grid_cap : g));
}

void launch_prf(const Launch& l, const ReqDesc& r, float4* Ep) {
    hipLaunchKernelGGL(k_prf, dim3(grid_of((int64_t)r.Wp * r.Hp, 256)), dim3(256), 0, l.st, r, Ep);
}
void launch_pack_tex(const Launch& l, const ReqDesc& r, const float* albedo, const float* rough, float4* tex4) {
    const int n = r.tw * r.th;
    hipLaunchKernelGGL(k_pack_tex, dim3(grid_of(n, 256)), dim3(256), 0, l.st, n, albedo, rough, tex4);
}
void launch_pack_tex_b(const Launch& l, const ReqDesc& r, const float* nmap, const float* metal, float4* tex4b) {
    const int n = r.tw * r.th;
    hipLaunchKernelGGL(k_pack_tex_b, dim3(grid_of(n, 256)), dim3(256), 0, l.st, n, nmap, metal, tex4b);
}
void launch_set_count(const Launch& l, uint32_t* cnt, int idx, uint32_t value, int zero_from, int zero_to) {
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, l.st, cnt, idx, value, zero_from, zero_to);
}
void launch_zero(const Launch& l, float* p, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_zero, dim3(grid_of(n, 256)), dim3(256), 0, l.st, p, n);
}
void ZeroList::add(float* ptr, int64_t count) {
    if (!ptr || count <= 0) return;
    if (k == ZERO_LIST_MAX) launch();   // full: clear what is held and start again
    a.p[k] = ptr;
    a.n[k] = count;
    ++k;
}
void ZeroList::launch() {
    if (k == 0) return;
    int64_t m = 0;
    for (int j = 0; j < k; ++j) m = std::max(m, a.n[j]);
    const unsigned gx = (unsigned)std::min<int64_t>(grid_of(m, 256), 4096);
    hipLaunchKernelGGL(k_zero_list, dim3(gx, (unsigned)k), dim3(256), 0, l.st, a);
    k = 0;
}
void launch_set_desc(const Launch& l, ReqDesc* table, int slot, const ReqDesc& r) {
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, l.st, r, table, slot);
}
void launch_raygen(const Launch& l, const Queues& q, const ReqDesc& r, const ReqDesc*, int slot, uint32_t g0,
                   uint32_t n, bool, const AdjQueues*) {
    if (n) hipLaunchKernelGGL(k_raygen, dim3(grid_of(n, 256)), dim3(256), 0, l.st, q, r, slot, g0, n);
}
void launch_trace(const Launch& l, const Queues& q, int cur, const ReqDesc& uni, const ReqDesc* table,
                  int64_t n_upper, bool cam) {
    const dim3 g(grid_cap(Launch{l.st, q.trace_blocks}, n_upper, TB)), b(TB);
    if (cam && !table) {
        if (q.stats) hipLaunchKernelGGL((k_trace<true, true, true>), g, b, 0, l.st, q, cur, uni, table);
        else hipLaunchKernelGGL((k_trace<true, false, true>), g, b, 0, l.st, q, cur, uni, table);
        return;
    }
    if (q.stats) {
        if (table) hipLaunchKernelGGL((k_trace<false, true>), g, b, 0, l.st, q, cur, uni, table);
        else hipLaunchKernelGGL((k_trace<true, true>), g, b, 0, l.st, q, cur, uni, table);
    } else {
        if (table) hipLaunchKernelGGL((k_trace<false, false>), g, b, 0, l.st, q, cur, uni, table);
        else hipLaunchKernelGGL((k_trace<true, false>), g, b, 0, l.st, q, cur, uni, table);
    }
}
void launch_shade(const Launch& l, const Queues& q, int cur, int depth, const ReqDesc& uni, const ReqDesc* table,
                  int64_t n_upper, bool cam) {
    const dim3 g(grid_of(n_upper, BLOCK)), b(BLOCK);
    if (cam && !table) {
        if (uni.tex4b) hipLaunchKernelGGL((k_shade<true, true, true>), g, b, 0, l.st, q, cur, depth, uni, table);
        else hipLaunchKernelGGL((k_shade<true, false, true>), g, b, 0, l.st, q, cur, depth, uni, table);
        return;
    }
    if (table) hipLaunchKernelGGL((k_shade<false, false>), g, b, 0, l.st, q, cur, depth, uni, table);
    else if (uni.tex4b) hipLaunchKernelGGL((k_shade<true, true>), g, b, 0, l.st, q, cur, depth, uni, table);
    else hipLaunchKernelGGL((k_shade<true, false>), g, b, 0, l.st, q, cur, depth, uni, table);
}
void launch_shadow(const Launch& l, const Queues& q, int which, const ReqDesc& uni, const ReqDesc* table,
                   int64_t n_upper, int depth, bool one_tree) {
    const dim3 g(grid_cap(Launch{l.st, q.trace_blocks}, n_upper, TB)), b(TB);
    if (table && one_tree) {
        hipLaunchKernelGGL((k_shadow<false, false, true>), g, b, 0, l.st, q, which, depth, uni, table);
        return;
    }
    if (q.stats) {
        if (table) hipLaunchKernelGGL((k_shadow<false, true>), g, b, 0, l.st, q, which, depth, uni, table);
        else hipLaunchKernelGGL((k_shadow<true, true>), g, b, 0, l.st, q, which, depth, uni, table);
    } else {
        if (table) hipLaunchKernelGGL((k_shadow<false, false>), g, b, 0, l.st, q, which, depth, uni, table);
        else hipLaunchKernelGGL((k_shadow<true, false>), g, b, 0, l.st, q, which, depth, uni, table);
    }
}
void launch_finalize(const Launch& l, const Queues& q, const ReqDesc& r, const ReqDesc*, int, uint32_t p0,
                     uint32_t p1) {
    if (p1 > p0)
        hipLaunchKernelGGL(k_finalize, dim3(grid_of((int64_t)(p1 - p0) * PIX_LANES, 256)), dim3(256), 0, l.st, q, r, p0, p1);
}
void launch_debug_intersect(const Launch& l, const float4* nodes4, const float4* nodes, const float4* tris,
                            const int* leaf_of_prim, int nt, float tmin, const float* rays, int64_t n, int mode,
                            int32_t* prim, float* t, float* b1, float* b2) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_debug_intersect, dim3(grid_of(n, TB)), dim3(TB), 0, l.st, nodes4, nodes, tris, leaf_of_prim,
                       nt, tmin, rays, n, mode, prim, t, b1, b2);
}
void launch_gbuffer(const Launch& l, const ReqDesc& r, float* out) {
    const int64_t n = (int64_t)r.Wc * r.Hc;
    hipLaunchKernelGGL(k_gbuffer, dim3(grid_cap(l, n, TB)), dim3(TB), 0, l.st, r, reinterpret_cast<float4*>(out));
}
void launch_debug_brdf(const Launch& l, int kind, const double* in, int64_t n, double* out) {
    if (n > 0) hipLaunchKernelGGL(k_debug_brdf, dim3(grid_of(n, 256)), dim3(256), 0, l.st, kind, in, n, out);
}
void launch_debug_philox(const Launch& l, uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out) {
    if (n > 0)
        hipLaunchKernelGGL(k_debug_philox, dim3(grid_of(n, 256)), dim3(256), 0, l.st, (uint32_t)seed,
                           (uint32_t)(seed >> 32), ctr, n, out);
}

}  // namespace dpcs
