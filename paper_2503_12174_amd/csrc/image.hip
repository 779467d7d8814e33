// image.hip -- image-space operators of the training objective: the cross-bilateral
// denoiser D of Eq. 11 with its adjoint, and the L1 data term and map regulariser L(m)
// of Eq. 9 with their gradients.  Entry points of the C ABI.
#include "runtime.hpp"

#include <cmath>
#include <cstring>

using namespace dpcs;

namespace {

// ---------------------------------------------------------------- denoiser
// One workgroup filters a 16 x 16 tile of output pixels, one thread per pixel.  The
// tile plus an r-pixel halo of guide features (float4 planes) and of the filtered
// values (rgb in a float4) is staged in LDS once; every window tap then reads LDS only.
// Weights are exp2 of a base-2 exponent (the factors carry log2 e), one v_exp_f32 per
// tap; guide differences are formed before scaling, so large guide values with small
// differences (depths) keep their relative accuracy.
constexpr int DN_T = 16;
constexpr int DN_TB = DN_T * DN_T;
constexpr float LOG2E = 1.44269504088896340736f;

enum { DN_FWD = 0, DN_NORM = 1, DN_ADJ = 2 };

struct DenoiseArgs {
    const float* val;    // DN_FWD: image H x W x 3; DN_NORM: cotangent H x W x 3; DN_ADJ: u H x W x 4
    const float* guide;  // H x W x G
    float* out;          // DN_FWD: H x W x 3; DN_NORM: u = cotangent / W_p, H x W x 4; DN_ADJ: H x W x 3
    int W, H, G, r;
    float as;            // a_s log2 e
    float ag[DPCS_DENOISE_MAX_GUIDE];   // a_k log2 e; 0 past G
};

// MODE DN_FWD: out_p = sum_q w(p,q) I_q / W_p.  DN_NORM: u_p = G_p / W_p.  DN_ADJ:
// out_q = sum_p w(q,p) u_p (w is symmetric and so is the window relation, so the
// transposed operator is the same gather with unnormalised weights).
template <int NG4, int MODE>
__global__ void __launch_bounds__(DN_TB) k_bilateral(DenoiseArgs a) {
    extern __shared__ float4 lds[];
    const int P = DN_T + 2 * a.r, PP = P * P;
    float4* lg = lds;              // NG4 planes of PP guide quadruples
    float4* lv = lds + NG4 * PP;   // PP values (unused by DN_NORM)
    const int x0 = (int)blockIdx.x * DN_T - a.r, y0 = (int)blockIdx.y * DN_T - a.r;
    for (int k = threadIdx.x; k < PP; k += DN_TB) {
        const int gx = x0 + k % P, gy = y0 + k / P;
        const bool in = gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
        const size_t pix = in ? (size_t)gy * a.W + gx : 0;
#pragma unroll
        for (int j = 0; j < NG4; ++j) {
            float c[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ch = 4 * j + e;
                c[e] = (in && ch < a.G) ? a.guide[pix * a.G + ch] : 0.0f;
            }
            lg[j * PP + k] = make_float4(c[0], c[1], c[2], c[3]);
        }
        if constexpr (MODE == DN_FWD)
            lv[k] = in ? make_float4(a.val[3 * pix], a.val[3 * pix + 1], a.val[3 * pix + 2], 0.0f)
                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (MODE == DN_ADJ)
            lv[k] = in ? reinterpret_cast<const float4*>(a.val)[pix] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    const int tx = (int)threadIdx.x % DN_T, ty = (int)threadIdx.x / DN_T;
    const int px = (int)blockIdx.x * DN_T + tx, py = (int)blockIdx.y * DN_T + ty;
    if (px >= a.W || py >= a.H) return;   // no barrier follows
    const int c = (ty + a.r) * P + tx + a.r;
    float4 gp[NG4 > 0 ? NG4 : 1];
#pragma unroll
    for (int j = 0; j < NG4; ++j) gp[j] = lg[j * PP + c];
    // the window clipped to the image
    const int dy0 = max(-a.r, -py), dy1 = min(a.r, a.H - 1 - py);
    const int dx0 = max(-a.r, -px), dx1 = min(a.r, a.W - 1 - px);
    float wsum = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
    for (int dy = dy0; dy <= dy1; ++dy) {
        const int row = c + dy * P;
        for (int dx = dx0; dx <= dx1; ++dx) {
            const int q = row + dx;
            float e = a.as * (float)(dx * dx + dy * dy);
#pragma unroll
            for (int j = 0; j < NG4; ++j) {
                const float4 g = lg[j * PP + q];
                const float d0 = g.x - gp[j].x, d1 = g.y - gp[j].y, d2 = g.z - gp[j].z, d3 = g.w - gp[j].w;
                e = fmaf(a.ag[4 * j] * d0, d0, e);
                e = fmaf(a.ag[4 * j + 1] * d1, d1, e);
                e = fmaf(a.ag[4 * j + 2] * d2, d2, e);
                e = fmaf(a.ag[4 * j + 3] * d3, d3, e);
            }
            const float w = __builtin_amdgcn_exp2f(-e);
            if constexpr (MODE != DN_ADJ) wsum += w;
            if constexpr (MODE != DN_NORM) {
                const float4 v = lv[q];
                s0 = fmaf(w, v.x, s0);
                s1 = fmaf(w, v.y, s1);
                s2 = fmaf(w, v.z, s2);
            }
        }
    }
    const size_t pix = (size_t)py * a.W + px;
    if constexpr (MODE == DN_FWD) {
        a.out[3 * pix] = s0 / wsum;
        a.out[3 * pix + 1] = s1 / wsum;
        a.out[3 * pix + 2] = s2 / wsum;
    } else if constexpr (MODE == DN_NORM) {
        reinterpret_cast<float4*>(a.out)[pix] =
            make_float4(a.val[3 * pix] / wsum, a.val[3 * pix + 1] / wsum, a.val[3 * pix + 2] / wsum, 0.0f);
    } else {
        a.out[3 * pix] = s0;
        a.out[3 * pix + 1] = s1;
        a.out[3 * pix + 2] = s2;
    }
}

template <int MODE>
void launch_bilateral(hipStream_t st, const DenoiseArgs& a) {
    const int ng4 = (a.G + 3) / 4;
    const int P = DN_T + 2 * a.r;
    const size_t lds = sizeof(float4) * (size_t)P * P * (ng4 + (MODE == DN_NORM ? 0 : 1));
    const dim3 grid((a.W + DN_T - 1) / DN_T, (a.H + DN_T - 1) / DN_T);
    if (ng4 == 0)
        hipLaunchKernelGGL((k_bilateral<0, MODE>), grid, dim3(DN_TB), lds, st, a);
    else if (ng4 == 1)
        hipLaunchKernelGGL((k_bilateral<1, MODE>), grid, dim3(DN_TB), lds, st, a);
    else
        hipLaunchKernelGGL((k_bilateral<2, MODE>), grid, dim3(DN_TB), lds, st, a);
}

bool denoise_args(dpcs_context ctx, const dpcs_denoise_params* p, const float* val, const float* guide, float* out,
                  DenoiseArgs& a, dpcs_status* st) {
    const char* bad = nullptr;
    if (!p) bad = "params is NULL";
    else if (p->width < 1 || p->height < 1 || p->width > 16384 || p->height > 16384)
        bad = "width/height must be in 1..16384";
    else if (p->guide_channels < 0 || p->guide_channels > DPCS_DENOISE_MAX_GUIDE) bad = "guide_channels must be in 0..8";
    else if (p->radius < 0 || p->radius > DPCS_DENOISE_MAX_RADIUS) bad = "radius must be in 0..8";
    else if (!(p->spatial >= 0.0f) || !std::isfinite(p->spatial)) bad = "spatial must be finite and >= 0";
    else if (!val || !out) bad = "image and output must not be NULL";
    else if (p->guide_channels > 0 && !guide) bad = "guide is NULL with guide_channels > 0";
    else
        for (int k = 0; k < p->guide_channels; ++k)
            if (!(p->guide[k] >= 0.0f) || !std::isfinite(p->guide[k])) bad = "guide factors must be finite and >= 0";
    if (bad) {
        *st = fail(ctx, DPCS_E_INVALID, std::string("denoise: ") + bad);
        return false;
    }
    std::memset(&a, 0, sizeof a);
    a.val = val;
    a.guide = guide;
    a.out = out;
    a.W = p->width;
    a.H = p->height;
    a.G = p->guide_channels;
    a.r = p->radius;
    a.as = p->spatial * LOG2E;
    for (int k = 0; k < a.G; ++k) a.ag[k] = p->guide[k] * LOG2E;
    return true;
}

// ---------------------------------------------------------------- losses
// Sums over a map or an image: each workgroup of a capped grid folds a grid-stride
// share into two FP64 partial sums; one workgroup then adds the partials in a fixed
// order.  No atomics: the loss is the same on every run.
constexpr int RED_TB = 256;
constexpr int RED_MAX_BLOCKS = 1024;

__device__ __forceinline__ void block_sum2(double& a, double& b, double* part) {
    __shared__ double sa[RED_TB / 64], sb[RED_TB / 64];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sa[wv] = a;
        sb[wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int k = 0; k < RED_TB / 64; ++k) {
            x += sa[k];
            y += sb[k];
        }
        part[0] = x;
        part[1] = y;
    }
}

// sums of |vertical| and |horizontal| neighbour differences of an h x w x c map
__global__ void __launch_bounds__(RED_TB) k_tv_partial(const float* __restrict__ m, int h, int w, int c,
                                                       double* __restrict__ part) {
    const int64_t n = (int64_t)h * w * c, wc = (int64_t)w * c;
    double sv = 0.0, sh = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_TB) {
        const int64_t y = i / wc, x = (i - y * wc) / c;
        const double v = m[i];
        if (y + 1 < h) sv += fabs((double)m[i + wc] - v);
        if (x + 1 < w) sh += fabs((double)m[i + c] - v);
    }
    block_sum2(sv, sh, part + 2 * blockIdx.x);
}

__global__ void __launch_bounds__(RED_TB) k_l1_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                       int64_t n, double* __restrict__ part) {
    double s = 0.0, z = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_TB)
        s += fabs((double)a[i] - (double)b[i]);
    block_sum2(s, z, part + 2 * blockIdx.x);
}

// loss = s0 / n0 + s1 / n1 (a term with n = 0 adds 0)
__global__ void __launch_bounds__(RED_TB) k_loss_final(const double* __restrict__ part, int nb, double n0, double n1,
                                                       float* __restrict__ loss) {
    __shared__ double tot[2];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += RED_TB) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    block_sum2(a, b, tot);
    if (threadIdx.x == 0) {
        const double l = (n0 > 0.0 ? tot[0] / n0 : 0.0) + (n1 > 0.0 ? tot[1] / n1 : 0.0);
        loss[0] = (float)l;
    }
}

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// dL/dm: every value gains +sign/n from the pair it ends and -sign/n from the pair it starts
__global__ void __launch_bounds__(RED_TB) k_tv_grad(const float* __restrict__ m, int h, int w, int c,
                                                    const float* __restrict__ gl, double nv, double nh,
                                                    float* __restrict__ g) {
    const int64_t n = (int64_t)h * w * c, wc = (int64_t)w * c;
    const double s = gl[0];
    for (int64_t i = (int64_t)blockIdx.x * RED_TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_TB) {
        const int64_t y = i / wc, x = (i - y * wc) / c;
        const double v = m[i];
        double hs = 0.0, vs = 0.0;
        if (x > 0) hs += sgn(v - (double)m[i - c]);
        if (x + 1 < w) hs -= sgn((double)m[i + c] - v);
        if (y > 0) vs += sgn(v - (double)m[i - wc]);
        if (y + 1 < h) vs -= sgn((double)m[i + wc] - v);
        g[i] = (float)(s * ((nh > 0.0 ? hs / nh : 0.0) + (nv > 0.0 ? vs / nv : 0.0)));
    }
}

__global__ void __launch_bounds__(RED_TB) k_l1_grad(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                                    const float* __restrict__ gl, float* __restrict__ g) {
    const double s = gl[0];
    for (int64_t i = (int64_t)blockIdx.x * RED_TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_TB)
        g[i] = (float)(s * sgn((double)a[i] - (double)b[i]) / (double)n);
}

unsigned red_grid(int64_t n) {
    const int64_t g = (n + RED_TB - 1) / RED_TB;
    return (unsigned)(g < 1 ? 1 : (g > RED_MAX_BLOCKS ? RED_MAX_BLOCKS : g));
}

dpcs_status begin(dpcs_context ctx) {
    if (ctx->sticky) return DPCS_E_DEVICE;
    if (!hip_ok(ctx, hipSetDevice(ctx->device), "hipSetDevice")) return DPCS_E_DEVICE;
    (void)hipGetLastError();
    return DPCS_OK;
}

dpcs_status end(dpcs_context ctx, const char* what) {
    if (!hip_ok(ctx, hipGetLastError(), what)) return DPCS_E_DEVICE;
    ctx->err.clear();
    return DPCS_OK;
}

bool map_ok(dpcs_context ctx, const float* m, int32_t h, int32_t w, int32_t c, dpcs_status* st) {
    if (!m || h < 1 || w < 1 || c < 1 || (int64_t)h * w * c >= (int64_t(1) << 31)) {
        *st = fail(ctx, DPCS_E_INVALID, "map must be non-NULL with h, w, c >= 1 and h w c < 2^31");
        return false;
    }
    return true;
}

}  // namespace

// ====================================================================== C ABI
extern "C" dpcs_status dpcs_denoise(dpcs_context ctx, const dpcs_denoise_params* p, const float* image,
                                    const float* guide, float* out) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    dpcs_status st = begin(ctx);
    if (st != DPCS_OK) return st;
    DenoiseArgs a;
    if (!denoise_args(ctx, p, image, guide, out, a, &st)) return st;
    if (image == out) return fail(ctx, DPCS_E_INVALID, "denoise: out must not be the input image");
    launch_bilateral<DN_FWD>(ctx->stream, a);
    return end(ctx, "denoise");
}

extern "C" dpcs_status dpcs_denoise_vjp(dpcs_context ctx, const dpcs_denoise_params* p, const float* grad_out,
                                        const float* guide, float* grad_image) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    dpcs_status st = begin(ctx);
    if (st != DPCS_OK) return st;
    DenoiseArgs a;
    if (!denoise_args(ctx, p, grad_out, guide, grad_image, a, &st)) return st;
    if (grad_out == grad_image) return fail(ctx, DPCS_E_INVALID, "denoise_vjp: grad_image must not be grad_out");
    float* u = (float*)scratch(ctx, "denoise.u", sizeof(float4) * (size_t)a.W * a.H, &st);
    if (!u) return st;
    DenoiseArgs a1 = a;   // u_p = G_p / W_p
    a1.out = u;
    launch_bilateral<DN_NORM>(ctx->stream, a1);
    DenoiseArgs a2 = a;   // grad_q = sum_p w(q,p) u_p
    a2.val = u;
    launch_bilateral<DN_ADJ>(ctx->stream, a2);
    return end(ctx, "denoise_vjp");
}

extern "C" dpcs_status dpcs_tv_loss(dpcs_context ctx, const float* map, int32_t h, int32_t w, int32_t c,
                                    float* loss) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    dpcs_status st = begin(ctx);
    if (st != DPCS_OK) return st;
    if (!map_ok(ctx, map, h, w, c, &st)) return st;
    if (!loss) return fail(ctx, DPCS_E_INVALID, "tv_loss: loss is NULL");
    double* part = (double*)scratch(ctx, "loss.part", sizeof(double) * 2 * RED_MAX_BLOCKS, &st);
    if (!part) return st;
    const int64_t n = (int64_t)h * w * c;
    const unsigned nb = red_grid(n);
    hipLaunchKernelGGL(k_tv_partial, dim3(nb), dim3(RED_TB), 0, ctx->stream, map, h, w, c, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(RED_TB), 0, ctx->stream, part, (int)nb,
                       (double)c * (h - 1) * w, (double)c * h * (w - 1), loss);
    return end(ctx, "tv_loss");
}

extern "C" dpcs_status dpcs_tv_vjp(dpcs_context ctx, const float* map, int32_t h, int32_t w, int32_t c,
                                   const float* grad_loss, float* grad_map) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    dpcs_status st = begin(ctx);
    if (st != DPCS_OK) return st;
    if (!map_ok(ctx, map, h, w, c, &st)) return st;
    if (!grad_loss || !grad_map) return fail(ctx, DPCS_E_INVALID, "tv_vjp: grad_loss and grad_map must not be NULL");
    if (grad_map == map) return fail(ctx, DPCS_E_INVALID, "tv_vjp: grad_map must not be the map");
    const int64_t n = (int64_t)h * w * c;
    hipLaunchKernelGGL(k_tv_grad, dim3(red_grid(n)), dim3(RED_TB), 0, ctx->stream, map, h, w, c, grad_loss,
                       (double)c * (h - 1) * w, (double)c * h * (w - 1), grad_map);
    return end(ctx, "tv_vjp");
}

extern "C" dpcs_status dpcs_l1_loss(dpcs_context ctx, const float* a, const float* b, int64_t n, float* loss) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    dpcs_status st = begin(ctx);
    if (st != DPCS_OK) return st;
    if (!a || !b || !loss || n < 1 || n >= (int64_t(1) << 31))
        return fail(ctx, DPCS_E_INVALID, "l1_loss: a, b, loss must not be NULL and 1 <= n < 2^31");
    double* part = (double*)scratch(ctx, "loss.part", sizeof(double) * 2 * RED_MAX_BLOCKS, &st);
    if (!part) return st;
    const unsigned nb = red_grid(n);
    hipLaunchKernelGGL(k_l1_partial, dim3(nb), dim3(RED_TB), 0, ctx->stream, a, b, n, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(RED_TB), 0, ctx->stream, part, (int)nb, (double)n, 0.0, loss);
    return end(ctx, "l1_loss");
}

extern "C" dpcs_status dpcs_l1_vjp(dpcs_context ctx, const float* a, const float* b, int64_t n,
                                   const float* grad_loss, float* grad_a) {
    if (!ctx) return DPCS_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    dpcs_status st = begin(ctx);
    if (st != DPCS_OK) return st;
    if (!a || !b || !grad_loss || !grad_a || n < 1 || n >= (int64_t(1) << 31))
        return fail(ctx, DPCS_E_INVALID, "l1_vjp: pointers must not be NULL and 1 <= n < 2^31");
    if (grad_a == a || grad_a == b) return fail(ctx, DPCS_E_INVALID, "l1_vjp: grad_a must not be an input");
    hipLaunchKernelGGL(k_l1_grad, dim3(red_grid(n)), dim3(RED_TB), 0, ctx->stream, a, b, n, grad_loss, grad_a);
    return end(ctx, "l1_vjp");
}
