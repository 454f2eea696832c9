// The separable filter mode: kernels on position alone by the exact sum,
// computed as two one-dimensional convolutions; the other kernels by the
// lattice.
//
// A kernel with features (x / theta, y / theta) (eq. gaussiankernel with
// App. G's scaling) is exp(-(dx^2 + dy^2) / (2 theta^2)) =
// g(dx) g(dy) with g(t) = exp(-t^2 / (2 theta^2)), so K Y is a convolution
// of every channel along the image rows with the taps g(-R..R) followed by
// one along the columns. Taps with |t| > theta sqrt(120 ln 2) are below
// 2^-60 of the centre tap and are dropped (no FP64 result changes); R is also
// capped at the image's larger side minus one. The sum includes the pixel
// itself (g(0) = 1), which the self-term subtraction removes as for every
// kernel: K'Y = sum_m w_m K_m Y - (sum_m w_m) Y.
//
// Row pass: a block holds one row segment of 64 pixels and its R-pixel halo
// (all channels) in LDS, loaded as one contiguous range. Column pass: a
// block holds a tile of TX columns by 64 rows plus its halo rows. Where the
// tile and halo do not fit in 64 KB of LDS (very wide kernels or many
// channels), each output reads its taps from global memory instead.

#include <cmath>
#include <vector>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

constexpr int kSepThreads = 256;
constexpr int kSepSeg = 64;                 // pixels per row segment / rows per column tile
constexpr size_t kSepLds = 64 * 1024;       // dynamic LDS limit of the staged passes

// out = taps[0] in + sum_t taps[t] (in[-t] + in[+t]) along the rows (LDS)
template <typename T>
__global__ void __launch_bounds__(kSepThreads)
k_sep_rows(int H, int W, int C, const T *__restrict__ in, T *__restrict__ out,
           const T *__restrict__ taps, int R) {
    extern __shared__ unsigned char sep_smem[];
    T *s = reinterpret_cast<T *>(sep_smem);
    const int r = blockIdx.y;
    const int x0 = blockIdx.x * kSepSeg;
    const int xa = x0 - R;
    const int span = kSepSeg + 2 * R;
    const T *row = in + (size_t)r * W * C;
    for (int i = threadIdx.x; i < span * C; i += kSepThreads) {
        const int px = xa + i / C;
        s[i] = (px >= 0 && px < W) ? row[(size_t)px * C + (i % C)] : T(0);
    }
    __syncthreads();
    const int nx = min(kSepSeg, W - x0);
    T *orow = out + ((size_t)r * W + x0) * C;
    for (int o = threadIdx.x; o < nx * C; o += kSepThreads) {
        const T *b = s + (o / C + R) * C + (o % C);
        T acc = taps[0] * b[0];
        for (int t = 1; t <= R; ++t) acc += taps[t] * (b[-t * C] + b[t * C]);
        orow[o] = acc;
    }
}

// the same along the columns, a tile of TX columns x kSepSeg rows (LDS)
template <typename T>
__global__ void __launch_bounds__(kSepThreads)
k_sep_cols(int H, int W, int C, int TX, const T *__restrict__ in, T *__restrict__ out,
           const T *__restrict__ taps, int R) {
    extern __shared__ unsigned char sep_smem[];
    T *s = reinterpret_cast<T *>(sep_smem);
    const int x0 = blockIdx.x * TX;
    const int y0 = blockIdx.y * kSepSeg;
    const int nx = min(TX, W - x0);
    const int seg = nx * C;            // contiguous values of one row of the tile
    const int ld = TX * C;
    const int span = kSepSeg + 2 * R;
    for (int i = threadIdx.x; i < span * seg; i += kSepThreads) {
        const int rr = i / seg, k = i - rr * seg;
        const int py = y0 - R + rr;
        s[rr * ld + k] = (py >= 0 && py < H) ? in[((size_t)py * W + x0) * C + k] : T(0);
    }
    __syncthreads();
    const int ny = min(kSepSeg, H - y0);
    for (int o = threadIdx.x; o < ny * seg; o += kSepThreads) {
        const int rr = o / seg, k = o - rr * seg;
        const T *b = s + (rr + R) * ld + k;
        T acc = taps[0] * b[0];
        for (int t = 1; t <= R; ++t) acc += taps[t] * (b[-t * ld] + b[t * ld]);
        out[((size_t)(y0 + rr) * W + x0) * C + k] = acc;
    }
}

// unstaged form of either pass: one thread per output value
template <typename T>
__global__ void k_sep_direct(int H, int W, int C, int along_rows, const T *__restrict__ in,
                             T *__restrict__ out, const T *__restrict__ taps, int R) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)H * W * C) return;
    const size_t a = e / C;
    const int y = int(a / W), x = int(a - (size_t)y * W);
    const int pos = along_rows ? x : y, len = along_rows ? W : H;
    const size_t step = along_rows ? (size_t)C : (size_t)W * C;
    T acc = taps[0] * in[e];
    for (int t = 1; t <= R; ++t) {
        const T lft = pos - t >= 0 ? in[e - t * step] : T(0);
        const T rgt = pos + t < len ? in[e + t * step] : T(0);
        acc += taps[t] * (lft + rgt);
    }
    out[e] = acc;
}

// y = a x (n values)
template <typename T>
__global__ void k_scale(size_t n, T a, const T *__restrict__ x, T *__restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// y += a x
template <typename T>
__global__ void k_axpy(size_t n, T a, const T *__restrict__ x, T *__restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

// K_m in for a position-only kernel m, exactly: rows, then columns
template <typename T>
void separable_kernel_t(dcrf_ctx *ctx, int m, const T *in, T *out, int C) {
    const hipStream_t st = ctx->stream;
    const int H = ctx->H, W = ctx->W;
    const size_t NC = (size_t)ctx->N * C, e = sizeof(T);
    const double theta = ctx->kern[m].theta_pos;
    int R = (int)std::ceil(theta * std::sqrt(120.0 * std::log(2.0)));
    R = std::max(0, std::min(R, std::max(H, W) - 1));
    std::vector<T> h(R + 1);
    for (int t = 0; t <= R; ++t) h[t] = T(std::exp(-double(t) * t / (2.0 * theta * theta)));
    ctx->sep_taps.ensure((size_t)(R + 1) * e, st);
    DCRF_TRY_HIP(hipMemcpyAsync(ctx->sep_taps.p, h.data(), (size_t)(R + 1) * e,
                                hipMemcpyHostToDevice, st));
    ctx->sep_tmp.ensure(NC * e, st);
    const T *taps = ctx->sep_taps.as<T>();
    T *mid = ctx->sep_tmp.as<T>();
    const size_t lds_rows = (size_t)(kSepSeg + 2 * R) * C * e;
    if (lds_rows <= kSepLds) {
        hipLaunchKernelGGL((k_sep_rows<T>), dim3(ceil_div(W, kSepSeg), H), dim3(kSepThreads),
                           lds_rows, st, H, W, C, in, mid, taps, R);
    } else {
        hipLaunchKernelGGL((k_sep_direct<T>), dim3(ceil_div((long long)NC, 256)), dim3(256), 0,
                           st, H, W, C, 1, in, mid, taps, R);
    }
    const size_t per_col = (size_t)(kSepSeg + 2 * R) * C * e;
    const int TX = (int)std::min<size_t>(16, kSepLds / per_col);
    if (TX >= 1) {
        hipLaunchKernelGGL((k_sep_cols<T>), dim3(ceil_div(W, TX), ceil_div(H, kSepSeg)),
                           dim3(kSepThreads), per_col * TX, st, H, W, C, TX, mid, out, taps, R);
    } else {
        hipLaunchKernelGGL((k_sep_direct<T>), dim3(ceil_div((long long)NC, 256)), dim3(256), 0,
                           st, H, W, C, 0, mid, out, taps, R);
    }
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void filter_separable_t(dcrf_ctx *ctx, const T *in, T *out, int C, bool adjoint) {
    const hipStream_t st = ctx->stream;
    const size_t NC = (size_t)ctx->N * C;
    const int g = ceil_div((long long)NC, 256);
    ctx->sep_acc.ensure(NC * sizeof(T), st);
    T *acc = ctx->sep_acc.as<T>();
    hipLaunchKernelGGL((k_scale<T>), dim3(g), dim3(256), 0, st, NC, T(-ctx->wsum), in, out);
    for (int m = 0; m < ctx->nk; ++m) {
        if (ctx->kern[m].use_rgb)
            filter_kernel(ctx, m, in, acc, C, adjoint);   // K~_m, calibrated lattice
        else
            separable_kernel_t<T>(ctx, m, in, acc, C);     // symmetric: its own adjoint
        hipLaunchKernelGGL((k_axpy<T>), dim3(g), dim3(256), 0, st, NC,
                           T(ctx->kern[m].weight), acc, out);
    }
    DCRF_CHECK_LAUNCH();
}

}  // namespace

void filter_separable(dcrf_ctx *ctx, const void *in, void *out, int C, bool adjoint) {
    if (ctx->nimg > 1)
        fail(DCRF_EUNSUPPORTED, "the separable filter mode takes a single image");
    if (ctx->dtype == DCRF_F64)
        filter_separable_t<double>(ctx, static_cast<const double *>(in),
                                   static_cast<double *>(out), C, adjoint);
    else
        filter_separable_t<float>(ctx, static_cast<const float *>(in),
                                  static_cast<float *>(out), C, adjoint);
}

}  // namespace dcrf
