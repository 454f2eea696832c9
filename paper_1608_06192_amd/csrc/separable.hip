// The separable filter mode: kernels on position alone by the exact sum,
// computed as two one-dimensional convolutions; the other kernels by the
// lattice. Also the filter's per-kernel and self-keeping variants.
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
// block holds a tile of TX columns by 64 rows plus its halo rows, TX chosen
// to keep the tile near 20 KB so that several blocks share a CU. The taps sit
// in LDS beside the tile. A lane computes 8 consecutive outputs of one
// channel with a window that slides in registers (one LDS read per input
// instead of two per tap and output). The column pass also forms the filter's result
// (the weighted sum, the other kernels' part and the self term) as it
// writes. Where a tile and its halo do not fit
// in 64 KB of LDS (very wide kernels or many channels), each output reads its
// taps from global memory instead.

#include <cmath>
#include <vector>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

constexpr int kSepThreads = 256;
constexpr int kSepSeg = 64;                 // pixels per row segment / rows per column tile
constexpr size_t kSepLds = 64 * 1024;       // dynamic LDS limit of the staged passes
constexpr size_t kSepColLds = 20 * 1024;    // target LDS of a column tile

// kRun consecutive outputs of one channel along the pass, from LDS:
// acc[j] = sum_{t=-R..R} tp[|t|] x[(j + t) ld]. A window of kRun inputs
// slides along t in registers, so each input is read from LDS once (kRun + 2R
// reads for kRun (2R + 1) multiply-adds); the taps sit in LDS (a broadcast
// read per t).
constexpr int kRun = 8;

template <typename T>
__device__ __forceinline__ void sep_window(const T *x, int ld, const T *tp, int R,
                                           T (&acc)[kRun]) {
    T w[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        w[j] = x[(j - R) * ld];
        acc[j] = T(0);
    }
#pragma unroll 4
    for (int t = -R; t <= R; ++t) {
        const T g = tp[t < 0 ? -t : t];
#pragma unroll
        for (int j = 0; j < kRun; ++j) acc[j] += g * w[j];
#pragma unroll
        for (int j = 0; j + 1 < kRun; ++j) w[j] = w[j + 1];
        if (t < R) w[kRun - 1] = x[(kRun + t) * ld];
    }
}

// out = sum_t taps[|t|] in[x + t] along the rows: a row segment of kSepSeg
// pixels and its halo in LDS, one lane per output value
template <typename T>
__global__ void __launch_bounds__(kSepThreads)
k_sep_rows(int H, int W, int C, const T *__restrict__ in, T *__restrict__ out,
           const T *__restrict__ taps, int R) {
    extern __shared__ unsigned char sep_smem[];
    T *tp = reinterpret_cast<T *>(sep_smem);
    T *s = tp + (R + 1);
    const int r = blockIdx.y;
    const int x0 = blockIdx.x * kSepSeg;
    const int xa = x0 - R;
    const int span = kSepSeg + 2 * R;
    const T *row = in + (size_t)r * W * C;
    for (int i = threadIdx.x; i <= R; i += kSepThreads) tp[i] = taps[i];
    // the segment and its halo are one contiguous range of the row: values
    // outside the row are zero
    const long long g0 = (long long)xa * C, gend = (long long)W * C;
    for (int i = threadIdx.x; i < span * C; i += kSepThreads) {
        const long long g = g0 + i;
        s[i] = (g >= 0 && g < gend) ? row[g] : T(0);
    }
    __syncthreads();
    const int nx = min(kSepSeg, W - x0);
    const int runs = (nx + kRun - 1) / kRun;
    T *orow = out + ((size_t)r * W + x0) * C;
    for (int task = threadIdx.x; task < runs * C; task += kSepThreads) {
        const int run = task / C, c = task - run * C;
        const int p0 = run * kRun;
        T acc[kRun];
        sep_window<T>(s + (p0 + R) * C + c, C, tp, R, acc);
#pragma unroll
        for (int j = 0; j < kRun; ++j)
            if (p0 + j < nx) orow[(size_t)(p0 + j) * C + c] = acc[j];
    }
}

// the same along the columns, a tile of TX columns x kSepSeg rows (LDS), 8
// rows per lane; the epilogue writes
// alpha conv + (add ? gamma add : 0) + beta self (self: the filter's input)
template <typename T>
__global__ void __launch_bounds__(kSepThreads)
k_sep_cols(int H, int W, int C, int TX, const T *__restrict__ in, T *out,
           const T *__restrict__ taps, int R, T alpha, const T *add, T gamma, T beta,
           const T *__restrict__ self) {
    extern __shared__ unsigned char sep_smem[];
    T *tp = reinterpret_cast<T *>(sep_smem);
    T *s = tp + (R + 1);
    const int x0 = blockIdx.x * TX;
    const int y0 = blockIdx.y * kSepSeg;
    const int nx = min(TX, W - x0);
    const int seg = nx * C;            // contiguous values of one row of the tile
    const int ld = TX * C;
    const int span = kSepSeg + 2 * R;
    for (int i = threadIdx.x; i <= R; i += kSepThreads) tp[i] = taps[i];
    // lane -> (first row, value in the row), then whole rows per step
    const int per = max(1, kSepThreads / seg);
    const int k0 = (int)threadIdx.x % seg, r0 = (int)threadIdx.x / seg;
    if (r0 < per) {
        for (int rr = r0; rr < span; rr += per) {
            const int py = y0 - R + rr;
            s[rr * ld + k0] = (py >= 0 && py < H) ? in[((size_t)py * W + x0) * C + k0] : T(0);
        }
    }
    // a row longer than the block: the rest of each row
    for (int k = kSepThreads + (int)threadIdx.x; k < seg; k += kSepThreads)
        for (int rr = 0; rr < span; ++rr) {
            const int py = y0 - R + rr;
            s[rr * ld + k] = (py >= 0 && py < H) ? in[((size_t)py * W + x0) * C + k] : T(0);
        }
    __syncthreads();
    const int ny = min(kSepSeg, H - y0);
    const int runs = (ny + kRun - 1) / kRun;
    for (int task = threadIdx.x; task < runs * seg; task += kSepThreads) {
        const int run = task / seg, k = task - run * seg;
        const int r0 = run * kRun;
        T acc[kRun];
        sep_window<T>(s + (r0 + R) * ld + k, ld, tp, R, acc);
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            if (r0 + j >= ny) continue;
            const size_t e = ((size_t)(y0 + r0 + j) * W + x0) * C + k;
            T v = alpha * acc[j] + beta * self[e];
            if (add) v += gamma * add[e];
            out[e] = v;
        }
    }
}

// unstaged form of either pass: one thread per output value
template <typename T>
__global__ void k_sep_direct(int H, int W, int C, int along_rows, const T *__restrict__ in,
                             T *out, const T *__restrict__ taps, int R, T alpha,
                             const T *add, T gamma, T beta, const T *__restrict__ self) {
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
    T v = alpha * acc;
    if (self) v += beta * self[e];
    if (add) v += gamma * add[e];
    out[e] = v;
}

// y = a x (n values; x and y may be the same array)
template <typename T>
__global__ void k_scale(size_t n, T a, const T *x, T *y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// y += a x
template <typename T>
__global__ void k_axpy(size_t n, T a, const T *__restrict__ x, T *__restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

// out = alpha K_m in + gamma add + beta in for a position-only kernel m, K_m
// exactly: the row pass, then the column pass with the combination fused in
// (add may be null)
template <typename T>
void separable_kernel_t(dcrf_ctx *ctx, int m, const T *in, T *out, int C, T alpha,
                        const T *add, T gamma, T beta) {
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
    const size_t lds_rows = ((size_t)(kSepSeg + 2 * R) * C + R + 1) * e;
    if (lds_rows <= kSepLds) {
        hipLaunchKernelGGL((k_sep_rows<T>), dim3(ceil_div(W, kSepSeg), H), dim3(kSepThreads),
                           lds_rows, st, H, W, C, in, mid, taps, R);
    } else {
        hipLaunchKernelGGL((k_sep_direct<T>), dim3(ceil_div((long long)NC, 256)), dim3(256), 0,
                           st, H, W, C, 1, in, mid, taps, R, T(1), (const T *)nullptr, T(0),
                           T(0), (const T *)nullptr);
    }
    // columns per tile: as many as keep the tile within kSepColLds (several
    // blocks per CU hide the LDS latency), at least one within kSepLds
    const size_t per_col = (size_t)(kSepSeg + 2 * R) * C * e;
    const size_t tap_bytes = (size_t)(R + 1) * e;
    int TX = (int)std::min<size_t>(16, kSepColLds / per_col);
    if (TX < 1 && per_col + tap_bytes <= kSepLds) TX = 1;
    if (TX >= 1) {
        hipLaunchKernelGGL((k_sep_cols<T>), dim3(ceil_div(W, TX), ceil_div(H, kSepSeg)),
                           dim3(kSepThreads), per_col * TX + tap_bytes, st, H, W, C, TX, mid, out,
                           taps, R,
                           alpha, add, gamma, beta, in);
    } else {
        hipLaunchKernelGGL((k_sep_direct<T>), dim3(ceil_div((long long)NC, 256)), dim3(256), 0,
                           st, H, W, C, 0, mid, out, taps, R, alpha, add, gamma, beta, in);
    }
    DCRF_CHECK_LAUNCH();
}

// K'Y = sum_m w_m K_m Y - (sum w) Y: the lattice kernels' sum into a
// scratch array, then the position-only kernels, the last of which writes
// out = w K Y + (the sum so far) - (sum w) Y in its column pass
template <typename T>
void filter_separable_t(dcrf_ctx *ctx, const T *in, T *out, int C, bool adjoint) {
    const hipStream_t st = ctx->stream;
    const size_t NC = (size_t)ctx->N * C;
    const int g = ceil_div((long long)NC, 256);
    int last_sep = -1;
    for (int m = 0; m < ctx->nk; ++m)
        if (!ctx->kern[m].use_rgb) last_sep = m;
    // acc * acc_w holds the sum of w_m K_m Y so far (acc_w: the weight of a
    // single lattice kernel, applied in the last pass's epilogue)
    T *acc = nullptr, *part = nullptr;
    T acc_w = T(1);
    bool have = false;
    auto need_acc = [&] {
        if (!acc) {
            ctx->sep_acc.ensure(NC * sizeof(T), st);
            acc = ctx->sep_acc.as<T>();
        }
    };
    for (int m = 0; m < ctx->nk; ++m) {
        if (!ctx->kern[m].use_rgb) continue;
        need_acc();
        if (!have) {
            filter_kernel(ctx, m, in, acc, C, adjoint);   // K~_m Y, calibrated lattice
            acc_w = T(ctx->kern[m].weight);
            have = true;
            continue;
        }
        if (acc_w != T(1)) {   // a second lattice kernel: make acc the plain sum
            hipLaunchKernelGGL((k_scale<T>), dim3(g), dim3(256), 0, st, NC, acc_w, acc, acc);
            acc_w = T(1);
        }
        if (!part) {
            ctx->sep_part.ensure(NC * sizeof(T), st);
            part = ctx->sep_part.as<T>();
        }
        filter_kernel(ctx, m, in, part, C, adjoint);
        hipLaunchKernelGGL((k_axpy<T>), dim3(g), dim3(256), 0, st, NC,
                           T(ctx->kern[m].weight), part, acc);
    }
    if (last_sep < 0) {   // no position-only kernel: out = acc_w acc - (sum w) Y
        hipLaunchKernelGGL((k_scale<T>), dim3(g), dim3(256), 0, st, NC, acc_w, acc, out);
        hipLaunchKernelGGL((k_axpy<T>), dim3(g), dim3(256), 0, st, NC, T(-ctx->wsum), in,
                           out);
        DCRF_CHECK_LAUNCH();
        return;
    }
    for (int m = 0; m < ctx->nk; ++m) {
        if (ctx->kern[m].use_rgb) continue;
        const T w = T(ctx->kern[m].weight);
        if (m == last_sep) {
            // symmetric: its own adjoint
            separable_kernel_t<T>(ctx, m, in, out, C, w, have ? acc : nullptr, acc_w,
                                  T(-ctx->wsum));
        } else {
            need_acc();
            separable_kernel_t<T>(ctx, m, in, acc, C, w, have ? acc : nullptr, acc_w, T(0));
            acc_w = T(1);
            have = true;
        }
    }
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void filter_parts_t(dcrf_ctx *ctx, const T *in, T *out, int C, bool adjoint, int kind,
                    bool keep_self, bool per_kernel) {
    const hipStream_t st = ctx->stream;
    const size_t NC = (size_t)ctx->N * C;
    const int g = ceil_div((long long)NC, 256);
    if (!per_kernel) {
        filter_apply(ctx, in, out, C, adjoint, kind);
        if (keep_self)
            hipLaunchKernelGGL((k_axpy<T>), dim3(g), dim3(256), 0, st, NC, T(ctx->wsum), in,
                               out);
        DCRF_CHECK_LAUNCH();
        return;
    }
    for (int m = 0; m < ctx->nk; ++m) {
        T *blk = out + (size_t)m * NC;
        const T w = T(ctx->kern[m].weight);
        // blk = K_m in with its self term
        if (kind == DCRF_FILTER_EXACT) {
            exact_kernel(ctx, m, in, blk, C);   // the pairs b != a
            hipLaunchKernelGGL((k_axpy<T>), dim3(g), dim3(256), 0, st, NC, T(1), in, blk);
        } else if (kind == DCRF_FILTER_SEPARABLE && !ctx->kern[m].use_rgb) {
            separable_kernel_t<T>(ctx, m, in, blk, C, T(1), nullptr, T(0), T(0));
        } else {
            filter_kernel(ctx, m, in, blk, C, adjoint);   // calibrated lattice
        }
        hipLaunchKernelGGL((k_scale<T>), dim3(g), dim3(256), 0, st, NC, w, blk, blk);
        if (!keep_self)
            hipLaunchKernelGGL((k_axpy<T>), dim3(g), dim3(256), 0, st, NC, -w, in, blk);
    }
    DCRF_CHECK_LAUNCH();
}

}  // namespace

void filter_parts(dcrf_ctx *ctx, const void *in, void *out, int C, bool adjoint, int kind,
                  bool keep_self, bool per_kernel) {
    if (kind == DCRF_FILTER_SEPARABLE && ctx->nimg > 1)
        fail(DCRF_EUNSUPPORTED, "the separable filter mode takes a single image");
    if (ctx->dtype == DCRF_F64)
        filter_parts_t<double>(ctx, static_cast<const double *>(in),
                               static_cast<double *>(out), C, adjoint, kind, keep_self,
                               per_kernel);
    else
        filter_parts_t<float>(ctx, static_cast<const float *>(in), static_cast<float *>(out),
                              C, adjoint, kind, keep_self, per_kernel);
}

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
