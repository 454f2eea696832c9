// Rounding of an LP point and the LP restricted to a subset of labels.
//
// Kleinberg and Tardos's rounding for the uniform metric (the Potts model;
// Sec. 6 cites it for the LP relaxation's factor-2 bound): rounds r = 0, 1,
// ... carry a label i_r and a threshold theta_r (drawn by the caller,
// uniform in [0, 1)); a pixel takes the label of the first round with
// y_a(i_r) > theta_r, so P(x_a = i) = y_a(i). The rounds are independent of
// the pixels, so every pixel scans them on its own: one thread per pixel,
// about L rounds each on average. Pixels that no round reaches take the
// argmax of y (lowest label on ties) and are counted.
//
// The LP restricted to a label subset S (Sec. 7 suggests restricting the LP
// to the labels present in another method's solution; App. I discards
// labels of small probability): the subset's columns of phi and y are
// gathered into N x |S| arrays, y's are projected onto the simplex, the
// projected subgradient descent runs on |S| labels (its cost is |S| sorts
// and divide-and-conquer passes instead of L), and the result is scattered
// back with the other labels at 0, where eq. potts-lp gives them no cost.

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

constexpr int kTP = 256;   // pixels per block

__global__ void k_fill_ints(int *__restrict__ p, int n, int v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(kTP)
k_kt_round(const int *__restrict__ seg, int nimg, int L, const T *__restrict__ y, int R,
           const int32_t *__restrict__ rlab, const T *__restrict__ rth,
           int32_t *__restrict__ x, int *__restrict__ counters) {
    int lo, hi;
    tile_range(seg, nimg, kTP, blockIdx.x, lo, hi);
    const int a = lo + (int)threadIdx.x;
    bool left = false, bad = false;
    if (a < hi) {
        const T *row = y + (size_t)a * L;
        int lab = -1;
        for (int r = 0; r < R && lab < 0; ++r) {
            const int i = rlab[r];
            if (i < 0 || i >= L) {
                bad = true;
                continue;
            }
            if (row[i] > rth[r]) lab = i;
        }
        if (lab < 0) {   // no round reached the pixel: the argmax of y
            lab = 0;
            T best = row[0];
            for (int i = 1; i < L; ++i)
                if (row[i] > best) best = row[i], lab = i;
            left = true;
        }
        x[a] = lab;
    }
    // counters[0]: pixels left to the argmax, counters[1]: a round's label
    // outside [0, L)
    const int nl = __syncthreads_count(left);
    const int nb = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
        if (nl) atomicAdd(&counters[0], nl);
        if (nb) atomicOr(&counters[1], 1);
    }
}

// flags[i] = 1 if some pixel has y_a(i) > tau
template <typename T>
__global__ void __launch_bounds__(kTP)
k_label_present(const int *__restrict__ seg, int nimg, int L, const T *__restrict__ y,
                T tau, int *__restrict__ flags) {
    int lo, hi;
    tile_range(seg, nimg, kTP, blockIdx.x, lo, hi);
    for (size_t e = (size_t)lo * L + threadIdx.x; e < (size_t)hi * L; e += kTP) {
        const int i = int(e % L);
        if (y[e] > tau && flags[i] == 0) atomicOr(&flags[i], 1);
    }
}

// flags[x_a] = 1 for every pixel; counters[0] = 1 for a label outside [0, L)
__global__ void __launch_bounds__(kTP)
k_labels_used(const int *__restrict__ seg, int nimg, int L, const int32_t *__restrict__ x,
              int *__restrict__ flags, int *__restrict__ bad) {
    int lo, hi;
    tile_range(seg, nimg, kTP, blockIdx.x, lo, hi);
    const int a = lo + (int)threadIdx.x;
    if (a >= hi) return;
    const int k = x[a];
    if (k < 0 || k >= L) {
        atomicOr(bad, 1);
        return;
    }
    if (flags[k] == 0) atomicOr(&flags[k], 1);
}

// dst[a][k] = src[a][idx[k]] (N x L -> N x S)
template <typename T>
__global__ void k_gather_cols(int N, int L, int S, const int32_t *__restrict__ idx,
                              const T *__restrict__ src, T *__restrict__ dst) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * S) return;
    const size_t a = e / S;
    dst[e] = src[a * L + idx[e - a * S]];
}

// dst[a][i] = src[a][k] if idx[k] = i, else 0 (N x S -> N x L); pos[i] = k
// or -1
template <typename T>
__global__ void k_scatter_cols(int N, int L, int S, const int32_t *__restrict__ pos,
                               const T *__restrict__ src, T *__restrict__ dst) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * L) return;
    const size_t a = e / L;
    const int k = pos[e - a * L];
    dst[e] = k >= 0 ? src[a * S + k] : T(0);
}

template <typename T>
int round_kt_t(dcrf_ctx *ctx, const T *y, int L, const int32_t *rlab, const T *rth,
               int R, int32_t *x) {
    const hipStream_t st = ctx->stream;
    ctx->small.ensure(4096, st);
    int *cnt = ctx->small.as<int>();
    hipLaunchKernelGGL((k_fill_ints), dim3(1), dim3(64), 0, st, cnt, 2, 0);
    hipLaunchKernelGGL((k_kt_round<T>), dim3(seg_tiles(ctx, kTP)), dim3(kTP), 0, st,
                       ctx->seg.as<int>(), ctx->nimg, L, y, R, rlab, rth, x, cnt);
    DCRF_CHECK_LAUNCH();
    int h[2] = {0, 0};
    DCRF_TRY_HIP(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    if (h[1]) fail(DCRF_EINVAL, "a round's label lies outside [0, L)");
    return h[0];
}

template <typename T>
int present_labels_t(dcrf_ctx *ctx, const T *y, int L, double tau, int32_t *out) {
    const hipStream_t st = ctx->stream;
    ctx->small.ensure(4096, st);
    int *flags = ctx->small.as<int>();
    hipLaunchKernelGGL((k_fill_ints), dim3(1), dim3(256), 0, st, flags, L, 0);
    hipLaunchKernelGGL((k_label_present<T>), dim3(seg_tiles(ctx, kTP)), dim3(kTP), 0, st,
                       ctx->seg.as<int>(), ctx->nimg, L, y, T(tau), flags);
    DCRF_CHECK_LAUNCH();
    int h[256];
    DCRF_TRY_HIP(hipMemcpyAsync(h, flags, (size_t)L * 4, hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    int n = 0;
    for (int i = 0; i < L; ++i)
        if (h[i]) out[n++] = i;
    return n;
}

int labels_used_t(dcrf_ctx *ctx, const int32_t *x, int L, int32_t *out) {
    const hipStream_t st = ctx->stream;
    ctx->small.ensure(4096, st);
    int *flags = ctx->small.as<int>();
    hipLaunchKernelGGL((k_fill_ints), dim3(1), dim3(256), 0, st, flags, L + 1, 0);
    hipLaunchKernelGGL((k_labels_used), dim3(seg_tiles(ctx, kTP)), dim3(kTP), 0, st,
                       ctx->seg.as<int>(), ctx->nimg, L, x, flags, flags + L);
    DCRF_CHECK_LAUNCH();
    int h[257];
    DCRF_TRY_HIP(hipMemcpyAsync(h, flags, (size_t)(L + 1) * 4, hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    if (h[L]) fail(DCRF_EINVAL, "a label lies outside [0, L)");
    int n = 0;
    for (int i = 0; i < L; ++i)
        if (h[i]) out[n++] = i;
    return n;
}

template <typename T>
void lp_descent_subset_t(dcrf_ctx *ctx, const T *phi, int L, T *y, const int32_t *subset,
                         int S, int steps, double beta0, double *best, T *best_y,
                         double *hist) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N;
    const size_t NS = (size_t)N * S, NL = (size_t)N * L;
    // subset indices, then each label's position in the subset (or -1)
    int h[512];
    for (int i = 0; i < L; ++i) h[S + i] = -1;
    for (int k = 0; k < S; ++k) h[k] = subset[k], h[S + subset[k]] = k;
    ctx->small.ensure(4096, st);
    int *idx = ctx->small.as<int>(), *pos = idx + S;
    DCRF_TRY_HIP(hipMemcpyAsync(idx, h, (size_t)(S + L) * 4, hipMemcpyHostToDevice, st));
    for (DevBuf *b : {&ctx->sub_phi, &ctx->sub_y}) b->ensure(NS * sizeof(T), st);
    if (best_y) ctx->sub_best.ensure(NS * sizeof(T), st);
    T *sp = ctx->sub_phi.as<T>(), *sy = ctx->sub_y.as<T>();
    const int gS = ceil_div((long long)NS, 256), gL = ceil_div((long long)NL, 256);
    hipLaunchKernelGGL((k_gather_cols<T>), dim3(gS), dim3(256), 0, st, N, L, S, idx, phi, sp);
    hipLaunchKernelGGL((k_gather_cols<T>), dim3(gS), dim3(256), 0, st, N, L, S, idx, y, sy);
    DCRF_CHECK_LAUNCH();
    project_simplex(ctx, sy, S, sy);
    lp_descent(ctx, sp, S, sy, steps, beta0, best, best_y ? ctx->sub_best.p : nullptr,
               hist);
    hipLaunchKernelGGL((k_scatter_cols<T>), dim3(gL), dim3(256), 0, st, N, L, S, pos, sy, y);
    if (best_y)
        hipLaunchKernelGGL((k_scatter_cols<T>), dim3(gL), dim3(256), 0, st, N, L, S, pos,
                           ctx->sub_best.as<T>(), best_y);
    DCRF_CHECK_LAUNCH();
}

}  // namespace

int round_kt(dcrf_ctx *ctx, const void *y, int L, const int32_t *rlab, const void *rth,
             int R, int32_t *labels) {
    if (ctx->dtype == DCRF_F64)
        return round_kt_t<double>(ctx, static_cast<const double *>(y), L, rlab,
                                  static_cast<const double *>(rth), R, labels);
    return round_kt_t<float>(ctx, static_cast<const float *>(y), L, rlab,
                             static_cast<const float *>(rth), R, labels);
}

int present_labels(dcrf_ctx *ctx, const void *y, int L, double tau, int32_t *out) {
    if (ctx->dtype == DCRF_F64)
        return present_labels_t<double>(ctx, static_cast<const double *>(y), L, tau, out);
    return present_labels_t<float>(ctx, static_cast<const float *>(y), L, tau, out);
}

int labels_used(dcrf_ctx *ctx, const int32_t *labels, int L, int32_t *out) {
    return labels_used_t(ctx, labels, L, out);
}

void lp_descent_subset(dcrf_ctx *ctx, const void *unary, int L, void *y,
                       const int32_t *subset, int S, int steps, double beta0,
                       double *best, void *best_y, double *hist) {
    if (ctx->dtype == DCRF_F64)
        lp_descent_subset_t<double>(ctx, static_cast<const double *>(unary), L,
                                    static_cast<double *>(y), subset, S, steps, beta0, best,
                                    static_cast<double *>(best_y), hist);
    else
        lp_descent_subset_t<float>(ctx, static_cast<const float *>(unary), L,
                                   static_cast<float *>(y), subset, S, steps, beta0, best,
                                   static_cast<float *>(best_y), hist);
}

}  // namespace dcrf
