// Reverse-mode derivative of a fixed number T of Frank-Wolfe iterations on the
// convex QP (Sec. 4, App. B), with respect to the unaries phi and the kernel
// weights w_m, for an upstream gradient dl/dy_T.
//
// Forward: y_0 = softmax(-phi), then T iterations of the Frank-Wolfe kernels,
// checkpointing y_t, the conditional gradient s_t and the step's quadratic
// (alpha_t, a2, b1, interior) for every t. P_t = Q y_t and S_t = Q s_t are
// recomputed in the reverse sweep rather than stored.
//
// Reverse sweep, for t = T-1 .. 0 (ybar = dl/dy_{t+1}, Pbar = dl/dP_{t+1}):
//   abar = <ybar, s - y> + <Pbar, S - P>
//   interior alpha = -b1 / (2 a2): b1bar = -abar / (2 a2), a2bar = -abar alpha / a2
//     (a clipped step, and the piecewise-constant s_t, pass no gradient)
//   b1 = cs - cy + B + C - 2A, a2 = D - B - C + A with A = <y,P>, B = <y,S>,
//     C = <s,P>, D = <s,S>, cy = <c,y>, cs = <c,s>
//   Sbar = alpha Pbar + Bbar y + Dbar s
//   ybar <- (1 - alpha) ybar + Abar P + Bbar S + cybar c
//   Pbar <- (1 - alpha) Pbar + Abar y + Cbar s,  cbar += cybar y + csbar s
// then P_0 = Q y_0 gives ybar += Q^T Pbar = K'^T (Pbar mu) + d * Pbar (the
// transposed lattice filter: blur directions reversed), c = phi - d gives
// phibar = cbar, and y_0 = softmax(-phi) the softmax backward.
// The weights enter Q (through K' and d) and c (through d):
//   d<Zbar, Q X>/dw_m = <Zbar mu, (K~_m - I) X> + sum_a rho_a (K~_m 1 - 1)_a,
//   rho_a = sum_i Zbar_a(i) X_a(i) sum_j |mu_ij|,
// with K~_m the lattice filter of kernel m alone.
//
// For a context that holds a batch of images every image has its own step
// sizes, step adjoints and weight gradient: the reductions are per tile of
// one image (whole pixels per block) and summed per image on the host.

#include <algorithm>
#include <cmath>
#include <vector>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

constexpr int kThreads = 256;
constexpr int kGroups = 8;   // pixel groups (kThreads / L pixels) per tile

template <typename T>
__global__ void k_softmax_neg(const int *__restrict__ seg, int nimg, int L,
                              const T *__restrict__ phi, T *__restrict__ y) {
    int lo, hi;
    tile_range(seg, nimg, 256, blockIdx.x, lo, hi);
    const int a = lo + threadIdx.x;
    if (a >= hi) return;
    const T *p = phi + (size_t)a * L;
    T mn = p[0];
    for (int i = 1; i < L; ++i) mn = fmin(mn, p[i]);
    T s = T(0);
    for (int i = 0; i < L; ++i) s += exp(mn - p[i]);
    for (int i = 0; i < L; ++i) y[(size_t)a * L + i] = exp(mn - p[i]) / s;
}

template <typename T>
__global__ void k_mabs(int L, const T *__restrict__ mu, T *__restrict__ mabs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    T s = T(0);
    for (int j = 0; j < L; ++j) s += fabs(mu[(size_t)i * L + j]);
    mabs[i] = s;
}

// c = phi - d, d_a(i) = mabs_i r_a
template <typename T>
__global__ void k_c(int N, int L, const T *__restrict__ phi,
                    const T *__restrict__ r, const T *__restrict__ mabs,
                    T *__restrict__ c) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * L) return;
    const int a = int(e / L);
    c[e] = phi[e] - mabs[e - (size_t)a * L] * r[a];
}

template <typename T>
__global__ void k_onehot_d(int N, int L, const int32_t *__restrict__ s,
                           T *__restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * L) return;
    const int a = int(e / L);
    out[e] = T(int(e - (size_t)a * L) == s[a] ? 1 : 0);
}

template <typename T>
__global__ void k_fill_d(size_t n, T *__restrict__ p, T v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int NV>
__device__ __forceinline__ void bsum(double (&v)[NV], double *lds) {
    block_sum<NV, kThreads>(v, lds);
}

// Pixel rows [lo, hi) of this block's tile (kGroups groups of ppb pixels);
// returns the image.
__device__ __forceinline__ int diff_tile(const int *seg, int nimg, int ppb,
                                         int &lo, int &hi) {
    return tile_range(seg, nimg, ppb * kGroups, blockIdx.x, lo, hi);
}

// per-tile partial sums of abar = <ybar, s - y> + <Pbar, S - P>
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_abar(const int *__restrict__ seg, int nimg, int L, const T *__restrict__ ybar,
       const T *__restrict__ y, const int32_t *__restrict__ s,
       const T *__restrict__ Pbar, const T *__restrict__ S,
       const T *__restrict__ P, double *__restrict__ part) {
    __shared__ double red[kThreads];
    double acc[1] = {0.0};
    int lo, hi;
    diff_tile(seg, nimg, kThreads / L, lo, hi);
    for (size_t e = (size_t)lo * L + threadIdx.x; e < (size_t)hi * L; e += kThreads) {
        const int a = int(e / L);
        const int i = int(e - (size_t)a * L);
        const double si = (i == s[a]) ? 1.0 : 0.0;
        acc[0] += double(ybar[e]) * (si - double(y[e])) +
                  double(Pbar[e]) * (double(S[e]) - double(P[e]));
    }
    bsum<1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

struct StepBar {
    double al, Abar, Bbar, Cbar, Dbar, cybar, csbar;
};

template <typename T>
struct UpdArgs {
    const int *seg;
    int nimg, L, nk;
    T *ybar, *Pbar, *cbar;
    const T *y, *P, *S, *c;
    const int32_t *s;
    const T *Ks[DCRF_MAXK];
    const T *mu, *mabs;
    double *rho;
    double *part;    // per tile: nk partial sums of <Sbar mu, K~_m s - s>
    const StepBar *sb;   // per image
};

// One reverse step (see the file comment), whole pixels per block so that
// (Sbar mu) can be formed from the pixel's row in LDS.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_diff_update(UpdArgs<T> A) {
    __shared__ double rowS[kThreads];
    __shared__ double red[DCRF_MAXK * kThreads];
    const int L = A.L;
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int i = t - lp * L;
    double acc[DCRF_MAXK];
#pragma unroll
    for (int m = 0; m < DCRF_MAXK; ++m) acc[m] = 0.0;
    int lo, hi;
    const int img = diff_tile(A.seg, A.nimg, ppb, lo, hi);
    const StepBar b = A.sb[img < 0 ? 0 : img];
    for (int g0 = lo; g0 < hi; g0 += ppb) {
        const long long a = (long long)g0 + lp;
        const bool act = lp < ppb && a < hi;
        const size_t e = (size_t)a * L + i;
        double sbar = 0.0;
        int sa = 0;
        if (act) {
            sa = A.s[a];
            const double si = i == sa ? 1.0 : 0.0;
            sbar = b.al * double(A.Pbar[e]) + b.Bbar * double(A.y[e]) + b.Dbar * si;
            rowS[t] = sbar;
        }
        __syncthreads();
        if (act) {
            const double si = i == sa ? 1.0 : 0.0;
            double smu = 0.0;   // (Sbar mu)_a(i) = sum_k Sbar_a(k) mu_ki
            for (int k = 0; k < L; ++k)
                smu += rowS[lp * L + k] * double(A.mu[(size_t)k * L + i]);
            for (int m = 0; m < A.nk; ++m)
                acc[m] += smu * (double(A.Ks[m][e]) - si);
            if (i == sa) A.rho[a] += sbar * double(A.mabs[i]);
            const double yv = A.y[e], yb = A.ybar[e], pb = A.Pbar[e];
            A.ybar[e] = T((1.0 - b.al) * yb + b.Abar * double(A.P[e]) +
                          b.Bbar * double(A.S[e]) + b.cybar * double(A.c[e]));
            A.Pbar[e] = T((1.0 - b.al) * pb + b.Abar * yv + b.Cbar * si);
            A.cbar[e] = T(double(A.cbar[e]) + b.cybar * yv + b.csbar * si);
        }
        __syncthreads();
    }
    bsum<DCRF_MAXK>(acc, red);
    if (t < DCRF_MAXK) A.part[(size_t)blockIdx.x * DCRF_MAXK + t] = acc[t];
}

// Z = X mu, row by row: Z_a(j) = sum_i X_a(i) mu_ij
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_rowmat(int N, int L, const T *__restrict__ X, const T *__restrict__ mu,
         T *__restrict__ Z) {
    __shared__ double row[kThreads];
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int j = t - lp * L;
    for (int g = blockIdx.x; (long long)g * ppb < N; g += gridDim.x) {
        const long long a = (long long)g * ppb + lp;
        const bool act = lp < ppb && a < N;
        if (act) row[t] = X[(size_t)a * L + j];
        __syncthreads();
        if (act) {
            double z = 0.0;
            for (int i = 0; i < L; ++i) z += row[lp * L + i] * double(mu[(size_t)i * L + j]);
            Z[(size_t)a * L + j] = T(z);
        }
        __syncthreads();
    }
}

template <typename T>
struct FinArgs {
    const int *seg;
    int nimg, L, nk;
    const T *ybar, *KtZ, *Z, *Pbar, *y0, *cbar, *r, *mabs;
    const T *Ky0[DCRF_MAXK];
    const T *K1[DCRF_MAXK];
    const double *rho;
    T *phibar;
    double *part;   // per tile: nk partial sums
};

// The end of the sweep: P_0 = Q y_0, c = phi - d, d's dependence on w, and
// y_0 = softmax(-phi).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_diff_final(FinArgs<T> A) {
    __shared__ double rowy[kThreads];
    __shared__ double rowr[kThreads];
    __shared__ double red[DCRF_MAXK * kThreads];
    const int L = A.L;
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int i = t - lp * L;
    double acc[DCRF_MAXK];
#pragma unroll
    for (int m = 0; m < DCRF_MAXK; ++m) acc[m] = 0.0;
    int lo, hi;
    diff_tile(A.seg, A.nimg, ppb, lo, hi);
    for (int g0 = lo; g0 < hi; g0 += ppb) {
        const long long a = (long long)g0 + lp;
        const bool act = lp < ppb && a < hi;
        const size_t e = (size_t)a * L + i;
        double yb0 = 0.0, y0 = 0.0;
        if (act) {
            y0 = A.y0[e];
            const double pb = A.Pbar[e];
            const double d = double(A.mabs[i]) * double(A.r[a]);
            yb0 = double(A.ybar[e]) + double(A.KtZ[e]) + d * pb;
            rowy[t] = yb0 * y0;
            // rho contributions of P_0 = Q y_0 and of c = phi - d
            rowr[t] = pb * y0 * double(A.mabs[i]) - double(A.cbar[e]) * double(A.mabs[i]);
            for (int m = 0; m < A.nk; ++m)
                acc[m] += double(A.Z[e]) * (double(A.Ky0[m][e]) - y0);
        }
        __syncthreads();
        if (act) {
            double dot = 0.0, rr = 0.0;
            for (int k = 0; k < L; ++k) {
                dot += rowy[lp * L + k];
                rr += rowr[lp * L + k];
            }
            A.phibar[e] = T(double(A.cbar[e]) - y0 * (yb0 - dot));
            if (i == 0) {
                const double rho = A.rho[a] + rr;
                for (int m = 0; m < A.nk; ++m)
                    acc[m] += rho * (double(A.K1[m][a]) - 1.0);
            }
        }
        __syncthreads();
    }
    bsum<DCRF_MAXK>(acc, red);
    if (t < DCRF_MAXK) A.part[(size_t)blockIdx.x * DCRF_MAXK + t] = acc[t];
}

struct DiffWork {
    DevBuf ybar, Pbar, cbar, P, S, OH, c, Z, KtZ, rho, part, mabs, ones, sb;
    DevBuf Ks[DCRF_MAXK], Ky0[DCRF_MAXK], K1[DCRF_MAXK];
};

DiffWork &diff_work(dcrf_ctx *ctx) {
    if (!ctx->diff) ctx->diff = new DiffWork();
    return *static_cast<DiffWork *>(ctx->diff);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct SavedLayout {
    size_t y, s, stats, total;
};

SavedLayout saved_layout(dcrf_ctx *ctx, int L, int iters) {
    SavedLayout o;
    const size_t NL = (size_t)ctx->N * L;
    o.y = 0;
    o.s = align256(o.y + (size_t)iters * NL * ctx->elt());
    o.stats = align256(o.s + (size_t)iters * ctx->N * 4);
    o.total = align256(o.stats + (size_t)iters * ctx->nimg * kFWStats * 8);
    return o;
}

// Per-image sums of per-tile partials (stride doubles per tile, component k):
// out[j] = sum over the tiles [toff[j], toff[j+1]) of image j.
void image_sums(dcrf_ctx *ctx, const double *d, const std::vector<int> &toff,
                int stride, int ncomp, std::vector<double> &out) {
    const int nt = toff.back();
    std::vector<double> h((size_t)nt * stride);
    DCRF_TRY_HIP(hipMemcpyAsync(h.data(), d, h.size() * 8, hipMemcpyDeviceToHost,
                                ctx->stream));
    DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
    const int nimg = int(toff.size()) - 1;
    out.assign((size_t)nimg * ncomp, 0.0);
    for (int j = 0; j < nimg; ++j)
        for (int t = toff[j]; t < toff[j + 1]; ++t)
            for (int k = 0; k < ncomp; ++k)
                out[(size_t)j * ncomp + k] += h[(size_t)t * stride + k];
}

template <typename T>
void backward_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, int iters,
                const char *saved, const T *grad_y, T *grad_phi, double *grad_w) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N, nk = ctx->nk, nimg = ctx->nimg;
    const int *seg = ctx->seg.as<int>();
    const size_t NL = (size_t)N * L;
    const size_t B = NL * sizeof(T);
    const int TPD = (kThreads / L) * kGroups;
    const int GD = seg_tiles(ctx, TPD);
    const std::vector<int> toff = seg_tile_offsets(ctx, TPD);
    DiffWork &W = diff_work(ctx);
    for (DevBuf *b : {&W.ybar, &W.Pbar, &W.cbar, &W.P, &W.S, &W.OH, &W.c, &W.Z,
                      &W.KtZ})
        b->ensure(B, st);
    for (int m = 0; m < nk; ++m) {
        W.Ks[m].ensure(B, st);
        W.Ky0[m].ensure(B, st);
        W.K1[m].ensure((size_t)N * sizeof(T), st);
    }
    W.rho.ensure((size_t)N * 8, st);
    W.part.ensure((size_t)GD * DCRF_MAXK * 8, st);
    W.mabs.ensure((size_t)L * sizeof(T), st);
    W.ones.ensure((size_t)N * sizeof(T), st);
    W.sb.ensure((size_t)nimg * sizeof(StepBar), st);
    const SavedLayout lay = saved_layout(ctx, L, iters);
    const T *ys = reinterpret_cast<const T *>(saved + lay.y);
    const int32_t *ss = reinterpret_cast<const int32_t *>(saved + lay.s);
    std::vector<double> stats((size_t)iters * nimg * kFWStats);
    DCRF_TRY_HIP(hipMemcpyAsync(stats.data(), saved + lay.stats, stats.size() * 8,
                                hipMemcpyDeviceToHost, st));
    const int gE = ceil_div((long long)NL, 256);
    T *ybar = W.ybar.as<T>(), *Pbar = W.Pbar.as<T>(), *cbar = W.cbar.as<T>();
    DCRF_TRY_HIP(hipMemcpyAsync(ybar, grad_y, B, hipMemcpyDeviceToDevice, st));
    DCRF_TRY_HIP(hipMemsetAsync(Pbar, 0, B, st));
    DCRF_TRY_HIP(hipMemsetAsync(cbar, 0, B, st));
    DCRF_TRY_HIP(hipMemsetAsync(W.rho.p, 0, (size_t)N * 8, st));
    hipLaunchKernelGGL((k_mabs<T>), dim3(1), dim3(256), 0, st, L, mu, W.mabs.as<T>());
    hipLaunchKernelGGL((k_c<T>), dim3(gE), dim3(256), 0, st, N, L, phi,
                       ctx->r.as<T>(), W.mabs.as<T>(), W.c.as<T>());
    DCRF_CHECK_LAUNCH();
    std::vector<double> gw((size_t)nimg * nk, 0.0), sums;
    std::vector<StepBar> sb(nimg);
    for (int t = iters - 1; t >= 0; --t) {
        const T *yt = ys + (size_t)t * NL;
        const int32_t *sl = ss + (size_t)t * N;
        qp_apply(ctx, yt, mu, L, W.P.p);
        hipLaunchKernelGGL((k_onehot_d<T>), dim3(gE), dim3(256), 0, st, N, L, sl,
                           W.OH.as<T>());
        qp_apply(ctx, W.OH.p, mu, L, W.S.p);
        for (int m = 0; m < nk; ++m) filter_kernel(ctx, m, W.OH.p, W.Ks[m].p, L, false);
        hipLaunchKernelGGL((k_abar<T>), dim3(GD), dim3(kThreads), 0, st, seg, nimg,
                           L, ybar, yt, sl, Pbar, W.S.as<T>(), W.P.as<T>(),
                           W.part.as<double>());
        DCRF_CHECK_LAUNCH();
        image_sums(ctx, W.part.as<double>(), toff, 1, 1, sums);
        for (int j = 0; j < nimg; ++j) {
            const double *stt = stats.data() + ((size_t)t * nimg + j) * kFWStats;
            const double abar = sums[j], al = stt[0], a2 = stt[1];
            double b1bar = 0.0, a2bar = 0.0;
            if (stt[3] != 0.0) {
                b1bar = -abar / (2.0 * a2);
                a2bar = -abar * al / a2;
            }
            sb[j] = StepBar{al, -2.0 * b1bar + a2bar, b1bar - a2bar, b1bar - a2bar,
                            a2bar, -b1bar, b1bar};
        }
        DCRF_TRY_HIP(hipMemcpyAsync(W.sb.p, sb.data(), nimg * sizeof(StepBar),
                                    hipMemcpyHostToDevice, st));
        UpdArgs<T> U{};
        U.seg = seg;
        U.nimg = nimg;
        U.L = L;
        U.nk = nk;
        U.ybar = ybar;
        U.Pbar = Pbar;
        U.cbar = cbar;
        U.y = yt;
        U.P = W.P.as<T>();
        U.S = W.S.as<T>();
        U.c = W.c.as<T>();
        U.s = sl;
        for (int m = 0; m < nk; ++m) U.Ks[m] = W.Ks[m].as<T>();
        U.mu = mu;
        U.mabs = W.mabs.as<T>();
        U.rho = W.rho.as<double>();
        U.part = W.part.as<double>();
        U.sb = W.sb.as<StepBar>();
        hipLaunchKernelGGL((k_diff_update<T>), dim3(GD), dim3(kThreads), 0, st, U);
        DCRF_CHECK_LAUNCH();
        image_sums(ctx, W.part.as<double>(), toff, DCRF_MAXK, nk, sums);
        for (size_t i = 0; i < gw.size(); ++i) gw[i] += sums[i];
    }
    // the end of the sweep
    const T *y0 = ys;
    hipLaunchKernelGGL((k_rowmat<T>), dim3(std::min(4096, ceil_div(N, kThreads / L))),
                       dim3(kThreads), 0, st, N, L, Pbar, mu, W.Z.as<T>());
    filter_apply(ctx, W.Z.p, W.KtZ.p, L, true, false);
    hipLaunchKernelGGL((k_fill_d<T>), dim3(ceil_div(N, 256)), dim3(256), 0, st,
                       (size_t)N, W.ones.as<T>(), T(1));
    for (int m = 0; m < nk; ++m) {
        filter_kernel(ctx, m, y0, W.Ky0[m].p, L, false);
        filter_kernel(ctx, m, W.ones.p, W.K1[m].p, 1, false);
    }
    FinArgs<T> F{};
    F.seg = seg;
    F.nimg = nimg;
    F.L = L;
    F.nk = nk;
    F.ybar = ybar;
    F.KtZ = W.KtZ.as<T>();
    F.Z = W.Z.as<T>();
    F.Pbar = Pbar;
    F.y0 = y0;
    F.cbar = cbar;
    F.r = ctx->r.as<T>();
    F.mabs = W.mabs.as<T>();
    for (int m = 0; m < nk; ++m) {
        F.Ky0[m] = W.Ky0[m].as<T>();
        F.K1[m] = W.K1[m].as<T>();
    }
    F.rho = W.rho.as<double>();
    F.phibar = grad_phi;
    F.part = W.part.as<double>();
    hipLaunchKernelGGL((k_diff_final<T>), dim3(GD), dim3(kThreads), 0, st, F);
    DCRF_CHECK_LAUNCH();
    image_sums(ctx, W.part.as<double>(), toff, DCRF_MAXK, nk, sums);
    for (size_t i = 0; i < gw.size(); ++i) gw[i] += sums[i];
    if (grad_w)
        for (size_t i = 0; i < gw.size(); ++i) grad_w[i] = gw[i];
}

template <typename T>
void forward_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, T *y, int iters,
               char *saved) {
    const SavedLayout lay = saved_layout(ctx, L, iters);
    hipLaunchKernelGGL((k_softmax_neg<T>), dim3(seg_tiles(ctx, 256)), dim3(256),
                       0, ctx->stream, ctx->seg.as<int>(), ctx->nimg, L, phi, y);
    DCRF_CHECK_LAUNCH();
    FWCheckpoint cp{saved + lay.y, reinterpret_cast<int32_t *>(saved + lay.s),
                    reinterpret_cast<double *>(saved + lay.stats)};
    frank_wolfe_checkpointed(ctx, phi, mu, L, y, iters, cp);
}

}  // namespace

size_t fw_saved_bytes(dcrf_ctx *ctx, int L, int iters) {
    return saved_layout(ctx, L, iters).total;
}

void fw_diff_forward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                     void *y_out, int iters, void *saved) {
    if (ctx->dtype == DCRF_F64)
        forward_t<double>(ctx, static_cast<const double *>(unary),
                          static_cast<const double *>(mu), L,
                          static_cast<double *>(y_out), iters,
                          static_cast<char *>(saved));
    else
        forward_t<float>(ctx, static_cast<const float *>(unary),
                         static_cast<const float *>(mu), L,
                         static_cast<float *>(y_out), iters,
                         static_cast<char *>(saved));
}

void fw_diff_backward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                      int iters, const void *saved, const void *grad_y,
                      void *grad_unary, double *grad_w) {
    if (ctx->dtype == DCRF_F64)
        backward_t<double>(ctx, static_cast<const double *>(unary),
                           static_cast<const double *>(mu), L, iters,
                           static_cast<const char *>(saved),
                           static_cast<const double *>(grad_y),
                           static_cast<double *>(grad_unary), grad_w);
    else
        backward_t<float>(ctx, static_cast<const float *>(unary),
                          static_cast<const float *>(mu), L, iters,
                          static_cast<const char *>(saved),
                          static_cast<const float *>(grad_y),
                          static_cast<float *>(grad_unary), grad_w);
}

void diff_release(dcrf_ctx *ctx) {
    if (!ctx->diff) return;
    DiffWork *W = static_cast<DiffWork *>(ctx->diff);
    for (DevBuf *b : {&W->ybar, &W->Pbar, &W->cbar, &W->P, &W->S, &W->OH, &W->c,
                      &W->Z, &W->KtZ, &W->rho, &W->part, &W->mabs, &W->ones,
                      &W->sb})
        b->release();
    for (int m = 0; m < DCRF_MAXK; ++m) {
        W->Ks[m].release();
        W->Ky0[m].release();
        W->K1[m].release();
    }
    delete W;
    ctx->diff = nullptr;
}

}  // namespace dcrf
