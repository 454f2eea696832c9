// Reverse-mode derivative of a fixed number T of Frank-Wolfe iterations on the
// convex QP (Sec. 4, App. B), with respect to the unaries phi and the kernel
// weights w_m, for an upstream gradient dl/dy_T.
//
// Forward: y_0 = softmax(-phi), then T iterations of the Frank-Wolfe kernels,
// checkpointing y_t, P_t = Q y_t, the conditional gradient s_t, the step's
// quadratic (alpha_t, a2, b1, interior) and, per lattice, the blurred vertex
// values of y_0 and of every one-hot s_t (a few MB per iteration), so that
// the reverse sweep needs no filter of its own until its last step.
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
//   d<Zbar, Q X>/dw_m = <Zbar mu, (K~_m - I) X> + sum_a rho_a kappa_m(a),
//   rho_a = sum_i Zbar_a(i) X_a(i) sum_j |mu_ij|,  kappa_m = K~_m 1 - 1,
// with K~_m the lattice filter of kernel m alone.
//
// How it runs: per iteration, k_sweep_a slices K~_m s_t of every lattice
// from the saved vertex values, forms S_t = Q s_t, and reduces per tile the
// pieces of abar and of the weight gradient; since Sbar is linear in
// (alpha, Bbar, Dbar), <Sbar mu, (K~_m - I) s> and the rho terms split into
// three scalar products each; the blocks add their sums to per-image
// accumulators (one set per XCD, device atomics, alternating by iteration
// parity). Every block of k_sweep_b adds the sets up in a fixed order, turns
// the sums into the step's adjoints and updates ybar and Pbar; the image's
// first tile also accumulates the weight gradient. No host synchronisation
// and no launch of its own for the step happen inside the sweep. cbar is not carried per iteration: with the recurrence
// y_t = (1 - alpha_{t-1}) y_{t-1} + alpha_{t-1} s_{t-1},
//   sum_t cybar_t y_t = a_0 y_0 + sum_k b_k s_k,
//   a_0 = sum_t cybar_t prod_{u<t} (1 - alpha_u),
//   b_k = alpha_k sum_{t>k} cybar_t prod_{k<u<t} (1 - alpha_u),
// so the last kernel rebuilds cbar from y_0 and the saved labels.
//
// For a context that holds a batch of images every image has its own step
// sizes, step adjoints and weight gradient: the reductions are per tile of
// one image.

#include <algorithm>
#include <cmath>
#include <vector>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

constexpr int kThreads = 256;
constexpr int kNP = 1 + 3 * DCRF_MAXK;   // sums per image of k_sweep_a
constexpr int kSets = 8;                 // accumulator sets, one per XCD

// acc[parity][set][image][kNP], parity = iteration & 1
__device__ __forceinline__ size_t sweep_acc_off(int par, int set, int nimg, int img) {
    return (((size_t)par * kSets + set) * nimg + img) * kNP;
}

// y = softmax(-phi) row by row; rows move through LDS tiles (coalesced)
template <typename T, int LMAX>
__global__ void __launch_bounds__(RowTile<T>::kPix)
k_softmax_neg(const int *__restrict__ seg, int nimg, int L, const T *__restrict__ phi,
              T *__restrict__ y) {
    constexpr int TP = RowTile<T>::kPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    int lo, hi;
    tile_range(seg, nimg, TP, xcd_block(blockIdx.x, gridDim.x), lo, hi);
    const int np = hi - lo;
    T p[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) p[j] = T(0);
    tile_load<T, LMAX, TP>(phi, lo, np, L, lds, p);
    T mn = p[0];
#pragma unroll
    for (int j = 1; j < LMAX; ++j)
        if (j < L) mn = fmin(mn, p[j]);
    T sum = T(0);
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        p[j] = (j < L) ? exp(mn - p[j]) : T(0);
        sum += p[j];
    }
#pragma unroll
    for (int j = 0; j < LMAX; ++j) p[j] /= sum;
    tile_store<T, LMAX, TP>(y, lo, np, L, lds, p);
}

template <typename T>
__global__ void k_mabs(int L, const T *__restrict__ mu, T *__restrict__ mabs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    T s = T(0);
    for (int j = 0; j < L; ++j) s += fabs(mu[(size_t)i * L + j]);
    mabs[i] = s;
}

template <typename T>
__global__ void k_fill_d(size_t n, T *__restrict__ p, T v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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

// gamma_m times the slice of lattice m at pixel a (weight 1, no self term).
// For d = 5 and d = 2 the vertex ids and weights are loaded first and every
// row load is issued unconditionally (a missing vertex reads row 0 with
// weight 0), so that all of them are in flight together.
template <typename T, int LMAX, int D>
__device__ __forceinline__ void slice_fixed(const LatView<T> &Lt, T gam, size_t a, int C,
                                            T (&q)[LMAX]) {
    int id[D + 1];
    T w[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        const int v = Lt.vid[a * (D + 1) + k];
        w[k] = v >= 0 ? gam * Lt.w[a * (D + 1) + k] : T(0);
        id[k] = v >= 0 ? v : 0;
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) axpy_row<LMAX>(q, w[k], Lt.Vf + (size_t)id[k] * Lt.ld, C);
}

template <typename T, int LMAX>
__device__ __forceinline__ void slice_one(const LatView<T> &Lt, T gam, size_t a, int C,
                                          T (&q)[LMAX]) {
#pragma unroll
    for (int j = 0; j < LMAX; ++j) q[j] = T(0);
    if (Lt.d == 5) {
        slice_fixed<T, LMAX, 5>(Lt, gam, a, C, q);
    } else if (Lt.d == 2) {
        slice_fixed<T, LMAX, 2>(Lt, gam, a, C, q);
    } else {
        const int D1 = Lt.d + 1;
        for (int k = 0; k < D1; ++k) {
            const int id = Lt.vid[a * D1 + k];
            if (id >= 0)
                axpy_row<LMAX>(q, gam * Lt.w[a * D1 + k], Lt.Vf + (size_t)id * Lt.ld, C);
        }
    }
}

// out = mu R (out_k = sum_i mu_ki R_i); Potts: sum(R) - R_k
template <typename T, int LMAX, bool POTTS>
__device__ __forceinline__ void mu_apply(const T *smu, int C, const T (&R)[LMAX],
                                         T (&out)[LMAX]) {
    if (POTTS) {
        T tot = T(0);
#pragma unroll
        for (int i = 0; i < LMAX; ++i) tot += (i < C) ? R[i] : T(0);
#pragma unroll
        for (int k = 0; k < LMAX; ++k) out[k] = (k < C) ? tot - R[k] : T(0);
    } else {
#pragma unroll
        for (int k = 0; k < LMAX; ++k) {
            T acc = T(0);
#pragma unroll
            for (int i = 0; i < LMAX; ++i)
                if (k < C && i < C) acc += smu[k * LMAX + i] * R[i];
            out[k] = acc;
        }
    }
}

// out = R mu^T (out_i = sum_j mu_ij R_j); Potts: the same as mu R
template <typename T, int LMAX, bool POTTS>
__device__ __forceinline__ void mu_apply_t(const T *smu, int C, const T (&R)[LMAX],
                                           T (&out)[LMAX]) {
    if (POTTS) {
        mu_apply<T, LMAX, true>(smu, C, R, out);
    } else {
#pragma unroll
        for (int i = 0; i < LMAX; ++i) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < LMAX; ++j)
                if (i < C && j < C) acc += smu[i * LMAX + j] * R[j];
            out[i] = acc;
        }
    }
}

template <typename T>
struct SweepA {
    const int *seg;
    int nimg, L, nk, t;
    const int32_t *s;
    const T *y, *P, *ybar, *Pbar, *r, *mabs, *mu;
    const double *stats;          // the forward's step records
    const T *kappa1[DCRF_MAXK];   // K~_m 1
    T w[DCRF_MAXK], gam[DCRF_MAXK], wsum;
    T *S;
    double *acc;    // per image: abar, then per kernel U, V, W (see sweep_acc_off)
};

// Per pixel of one tile: S = Q s from the saved vertex values of the
// one-hot s, the abar terms, and per kernel the weight-gradient pieces
// U = alpha (X1 + Z1), V = X2 + Z2, W = X3 + Z3 with
//   X1 = <Pbar mu, R_m>, X2 = <y mu, R_m>, X3 = <s mu, R_m>, R_m = K~_m s - s,
//   Z1 = Pbar(s) |mu|_s kappa_m, Z2 = y(s) |mu|_s kappa_m, Z3 = |mu|_s kappa_m
// (the step's weight gradient is then U + Bbar V + Dbar W). The rows of y,
// Pbar, ybar and P pass through three LDS tiles, so that only the slice and
// a few sums live in registers.
template <typename T, int LMAX, bool POTTS>
__global__ void __launch_bounds__(RowTile<T>::kPix)
k_sweep_a(SweepA<T> A, LatSet<T> ls) {
    constexpr int TP = RowTile<T>::kPix;
    __shared__ __align__(16) T ty[TP * (LMAX | 1)];
    __shared__ __align__(16) T tp[TP * (LMAX | 1)];
    __shared__ __align__(16) T tq[TP * (LMAX | 1)];
    __shared__ T smu[POTTS ? 1 : LMAX * LMAX];
    __shared__ double red[kNP * (TP / 64)];
    const int L = A.L;
    const int Ls = lds_stride(L);
    if (!POTTS)
        for (int i = threadIdx.x; i < L * L; i += TP)
            smu[(i / L) * LMAX + (i % L)] = A.mu[i];
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int lo, hi;
    const int img = tile_range(A.seg, A.nimg, TP, tile, lo, hi);
    const int np = hi - lo;
    const size_t a = (size_t)lo + threadIdx.x;
    const bool act = (int)threadIdx.x < np;
    const double al = A.stats[((size_t)A.t * A.nimg + (img < 0 ? 0 : img)) * kFWStats];
    tile_copy_in<T, TP, LMAX>(A.y + (size_t)lo * L, np * L, L, ty);
    tile_copy_in<T, TP, LMAX>(A.Pbar + (size_t)lo * L, np * L, L, tp);
    __syncthreads();
    const T *yr = ty + threadIdx.x * Ls;
    const T *pr = tp + threadIdx.x * Ls;
    double acc[kNP];
#pragma unroll
    for (int i = 0; i < kNP; ++i) acc[i] = 0.0;
    T S[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) S[j] = T(0);
    const int sa = act ? A.s[a] : 0;
    if (act) {
        T ks[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) ks[j] = (j == sa) ? -A.wsum : T(0);
        const double pbs = pr[sa], ysa = yr[sa];
        double sum_pb = 0.0, sum_y = 0.0;
        if (POTTS)
            for (int k = 0; k < L; ++k) sum_pb += pr[k], sum_y += yr[k];
        const double ms = A.mabs[sa];
#pragma unroll
        for (int m = 0; m < DCRF_MAXK; ++m) {
            if (m >= A.nk) break;
            T q[LMAX];
            slice_one<T, LMAX>(ls.l[m], A.gam[m], a, L, q);
#pragma unroll
            for (int j = 0; j < LMAX; ++j) ks[j] += A.w[m] * q[j];
#pragma unroll
            for (int j = 0; j < LMAX; ++j)
                if (j == sa) q[j] -= T(1);
            double x1 = 0.0, x2 = 0.0, x3 = 0.0;
            if (POTTS) {
                // (v mu)_i = sum(v) - v_i
                double totR = 0.0, pR = 0.0, yR = 0.0, Rs = 0.0;
#pragma unroll
                for (int k = 0; k < LMAX; ++k) {
                    if (k < L) {
                        totR += double(q[k]);
                        pR += double(pr[k]) * double(q[k]);
                        yR += double(yr[k]) * double(q[k]);
                        if (k == sa) Rs = double(q[k]);
                    }
                }
                x1 = totR * sum_pb - pR;
                x2 = totR * sum_y - yR;
                x3 = totR - Rs;
            } else {
#pragma unroll
                for (int i = 0; i < LMAX; ++i) {
                    if (i < L) {
                        double pm = 0.0, ym = 0.0;
                        for (int k = 0; k < L; ++k) {
                            pm += double(pr[k]) * double(smu[k * LMAX + i]);
                            ym += double(yr[k]) * double(smu[k * LMAX + i]);
                        }
                        x1 += pm * double(q[i]);
                        x2 += ym * double(q[i]);
                        x3 += double(smu[sa * LMAX + i]) * double(q[i]);
                    }
                }
            }
            const double mk = ms * (double(A.kappa1[m][a]) - 1.0);
            acc[1 + 3 * m + 0] += al * (x1 + pbs * mk);
            acc[1 + 3 * m + 1] += x2 + ysa * mk;
            acc[1 + 3 * m + 2] += x3 + mk;
        }
        // S = (K's) mu^T + d * s
        mu_apply_t<T, LMAX, POTTS>(smu, L, ks, S);
        const T dself = A.mabs[sa] * A.r[a];
#pragma unroll
        for (int i = 0; i < LMAX; ++i)
            if (i == sa) S[i] += dself;
        // <Pbar, S>
#pragma unroll
        for (int k = 0; k < LMAX; ++k)
            if (k < L) acc[0] += double(pr[k]) * double(S[k]);
    }
    // <ybar, s - y>
    __syncthreads();
    tile_copy_in<T, TP, LMAX>(A.ybar + (size_t)lo * L, np * L, L, tq);
    __syncthreads();
    if (act) {
        const T *br = tq + threadIdx.x * Ls;
        double d = double(br[sa]);
        for (int k = 0; k < L; ++k) d -= double(br[k]) * double(yr[k]);
        acc[0] += d;
    }
    // -<Pbar, P>
    __syncthreads();
    tile_copy_in<T, TP, LMAX>(A.P + (size_t)lo * L, np * L, L, ty);
    __syncthreads();
    if (act) {
        double d = 0.0;
        for (int k = 0; k < L; ++k) d += double(pr[k]) * double(ty[threadIdx.x * Ls + k]);
        acc[0] -= d;
        T *out = tq + threadIdx.x * Ls;
#pragma unroll
        for (int k = 0; k < LMAX; ++k)
            if (k < L) out[k] = S[k];
    }
    __syncthreads();
    tile_copy_out<T, TP, LMAX>(A.S + (size_t)lo * L, np * L, L, tq);
    const double tot = block_sum_waves<kNP, TP>(acc, red);
    if (img >= 0 && (int)threadIdx.x < kNP)
        unsafeAtomicAdd(&A.acc[sweep_acc_off(A.t & 1, blockIdx.x & (kSets - 1), A.nimg, img) +
                               threadIdx.x], tot);
}

struct StepBar {
    double al, Abar, Bbar, Cbar, Dbar, cybar, csbar;
};

// The step's adjoints from the image's sums tot (k_sweep_a) and the
// checkpointed step quadratic: abar, then for an interior step
// b1bar = -abar / (2 a2), a2bar = -abar alpha / a2 (a clipped step passes no
// gradient), and the adjoints of A, B, C, D, cy, cs through b1 and a2.
__device__ __forceinline__ StepBar step_bar(const double *tot, const double *st) {
    const double abar = tot[0], al = st[0], a2 = st[1];
    double b1bar = 0.0, a2bar = 0.0;
    if (st[3] != 0.0) {
        b1bar = -abar / (2.0 * a2);
        a2bar = -abar * al / a2;
    }
    return StepBar{al, -2.0 * b1bar + a2bar, b1bar - a2bar, b1bar - a2bar, a2bar,
                   -b1bar, b1bar};
}

// Per block: the step adjoints of iteration t of its image from the
// accumulated sums (sets added in a fixed order); the image's first tile adds
// the step's weight gradient to gw and records (cybar, csbar); block 0 clears
// the other parity, which k_sweep_a of iteration t - 1 fills next. Then
// ybar <- (1 - alpha) ybar + Abar P + Bbar S + cybar c,
// Pbar <- (1 - alpha) Pbar + Abar y + Cbar s, with c = phi - |mu| r.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_sweep_b(const int *__restrict__ seg, int nimg, int L, int TPB,
          double *__restrict__ acc, const double *__restrict__ stats, int t, int nk,
          double *__restrict__ gw, double *__restrict__ coef,
          const int32_t *__restrict__ s,
          const T *__restrict__ y, const T *__restrict__ P, const T *__restrict__ S,
          const T *__restrict__ phi, const T *__restrict__ r, const T *__restrict__ mabs,
          T *__restrict__ ybar, T *__restrict__ Pbar) {
    __shared__ double stot[kNP];
    int lo, hi;
    const int img = tile_range(seg, nimg, TPB, xcd_block(blockIdx.x, gridDim.x), lo, hi);
    if (img >= 0 && (int)threadIdx.x < kNP) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < kSets; ++k) v += acc[sweep_acc_off(t & 1, k, nimg, img) + threadIdx.x];
        stot[threadIdx.x] = v;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kSets * nimg * kNP; i += kThreads)
            acc[sweep_acc_off((t + 1) & 1, 0, nimg, 0) + i] = 0.0;
    __syncthreads();
    if (img < 0) return;
    const StepBar b = step_bar(stot, stats + ((size_t)t * nimg + img) * kFWStats);
    if (threadIdx.x == 0 && lo == seg[2 * img]) {
        for (int m = 0; m < nk; ++m) {
            const double *x = stot + 1 + 3 * m;
            gw[(size_t)img * nk + m] += x[0] + b.Bbar * x[1] + b.Dbar * x[2];
        }
        coef[((size_t)t * nimg + img) * 2 + 0] = b.cybar;
        coef[((size_t)t * nimg + img) * 2 + 1] = b.csbar;
    }
    const T om = T(1.0 - b.al), Ab = T(b.Abar), Bb = T(b.Bbar), Cb = T(b.Cbar),
            cy = T(b.cybar);
    for (size_t e = (size_t)lo * L + threadIdx.x; e < (size_t)hi * L; e += kThreads) {
        const size_t a = e / L;
        const int i = int(e - a * L);
        const T c = phi[e] - mabs[i] * r[a];
        ybar[e] = om * ybar[e] + Ab * P[e] + Bb * S[e] + cy * c;
        Pbar[e] = om * Pbar[e] + Ab * y[e] + (i == s[a] ? Cb : T(0));
    }
}

template <typename T>
struct SweepF {
    const int *seg;
    int nimg, L, nk, iters;
    const T *ybar, *KtZ, *Pbar, *y0, *r, *mabs, *mu;
    const int32_t *s;          // iters x N saved labels
    const double *cb;          // per image: a_0, then b_k + csbar_k for k < iters
    const T *kappa1[DCRF_MAXK];
    T gam[DCRF_MAXK];
    T *phibar;
    double *part;              // per tile: nk sums
};

// The end of the sweep: P_0 = Q y_0 (ybar += K'^T (Pbar mu) + d Pbar and the
// weight terms with X = y_0), cbar rebuilt from y_0 and the labels, c = phi -
// d (its rho terms), and y_0 = softmax(-phi).
template <typename T, int LMAX, bool POTTS>
__global__ void __launch_bounds__(RowTile<T>::kPix)
k_sweep_final(SweepF<T> A, LatSet<T> ls) {
    constexpr int TP = RowTile<T>::kPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    __shared__ T smu[POTTS ? 1 : LMAX * LMAX];
    __shared__ double red[DCRF_MAXK * TP];
    const int L = A.L;
    if (!POTTS) {
        for (int i = threadIdx.x; i < L * L; i += TP)
            smu[(i / L) * LMAX + (i % L)] = A.mu[i];
        __syncthreads();
    }
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int lo, hi;
    const int img = tile_range(A.seg, A.nimg, TP, tile, lo, hi);
    const int np = hi - lo;
    const size_t a = (size_t)lo + threadIdx.x;
    const bool act = (int)threadIdx.x < np;
    const size_t N = (size_t)A.seg[2 * A.nimg - 1];
    double acc[DCRF_MAXK];
#pragma unroll
    for (int m = 0; m < DCRF_MAXK; ++m) acc[m] = 0.0;
    T y0[LMAX], pb[LMAX], g[LMAX], kz[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) y0[j] = pb[j] = g[j] = kz[j] = T(0);
    tile_load<T, LMAX, TP>(A.y0, lo, np, L, lds, y0);
    tile_load<T, LMAX, TP>(A.Pbar, lo, np, L, lds, pb);
    tile_load<T, LMAX, TP>(A.ybar, lo, np, L, lds, g);
    tile_load<T, LMAX, TP>(A.KtZ, lo, np, L, lds, kz);
    T out[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) out[j] = T(0);
    if (act) {
        const double *cb = A.cb + (size_t)(img < 0 ? 0 : img) * (A.iters + 1);
        const T ra = A.r[a];
        // cbar = a_0 y_0 + sum_k b_k s_k
        T cbar[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) cbar[j] = T(cb[0]) * y0[j];
        for (int k = 0; k < A.iters; ++k) {
            const int sk = A.s[(size_t)k * N + a];
            const T v = T(cb[1 + k]);
#pragma unroll
            for (int j = 0; j < LMAX; ++j)
                if (j == sk) cbar[j] += v;
        }
        // ybar_0, the rho terms of P_0 = Q y_0 and of c = phi - d, the
        // softmax backward
        double dot = 0.0, rho = 0.0;
#pragma unroll
        for (int j = 0; j < LMAX; ++j) {
            if (j < L) {
                g[j] = g[j] + kz[j] + A.mabs[j] * ra * pb[j];
                dot += double(g[j]) * double(y0[j]);
                rho += (double(pb[j]) * double(y0[j]) - double(cbar[j])) * double(A.mabs[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < LMAX; ++j)
            out[j] = (j < L) ? T(double(cbar[j]) - double(y0[j]) * (double(g[j]) - dot))
                             : T(0);
        for (int m = 0; m < A.nk; ++m) {
            T q[LMAX], t[LMAX];
            slice_one<T, LMAX>(ls.l[m], A.gam[m], a, L, q);
#pragma unroll
            for (int j = 0; j < LMAX; ++j) q[j] -= y0[j];
            mu_apply<T, LMAX, POTTS>(smu, L, q, t);
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < LMAX; ++k)
                if (k < L) x += double(pb[k]) * double(t[k]);
            acc[m] += x + rho * (double(A.kappa1[m][a]) - 1.0);
        }
    }
    tile_store<T, LMAX, TP>(A.phibar, lo, np, L, lds, out);
    block_sum<DCRF_MAXK, TP>(acc, red);
    if (threadIdx.x < DCRF_MAXK)
        A.part[(size_t)tile * DCRF_MAXK + threadIdx.x] = acc[threadIdx.x];
}

struct DiffWork {
    DevBuf ybar, Pbar, S, Z, KtZ, part, mabs, ones, acc, gw, coef, cb;
    DevBuf K1[DCRF_MAXK];
};

DiffWork &diff_work(dcrf_ctx *ctx) {
    if (!ctx->diff) ctx->diff = new DiffWork();
    return *static_cast<DiffWork *>(ctx->diff);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct SavedLayout {
    size_t y, P, s, V, vblock, stats, total;
};

SavedLayout saved_layout(dcrf_ctx *ctx, int L, int iters) {
    SavedLayout o;
    const size_t NL = (size_t)ctx->N * L;
    const size_t e = ctx->elt();
    o.vblock = 0;
    for (int m = 0; m < ctx->nk; ++m)
        o.vblock += (size_t)ctx->lat[m].M * row_stride(L, e);
    o.y = 0;
    o.P = align256(o.y + (size_t)iters * NL * e);
    o.s = align256(o.P + (size_t)iters * NL * e);
    o.V = align256(o.s + (size_t)iters * ctx->N * 4);
    o.stats = align256(o.V + (size_t)(iters + 1) * o.vblock * e);
    o.total = align256(o.stats + (size_t)iters * ctx->nimg * kFWStats * 8);
    return o;
}

// the lattices of the context with their blurred values taken from a saved
// block of vertex values
template <typename T>
LatSet<T> saved_lat_set(dcrf_ctx *ctx, int L, const T *block) {
    LatSet<T> ls = make_lat_set<T>(ctx, L);
    const T *p = block;
    for (int m = 0; m < ctx->nk; ++m) {
        ls.l[m].Vf = p;
        p += (size_t)ctx->lat[m].M * ls.l[m].ld;
    }
    ls.shape52 = 0;
    return ls;
}

// whether mu is the Potts compatibility (read once per call)
template <typename T>
bool mu_is_potts(dcrf_ctx *ctx, const T *mu, int L) {
    if (is_internal_potts(ctx, mu)) return true;
    std::vector<T> h((size_t)L * L);
    DCRF_TRY_HIP(hipMemcpyAsync(h.data(), mu, h.size() * sizeof(T), hipMemcpyDeviceToHost,
                                ctx->stream));
    DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j)
            if (h[(size_t)i * L + j] != T(i != j ? 1 : 0)) return false;
    return true;
}

template <typename T>
void backward_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, int iters,
                const char *saved, const T *grad_y, T *grad_phi, double *grad_w) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N, nk = ctx->nk, nimg = ctx->nimg;
    const int *seg = ctx->seg.as<int>();
    const size_t NL = (size_t)N * L;
    const size_t B = NL * sizeof(T);
    constexpr int TP = RowTile<T>::kPix;
    const int GA = seg_tiles(ctx, TP);
    constexpr int TPB = 256;   // pixels per block of k_sweep_b
    const int GB = seg_tiles(ctx, TPB);
    DiffWork &W = diff_work(ctx);
    for (DevBuf *b : {&W.ybar, &W.Pbar, &W.S, &W.Z, &W.KtZ}) b->ensure(B, st);
    for (int m = 0; m < nk; ++m) W.K1[m].ensure((size_t)N * sizeof(T), st);
    W.part.ensure((size_t)GA * kNP * 8, st);
    W.mabs.ensure((size_t)L * sizeof(T), st);
    W.ones.ensure((size_t)N * sizeof(T), st);
    W.acc.ensure((size_t)2 * kSets * nimg * kNP * 8, st);
    W.gw.ensure((size_t)nimg * nk * 8, st);
    W.coef.ensure((size_t)iters * nimg * 2 * 8, st);
    W.cb.ensure((size_t)nimg * (iters + 1) * 8, st);
    const SavedLayout lay = saved_layout(ctx, L, iters);
    const T *ys = reinterpret_cast<const T *>(saved + lay.y);
    const T *Ps = reinterpret_cast<const T *>(saved + lay.P);
    const int32_t *ss = reinterpret_cast<const int32_t *>(saved + lay.s);
    const T *Vs = reinterpret_cast<const T *>(saved + lay.V);
    const double *stats = reinterpret_cast<const double *>(saved + lay.stats);
    const bool potts = mu_is_potts<T>(ctx, mu, L);
    T *ybar = W.ybar.as<T>(), *Pbar = W.Pbar.as<T>();
    DCRF_TRY_HIP(hipMemcpyAsync(ybar, grad_y, B, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL((k_fill_d<T>), dim3(ceil_div((long long)NL, 256)), dim3(256), 0, st,
                       NL, Pbar, T(0));
    hipLaunchKernelGGL((k_fill_d<double>), dim3(1), dim3(256), 0, st,
                       (size_t)nimg * nk, W.gw.as<double>(), 0.0);
    hipLaunchKernelGGL((k_mabs<T>), dim3(1), dim3(256), 0, st, L, mu, W.mabs.as<T>());
    // kappa_m + 1 = K~_m 1
    hipLaunchKernelGGL((k_fill_d<T>), dim3(ceil_div(N, 256)), dim3(256), 0, st,
                       (size_t)N, W.ones.as<T>(), T(1));
    for (int m = 0; m < nk; ++m) filter_kernel(ctx, m, W.ones.p, W.K1[m].p, 1, false);
    DCRF_CHECK_LAUNCH();

    SweepA<T> A{};
    A.seg = seg;
    A.nimg = nimg;
    A.L = L;
    A.nk = nk;
    A.ybar = ybar;
    A.Pbar = Pbar;
    A.r = ctx->r.as<T>();
    A.mabs = W.mabs.as<T>();
    A.mu = mu;
    A.wsum = T(ctx->wsum);
    for (int m = 0; m < nk; ++m) {
        A.kappa1[m] = W.K1[m].as<T>();
        A.w[m] = T(ctx->kern[m].weight);
        A.gam[m] = T(ctx->lat[m].gamma);
    }
    A.S = W.S.as<T>();
    A.acc = W.acc.as<double>();
    A.stats = stats;
    DCRF_TRY_HIP(hipMemsetAsync(A.acc, 0, (size_t)2 * kSets * nimg * kNP * 8, st));
    for (int t = iters - 1; t >= 0; --t) {
        A.t = t;
        A.s = ss + (size_t)t * N;
        A.y = ys + (size_t)t * NL;
        A.P = Ps + (size_t)t * NL;
        const LatSet<T> ls = saved_lat_set<T>(ctx, L, Vs + (size_t)(t + 1) * lay.vblock);
        if (potts)
            DCRF_DISPATCH_ROWS(L, hipLaunchKernelGGL((k_sweep_a<T, LMAX, true>), dim3(GA),
                                                     dim3(TP), 0, st, A, ls));
        else
            DCRF_DISPATCH_ROWS(L, hipLaunchKernelGGL((k_sweep_a<T, LMAX, false>), dim3(GA),
                                                     dim3(TP), 0, st, A, ls));
        hipLaunchKernelGGL((k_sweep_b<T>), dim3(GB), dim3(kThreads), 0, st, seg, nimg, L,
                           TPB, A.acc, stats, t, nk, W.gw.as<double>(),
                           W.coef.as<double>(), A.s, A.y, A.P, W.S.as<T>(), phi,
                           ctx->r.as<T>(), W.mabs.as<T>(), ybar, Pbar);
        DCRF_CHECK_LAUNCH();
    }
    // coefficients of cbar = a_0 y_0 + sum_k (b_k + csbar_k) s_k, per image
    std::vector<double> coef((size_t)iters * nimg * 2), sth((size_t)iters * nimg * kFWStats);
    DCRF_TRY_HIP(hipMemcpyAsync(coef.data(), W.coef.p, coef.size() * 8,
                                hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipMemcpyAsync(sth.data(), stats, sth.size() * 8, hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    std::vector<double> cb((size_t)nimg * (iters + 1));
    for (int j = 0; j < nimg; ++j) {
        auto al = [&](int t) { return sth[((size_t)t * nimg + j) * kFWStats]; };
        auto cy = [&](int t) { return coef[((size_t)t * nimg + j) * 2 + 0]; };
        auto cs = [&](int t) { return coef[((size_t)t * nimg + j) * 2 + 1]; };
        // tail = sum_{t>k} cybar_t prod_{k<u<t} (1 - alpha_u), built from the
        // last iteration backwards; at the end it is a_0
        double tail = 0.0;
        for (int k = iters - 1; k >= 0; --k) {
            cb[(size_t)j * (iters + 1) + 1 + k] = al(k) * tail + cs(k);
            tail = cy(k) + (1.0 - al(k)) * tail;
        }
        cb[(size_t)j * (iters + 1)] = tail;
    }
    DCRF_TRY_HIP(hipMemcpyAsync(W.cb.p, cb.data(), cb.size() * 8, hipMemcpyHostToDevice, st));
    // the end of the sweep: ybar += K'^T (Pbar mu) + d Pbar and the rest
    hipLaunchKernelGGL((k_rowmat<T>), dim3(std::min(4096, ceil_div(N, kThreads / L))),
                       dim3(kThreads), 0, st, N, L, Pbar, mu, W.Z.as<T>());
    filter_apply(ctx, W.Z.p, W.KtZ.p, L, true, DCRF_FILTER_LATTICE);
    SweepF<T> F{};
    F.seg = seg;
    F.nimg = nimg;
    F.L = L;
    F.nk = nk;
    F.iters = iters;
    F.ybar = ybar;
    F.KtZ = W.KtZ.as<T>();
    F.Pbar = Pbar;
    F.y0 = ys;
    F.r = ctx->r.as<T>();
    F.mabs = W.mabs.as<T>();
    F.mu = mu;
    F.s = ss;
    F.cb = W.cb.as<double>();
    for (int m = 0; m < nk; ++m) {
        F.kappa1[m] = W.K1[m].as<T>();
        F.gam[m] = T(ctx->lat[m].gamma);
    }
    F.phibar = grad_phi;
    F.part = W.part.as<double>();
    const LatSet<T> ls0 = saved_lat_set<T>(ctx, L, Vs);
    if (potts)
        DCRF_DISPATCH_ROWS(L, hipLaunchKernelGGL((k_sweep_final<T, LMAX, true>), dim3(GA),
                                                 dim3(TP), 0, st, F, ls0));
    else
        DCRF_DISPATCH_ROWS(L, hipLaunchKernelGGL((k_sweep_final<T, LMAX, false>), dim3(GA),
                                                 dim3(TP), 0, st, F, ls0));
    DCRF_CHECK_LAUNCH();
    std::vector<double> part((size_t)GA * DCRF_MAXK), gw((size_t)nimg * nk);
    DCRF_TRY_HIP(hipMemcpyAsync(part.data(), W.part.p, part.size() * 8,
                                hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipMemcpyAsync(gw.data(), W.gw.p, gw.size() * 8, hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    const std::vector<int> toff = seg_tile_offsets(ctx, TP);
    for (int j = 0; j < nimg; ++j)
        for (int t = toff[j]; t < toff[j + 1]; ++t)
            for (int m = 0; m < nk; ++m)
                gw[(size_t)j * nk + m] += part[(size_t)t * DCRF_MAXK + m];
    if (grad_w)
        for (size_t i = 0; i < gw.size(); ++i) grad_w[i] = gw[i];
}

template <typename T>
void forward_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, T *y, int iters,
               char *saved) {
    const SavedLayout lay = saved_layout(ctx, L, iters);
    constexpr int TP = RowTile<T>::kPix;
    DCRF_DISPATCH_ROWS(L, hipLaunchKernelGGL((k_softmax_neg<T, LMAX>),
                                             dim3(seg_tiles(ctx, TP)), dim3(TP), 0,
                                             ctx->stream, ctx->seg.as<int>(), ctx->nimg,
                                             L, phi, y));
    DCRF_CHECK_LAUNCH();
    FWCheckpoint cp{saved + lay.y, saved + lay.P, reinterpret_cast<int32_t *>(saved + lay.s),
                    saved + lay.V, reinterpret_cast<double *>(saved + lay.stats)};
    frank_wolfe_checkpointed(ctx, phi, mu, L, y, iters, cp);
}

}  // namespace

size_t fw_saved_bytes(dcrf_ctx *ctx, int L, int iters) {
    return saved_layout(ctx, L, iters).total;
}

void fw_diff_forward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                     void *y_out, int iters, void *saved) {
    if (L > kRowMaxC)
        fail(DCRF_EUNSUPPORTED, "differentiation serves at most 32 labels");
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
    if (L > kRowMaxC)
        fail(DCRF_EUNSUPPORTED, "differentiation serves at most 32 labels");
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
    for (DevBuf *b : {&W->ybar, &W->Pbar, &W->S, &W->Z, &W->KtZ, &W->part, &W->mabs,
                      &W->ones, &W->acc, &W->gw, &W->coef, &W->cb})
        b->release();
    for (int m = 0; m < DCRF_MAXK; ++m) W->K1[m].release();
    delete W;
    ctx->diff = nullptr;
}

}  // namespace dcrf
