// CCCP on the DC decomposition for negative semi-definite label
// compatibilities (Sec. 5.2, eq. QP-concave-CCCP; App. C,
// eq. convexpb-concavecccp and eq. convexpb-onevar).
//
// With Kbar = sum_m w_m K_m and K' = Kbar - wsum I (wsum = sum_m w_m),
//   S(y) = phi^T y + y^T (mu (x) K') y
//        = [phi^T y - wsum y^T (mu (x) I) y] + y^T (mu (x) Kbar) y,
// a convex part and a concave one when mu is negative semi-definite on the
// directions that keep every pixel on its simplex (Potts mu = [i != j] acts
// as -I there). A CCCP step replaces the concave part by its tangent at y^k,
// whose gradient 2 (Kbar Y^k) mu^T costs one filter call, and leaves one
// small convex problem per pixel:
//   min over the simplex of c_a^T y_a - wsum y_a^T mu y_a,
//   c_a = phi_a + 2 (Kbar Y^k)_a mu^T.
// For Potts y_a^T mu y_a = 1 - |y_a|^2 on the simplex, so the minimiser is
// the Euclidean projection of -c_a / (2 wsum) (the vertex of the smallest
// c_a(i) when wsum = 0); for another mu the step runs the paper's per-pixel
// Frank-Wolfe with its exact step, `inner` iterations from y^k.
//
// One step is splat(y^k), blur, then k_dcneg_rows: the slice gathers
// (K~ Y^k)_a (the lattice's Kbar Y), the block reads phi and y^k for its
// tile, every thread solves its pixel's problem in registers and writes
// y^{k+1} over y^k in place (a pixel's row is read and written by the same
// thread; the gathers read only vertex rows). The same pass adds up the
// partial sums of S(y^k) = phi^T y + y^T ((K~ Y - wsum Y) mu^T), one per
// pixel tile, so the objective history costs no extra pass except one final
// filter for S(y^outer).

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

template <typename T>
struct DCNegArgs {
    int L;
    T *y;               // y^k in, y^{k+1} out (update != 0)
    const T *phi;
    const T *mu;        // L x L (read only for a non-Potts mu)
    const T *pre;       // K'Y^k from the exact filter, or null (lattice)
    T wsum;
    int inner;          // per-pixel Frank-Wolfe iterations (non-Potts mu)
    int update;         // 0: only the partial sums of S(y^k)
    double *part;       // one partial sum of S(y^k) per tile
    const int *seg;
    int nimg;
};

// out = mu v for a register row v (L <= LMAX valid entries) and mu staged
// in LDS (row stride LMAX); v passes through the caller's own LDS row.
template <typename T, int LMAX>
__device__ __forceinline__ void mu_times(const T *smu, const T (&v)[LMAX], int L,
                                         T *row, T (&out)[LMAX]) {
#pragma unroll
    for (int j = 0; j < LMAX; ++j)
        if (j < L) row[j] = v[j];
#pragma unroll
    for (int i = 0; i < LMAX; ++i) out[i] = T(0);
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
        const T vj = row[j];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) out[i] += smu[i * LMAX + j] * vj;
    }
}

template <typename T, int LMAX, bool POTTS>
__global__ void __launch_bounds__(RowTile<T>::kPix, 2)
k_dcneg_rows(DCNegArgs<T> A, LatSet<T> ls) {
    constexpr int TP = RowTile<T>::kPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    __shared__ int32_t sid[TP * kCorners52];
    __shared__ T swc[TP * kCorners52];
    __shared__ T smu[POTTS ? 1 : LMAX * LMAX];
    __shared__ double red[TP / 64];
    const int L = A.L;
    if (!POTTS) {
        for (int i = threadIdx.x; i < L * L; i += TP)
            smu[(i / L) * LMAX + (i % L)] = A.mu[i];
        __syncthreads();
    }
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int lo, hi;
    tile_range(A.seg, A.nimg, TP, tile, lo, hi);
    const long long p0 = lo;
    const int np = hi - lo;
    const long long a = p0 + threadIdx.x;
    const bool act = (int)threadIdx.x < np;
    // q = (K~ Y^k)_a: the lattice's Kbar Y (the self-term is not removed)
    T q[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) q[j] = T(0);
    const bool staged = !A.pre && ls.shape52 && np > 0;   // uniform over the block
    if (A.pre) {
        tile_load<T, LMAX, TP>(A.pre, p0, np, L, lds, q);
    } else if (staged) {
        stage_corners52<T, TP>(ls, p0, np, sid, swc);
        __syncthreads();
        slice_tile52_coop<T, LMAX, TP>(ls, np, L, sid, swc, lds);
        __syncthreads();
        tile_read_own<T, LMAX>(np, L, lds, q);
        __syncthreads();
    } else if (act) {
        slice_pixel<T, LMAX>(ls, a, L, q);
    }
    T y[LMAX], ph[LMAX];
    tile_load<T, LMAX, TP>(A.y, p0, np, L, lds, y);
    tile_load<T, LMAX, TP>(A.phi, p0, np, L, lds, ph);
    T *row = lds + threadIdx.x * lds_stride(L);   // this thread's row from here on
    if (A.pre) {   // exact mode: K'Y given, Kbar Y = K'Y + wsum Y
#pragma unroll
        for (int j = 0; j < LMAX; ++j) q[j] += A.wsum * y[j];
    }
    // (Kbar Y) mu^T and Psi y = ((Kbar Y - wsum Y) mu^T)
    T qm[LMAX], py[LMAX];
    if (POTTS) {
        T tq = T(0), tp = T(0);
#pragma unroll
        for (int j = 0; j < LMAX; ++j)
            if (j < L) tq += q[j], tp += q[j] - A.wsum * y[j];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) {
            qm[i] = (i < L) ? tq - q[i] : T(0);
            py[i] = (i < L) ? tp - (q[i] - A.wsum * y[i]) : T(0);
        }
    } else {
        // general mu: the vector goes through this thread's own LDS row (free
        // after the tile loads) so that only the L accumulators stay live
        // across the loop over j
        mu_times<T, LMAX>(smu, q, L, row, qm);
#pragma unroll
        for (int j = 0; j < LMAX; ++j) q[j] -= A.wsum * y[j];
        mu_times<T, LMAX>(smu, q, L, row, py);
    }
    double acc[1] = {0.0};
    if (act)
#pragma unroll
        for (int i = 0; i < LMAX; ++i)
            if (i < L) acc[0] += double(ph[i]) * double(y[i]) + double(y[i]) * double(py[i]);
    if (A.update) {
        T c[LMAX];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) c[i] = (i < L) ? ph[i] + T(2) * qm[i] : T(0);
        T yn[LMAX];
        if (POTTS) {
            if (A.wsum > T(0)) {
                constexpr int P = Pow2<LMAX>::v;
                T v[P];
                const T sc = T(-0.5) / A.wsum;
#pragma unroll
                for (int i = 0; i < P; ++i) v[i] = (i < L) ? c[i] * sc : T(0);
                const T tau = simplex_tau<T, P>(v, L);
#pragma unroll
                for (int i = 0; i < LMAX; ++i) yn[i] = (i < L) ? fmax(v[i] - tau, T(0)) : T(0);
            } else {   // linear: the vertex of the smallest c (lowest label on ties)
                int best = 0;
                T bv = c[0];
#pragma unroll
                for (int i = 1; i < LMAX; ++i)
                    if (i < L && c[i] < bv) bv = c[i], best = i;
#pragma unroll
                for (int i = 0; i < LMAX; ++i) yn[i] = (i == best) ? T(1) : T(0);
            }
        } else {
            // per-pixel Frank-Wolfe on h(y) = c^T y - wsum y^T mu y
#pragma unroll
            for (int i = 0; i < LMAX; ++i) yn[i] = y[i];
            for (int it = 0; it < A.inner; ++it) {
                T my[LMAX];
                mu_times<T, LMAX>(smu, yn, L, row, my);
                int sl = 0;
                T gb = c[0] - T(2) * A.wsum * my[0];
#pragma unroll
                for (int i = 1; i < LMAX; ++i) {
                    const T g = c[i] - T(2) * A.wsum * my[i];
                    if (i < L && g < gb) gb = g, sl = i;
                }
                // d = e_s - y: b1 = c^T d - 2 wsum (mu y)^T d,
                // a2 = -wsum d^T mu d = -wsum (sum_i d_i mu_is - d^T mu y)
                T cd = T(0), myd = T(0), dms = T(0);
#pragma unroll
                for (int i = 0; i < LMAX; ++i) {
                    if (i < L) {
                        const T d = (i == sl ? T(1) : T(0)) - yn[i];
                        cd += c[i] * d;
                        myd += my[i] * d;
                        dms += d * smu[i * LMAX + sl];
                    }
                }
                const T b1 = cd - T(2) * A.wsum * myd;
                const T a2 = -A.wsum * (dms - myd);
                T al;
                if (a2 > T(0))
                    al = fmin(fmax(-b1 / (T(2) * a2), T(0)), T(1));
                else
                    al = (a2 + b1 < T(0)) ? T(1) : T(0);
#pragma unroll
                for (int i = 0; i < LMAX; ++i)
                    yn[i] += al * ((i == sl ? T(1) : T(0)) - yn[i]);
            }
        }
        tile_store<T, LMAX, TP>(A.y, p0, np, L, lds, yn);
    }
    const double tot = block_sum_waves<1, TP>(acc, red);
    if (threadIdx.x == 0) A.part[tile] = tot;
}

template <typename T, bool POTTS>
void launch_dcneg(dcrf_ctx *ctx, const DCNegArgs<T> &a, const LatSet<T> &ls, int G) {
    ProfScope ps(ctx, PROF_DCNEG);
    DCRF_DISPATCH_ROWS(a.L, DCRF_PLAUNCH(ps, (k_dcneg_rows<T, LMAX, POTTS>), dim3(G),
                                         dim3(RowTile<T>::kPix), 0, ctx->stream, a, ls));
    DCRF_CHECK_LAUNCH();
}

// Whether mu is Potts: known without a host read for the context's own copy.
template <typename T>
bool potts_mu(dcrf_ctx *ctx, const T *mu, int L) {
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
void dc_neg_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, T *y, int outer,
              int inner, double *S_hist) {
    if (L > kRowMaxC) fail(DCRF_EUNSUPPORTED, "DC_neg takes at most 32 labels");
    const hipStream_t st = ctx->stream;
    const int N = ctx->N;
    constexpr int TP = RowTile<T>::kPix;
    const int G = seg_tiles(ctx, TP);
    const bool exact = ctx->mode != DCRF_FILTER_LATTICE;   // a dense K'Y first
    const bool potts = potts_mu<T>(ctx, mu, L);
    // rows of partial sums: S(y^k) for k = 0..outer when asked, else one
    // scratch row that each step overwrites
    const int rows = S_hist ? outer + 1 : 1;
    ctx->hist.ensure((size_t)rows * G * 8, st);
    if (exact) ctx->tmpA.ensure((size_t)N * L * sizeof(T), st);
    else ensure_vertex_buffers(ctx, L);
    DCNegArgs<T> a{L, y, phi, mu, nullptr, T(ctx->wsum), inner, 1, nullptr,
                   ctx->seg.as<int>(), ctx->nimg};
    auto pass = [&](int k, int update) {
        LatSet<T> ls{};
        if (exact) {
            filter_apply(ctx, y, ctx->tmpA.p, L, false, ctx->mode);
            a.pre = ctx->tmpA.as<T>();
        } else {
            splat_dense(ctx, y, L);
            blur_all(ctx, L, false);
            ls = make_lat_set<T>(ctx, L);
        }
        a.update = update;
        a.part = ctx->hist.as<double>() + (size_t)(S_hist ? k : 0) * G;
        if (potts)
            launch_dcneg<T, true>(ctx, a, ls, G);
        else
            launch_dcneg<T, false>(ctx, a, ls, G);
    };
    for (int k = 0; k < outer; ++k) pass(k, 1);
    if (!S_hist) return;
    pass(outer, 0);   // S(y^outer): one more filter, no update
    std::vector<double> h((size_t)rows * G);
    DCRF_TRY_HIP(hipMemcpyAsync(h.data(), ctx->hist.p, h.size() * 8, hipMemcpyDeviceToHost,
                                st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < rows; ++k) {
        double v = 0.0;
        for (int i = 0; i < G; ++i) v += h[(size_t)k * G + i];
        S_hist[k] = v;
    }
}

}  // namespace

void dc_neg(dcrf_ctx *ctx, const void *unary, const void *mu, int L, void *y,
            int outer, int inner, double *S_hist) {
    if (ctx->dtype == DCRF_F64)
        dc_neg_t<double>(ctx, static_cast<const double *>(unary),
                         static_cast<const double *>(mu), L, static_cast<double *>(y),
                         outer, inner, S_hist);
    else
        dc_neg_t<float>(ctx, static_cast<const float *>(unary),
                        static_cast<const float *>(mu), L, static_cast<float *>(y), outer,
                        inner, S_hist);
}

}  // namespace dcrf
