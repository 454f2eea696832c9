// Solvers on top of the pairwise filter.
//
// Frank-Wolfe on the convex QP relaxation (Sec. 4, Alg. fw, App. B):
//   f(y) = c^T y + y^T (Psi + D) y over the product of simplices,
//   c = phi - d (eq. cvx-qp-min) or, inside CCCP, phi - 2 d * y^k
//   (eq. cccp-qp), with (Psi y)_a(i) = sum_j mu_ij (K'Y)_a(j) and
//   d_a(i) = (sum_j |mu_ij|) (K'1)_a (eq. pairwise-matrix, eq. RL-diagonal).
// One iteration is five kinds of launch, with no host synchronisation:
//   1. k_fw_lmo: apply the previous step (y <- y + alpha (s - y) and
//      P_y <- (1 - alpha) P_y + alpha P_s, App. B's recurrence), form the
//      gradient g = c + 2 P_y (eq. LRQP-grad), take the conditional gradient
//      s_a = argmin_i g_a(i) (eq. LRQP-lp, lowest label on ties), and reduce
//      <y,P_y>, <s,P_y>, <c,y>, <c,s>, <g,y>, <g,s> per block;
//   2. the gather splat of the one-hot s into the lattices;
//   3. the blur passes;
//   4. k_fw_slice: slice, apply mu and the diagonal, P_s = (Psi + D) s,
//      reduce <y,P_s> and <s,P_s> per block.
// The blocks of steps 1 and 4 add their sums to per-image accumulators, one
// set per XCD (device atomics), and every block of the next iteration's step
// 1 (or k_fw_final after the last) adds the sets up in a fixed order and
// solves the step size itself (App. B, eq. alpha-opt, written with the four
// products so that it is exact for a non-symmetric approximate Psi;
// endpoints when the quadratic is not convex): no launch of its own and no
// host synchronisation. The accumulators alternate by iteration parity; the
// first block of step 4 clears the parity that is no longer read.
// The per-pixel kernels run one block per tile of one image, so a context
// that holds a batch of images (concatenated lattices, see batch.hip) solves
// every image's QP, each with its own step size, in the same launches.
// Up to 32 labels the per-pixel kernels keep a pixel's labels in registers
// (one thread per pixel, rows staged through LDS); above that one lane per
// (pixel, label). Dot products accumulate in FP64.

#include <algorithm>
#include <vector>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {

void slice_into(dcrf_ctx *ctx, const void *Y, const void *pre, int C,
                const void *mu, const void *mabs, void *out, bool qp);

namespace {

constexpr int kThreads = 256;
constexpr int kMaxGrid = 2048;
// pixel groups per block of the flat (one lane per label) kernels
constexpr int kFlatGroups = 8;
constexpr int kP1 = 8;   // partial sums written by k_fw_lmo
constexpr int kP2 = 2;   // partial sums written by k_fw_slice

// fw_scal holds the step-size accumulators (acc_off below)
// doubles per iteration in a forward checkpoint: alpha, a2, b1, interior
constexpr int kStats = 4;
constexpr int kPT = kP1 + kP2;   // sums per image and iteration
constexpr int kSets = 8;         // accumulator sets, one per XCD

// acc[parity][set][image][kPT], parity = iteration & 1
__device__ __forceinline__ size_t acc_off(int par, int set, int nimg, int img) {
    return (((size_t)par * kSets + set) * nimg + img) * kPT;
}

// sum i of image img of the iteration with parity par, sets in a fixed order
__device__ __forceinline__ double acc_total(const double *acc, int par, int nimg,
                                            int img, int i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kSets; ++k) s += acc[acc_off(par, k, nimg, img) + i];
    return s;
}

// exact line search from the sums (App. B): f(y + alpha D) = f(y) + alpha b1
// + alpha^2 a2 over [0, 1]
__device__ __forceinline__ double fw_line_search(const double *tot, double &a2,
                                                 double &b1) {
    const double Ayy = tot[0], Csy = tot[1], cy = tot[2], cs = tot[3];
    const double Bys = tot[kP1 + 0], Dss = tot[kP1 + 1];
    b1 = cs - cy + Bys + Csy - 2.0 * Ayy;
    a2 = Dss - Bys - Csy + Ayy;
    if (a2 > 0.0) return fmin(fmax(-b1 / (2.0 * a2), 0.0), 1.0);
    return (a2 + b1 < 0.0) ? 1.0 : 0.0;
}

// trace entry (f(y_t), gap, alpha, labels changed) and checkpoint entry of
// iteration it of image img
__device__ __forceinline__ void fw_record(const double *tot, double alpha, double a2,
                                          double b1, double *trace, double *stats,
                                          int it, int nimg, int img) {
    double *tr = trace + ((size_t)it * nimg + img) * 4;
    tr[0] = tot[2] + tot[0];   // <c, y> + <y, P_y>
    tr[1] = tot[4] - tot[5];   // <g, y - s>
    tr[2] = alpha;
    tr[3] = tot[6];
    if (stats) {   // checkpoint for the reverse sweep
        double *st = stats + ((size_t)it * nimg + img) * kStats;
        st[0] = alpha;
        st[1] = a2;
        st[2] = b1;
        st[3] = (a2 > 0.0 && -b1 / (2.0 * a2) > 0.0 && -b1 / (2.0 * a2) < 1.0) ? 1.0 : 0.0;
    }
}

// Step size of iteration it of image img (< 0: none) for every thread of the
// block; all threads call it. `mine` is this thread's sum when below kPT
// (loaded earlier, so that its latency overlaps other loads); the sums meet in
// LDS `stot`. If `record`, thread 0 writes the trace and checkpoint entries.
__device__ __forceinline__ double fw_block_step(double mine, int it, int nimg, int img,
                                                bool record, double *trace,
                                                double *stats, double *stot) {
    if ((int)threadIdx.x < kPT) stot[threadIdx.x] = mine;
    __syncthreads();
    if (img < 0) return 0.0;
    double a2, b1;
    const double alpha = fw_line_search(stot, a2, b1);
    if (record && threadIdx.x == 0) fw_record(stot, alpha, a2, b1, trace, stats, it, nimg, img);
    return alpha;
}

__device__ __forceinline__ double fw_load_sum(const double *acc, int it, int nimg,
                                              int img) {
    return (img >= 0 && (int)threadIdx.x < kPT)
               ? acc_total(acc, it & 1, nimg, img, threadIdx.x) : 0.0;
}

template <typename T>
__global__ void k_fill(T *p, size_t n, T v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// mabs[i] = sum_j |mu_ij|
template <typename T>
__global__ void k_mu_abs(int L, const T *__restrict__ mu, T *__restrict__ mabs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    T s = T(0);
    for (int j = 0; j < L; ++j) s += fabs(mu[(size_t)i * L + j]);
    mabs[i] = s;
}

// c = phi - scale * d * z, d_a(i) = mabs_i r_a; z = 1 when y == nullptr
template <typename T>
__global__ void k_linear_term(int N, int L, const T *__restrict__ phi,
                              const T *__restrict__ r, const T *__restrict__ mabs,
                              const T *__restrict__ y, T scale, T *__restrict__ c) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * L) return;
    const int a = int(e / L);
    const int i = int(e - (size_t)a * L);
    const T z = y ? y[e] : T(1);
    c[e] = phi[e] - scale * mabs[i] * r[a] * z;
}

template <typename T>
struct FWArgs {
    int N, L;
    T *y, *Py;
    const T *Ps, *c;
    int32_t *s;
    const int32_t *sprev;
    double *acc;              // accumulated sums, see acc_off
    double *trace, *stats;    // entries of the previous iteration (stats may be null)
    int it, first;
    const int *seg;   // image segments, one block per tile of an image
    int nimg;
    T *ysave, *Psave;   // checkpoint slots of y_t and P_t, or null
    int32_t *ssave;     // checkpoint slot of s_t, or null
};

template <typename T>
struct FWSliceArgs {
    int N, L;
    const T *y;
    const int32_t *s;
    T *Ps;
    const T *mu, *mabs, *r, *pre;
    T wsum;
    double *acc;   // accumulated sums, see acc_off
    int it;
    const int *seg;
    int nimg;
};

// ---------------------------------------------------------- row kernels

// Step 1, one thread per pixel (see the file comment).
// Pixels per block of k_fw_lmo_rows: one staged tile at a time keeps the LDS
// footprint small, so more blocks fit on a CU to hide memory latency.
template <typename T> struct LmoTile;
template <> struct LmoTile<float> { static constexpr int kPix = 256; };
template <> struct LmoTile<double> { static constexpr int kPix = 128; };

// SPLAT: the kernel also splats the one-hot s into the lattices (step 2),
// pixel-major: 1 for any lattice set, 2 for a 5-D + 2-D pair (corners loaded
// at the start, so that their latency overlaps the tiles').
// One tile of TP pixels (a block of TP threads); lds holds TP (LMAX | 1)
// values, red kP1 TP / 64 doubles, stot kPT doubles.
template <typename T, int LMAX, int SPLAT, int TP>
__device__ __forceinline__ void fw_lmo_tile(const FWArgs<T> &A, const LatSet<T> &ls,
                                            int tile, T *lds, double *red, double *stot) {
    const int L = A.L;
    int lo, hi;
    const int img = tile_range(A.seg, A.nimg, TP, tile, lo, hi);
    // the previous step's sums, loaded now so that they arrive with the tiles
    const double mine = A.first ? 0.0 : fw_load_sum(A.acc, A.it - 1, A.nimg, img);
    double acc[kP1];
#pragma unroll
    for (int i = 0; i < kP1; ++i) acc[i] = 0.0;
    {
        const long long p0 = lo;
        const int np = hi - lo;
        const long long a = p0 + threadIdx.x;
        const bool act = (int)threadIdx.x < np;
        Corners52<T> cn;
        if (SPLAT == 2) load_corners52<T>(ls, a, act, cn);
        T y[LMAX], py[LMAX], c[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) y[j] = py[j] = c[j] = T(0);
        tile_load<T, LMAX, TP>(A.y, p0, np, L, lds, y);
        tile_load<T, LMAX, TP>(A.Py, p0, np, L, lds, py);
        const int sp = act ? A.sprev[a] : -1;
        if (!A.first) {
            const T al = T(fw_block_step(mine, A.it - 1, A.nimg, img,
                                         img >= 0 && lo == A.seg[2 * img], A.trace,
                                         A.stats, stot));
            T ps[LMAX];
#pragma unroll
            for (int j = 0; j < LMAX; ++j) ps[j] = T(0);
            tile_load<T, LMAX, TP>(A.Ps, p0, np, L, lds, ps);
#pragma unroll
            for (int j = 0; j < LMAX; ++j) {
                y[j] = y[j] + al * (T(j == sp ? 1 : 0) - y[j]);
                py[j] = (T(1) - al) * py[j] + al * ps[j];
            }
            tile_store<T, LMAX, TP>(A.y, p0, np, L, lds, y);
            tile_store<T, LMAX, TP>(A.Py, p0, np, L, lds, py);
        }
        if (A.ysave) {
            tile_store<T, LMAX, TP>(A.ysave, p0, np, L, lds, y);
            tile_store<T, LMAX, TP>(A.Psave, p0, np, L, lds, py);
        }
        tile_load<T, LMAX, TP>(A.c, p0, np, L, lds, c);
        int lab = -1;
        if (act) {
            int best = 0;
            T bv = c[0] + T(2) * py[0];
#pragma unroll
            for (int j = 1; j < LMAX; ++j) {
                const T g = c[j] + T(2) * py[j];
                if (j < L && g < bv) {
                    bv = g;
                    best = j;
                }
            }
            A.s[a] = best;
            lab = best;
            if (A.ssave) A.ssave[a] = best;
            acc[6] += (best != sp) ? 1.0 : 0.0;
#pragma unroll
            for (int j = 0; j < LMAX; ++j) {
                if (j < L) {
                    const double yv = y[j], pv = py[j], cv = c[j];
                    const double gv = double(c[j] + T(2) * py[j]);
                    acc[0] += yv * pv;
                    acc[2] += cv * yv;
                    acc[4] += gv * yv;
                    if (j == best) {
                        acc[1] += pv;
                        acc[3] += cv;
                        acc[5] += gv;
                    }
                }
            }
        }
        if (SPLAT == 2) splat_onehot52<T>(ls, cn, lab);
        if (SPLAT == 1) splat_onehot<T>(ls, a, act, lab);
    }
    const double tot = block_sum_waves<kP1, TP>(acc, red);
    if (img >= 0 && threadIdx.x < kP1)
        unsafeAtomicAdd(&A.acc[acc_off(A.it & 1, tile & (kSets - 1), A.nimg, img) +
                               threadIdx.x], tot);
}

template <typename T, int LMAX, int SPLAT>
__global__ void __launch_bounds__(LmoTile<T>::kPix)
k_fw_lmo_rows(FWArgs<T> A, LatSet<T> ls) {
    constexpr int TP = LmoTile<T>::kPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    __shared__ double red[kP1 * (TP / 64)];
    __shared__ double stot[kPT];
    fw_lmo_tile<T, LMAX, SPLAT, TP>(A, ls, xcd_block(blockIdx.x, gridDim.x), lds, red, stot);
}

// Step 4, one thread per pixel (see the file comment). POTTS: mu = 1 - I,
// so (Q mu^T)_i = sum_j Q_j - Q_i.
// One tile of TP pixels (a block of TP threads); lds holds TP (LMAX | 1)
// values, sid and swc TP kCorners52 each, smu LMAX^2 (general mu), red
// kP2 TP / 64 doubles.
template <typename T, int LMAX, bool POTTS, int TP>
__device__ __forceinline__ void fw_slice_tile(const FWSliceArgs<T> &A, const LatSet<T> &ls,
                                              int tile, T *lds, int32_t *sid, T *swc,
                                              T *smu, double *red) {
    const int L = A.L;
    if (!POTTS) {
        for (int i = threadIdx.x; i < L * L; i += TP)
            smu[(i / L) * LMAX + (i % L)] = A.mu[i];
        __syncthreads();
    }
    double acc[kP2] = {0.0, 0.0};
    int lo, hi;
    const int img = tile_range(A.seg, A.nimg, TP, tile, lo, hi);
    {
        const long long p0 = lo;
        const int np = hi - lo;
        const long long a = p0 + threadIdx.x;
        const bool act = (int)threadIdx.x < np;
        T q[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) q[j] = T(0);
        const int sa = act ? A.s[a] : 0;
        // with Potts and no precomputed K'S the tile of y goes to LDS first,
        // so that its loads overlap the gathers of the slice
        const bool staged = !A.pre && ls.shape52 && np > 0;   // uniform over the block
        const bool early = POTTS && !A.pre && !staged;
        // staged: the tile of y is fetched into registers with the corners,
        // so that its loads overlap theirs and the gathers of the slice
        TileRegs<T, TP, LMAX> fy;
        if (staged) {
            tile_fetch<T, TP, LMAX>(A.y + p0 * L, np * L, L, fy);
            stage_corners52<T, TP>(ls, p0, np, sid, swc);
        }
        if (early) tile_copy_in<T, TP, LMAX>(A.y + p0 * L, np * L, L, lds);
        if (A.pre) {
            tile_load<T, LMAX, TP>(A.pre, p0, np, L, lds, q);
        } else {
            if (staged) {
                __syncthreads();
                slice_tile52_coop<T, LMAX, TP>(ls, np, L, sid, swc, lds);
                __syncthreads();
            }
            if (act) {
                if (staged)
                    tile_read_own<T, LMAX>(np, L, lds, q);
                else
                    slice_pixel<T, LMAX>(ls, a, L, q);
#pragma unroll
                for (int j = 0; j < LMAX; ++j)
                    if (j == sa) q[j] -= A.wsum;
            }
        }
        if (staged) __syncthreads();   // every row of the slice read: lds is reused
        T P[LMAX];
        const T dself = act ? A.mabs[sa] * A.r[a] : T(0);
        if (POTTS) {
            T tot = T(0);
#pragma unroll
            for (int j = 0; j < LMAX; ++j) tot += (j < L) ? q[j] : T(0);
#pragma unroll
            for (int i = 0; i < LMAX; ++i)
                P[i] = (i < L) ? (tot - q[i]) + (i == sa ? dself : T(0)) : T(0);
        } else {
            // general mu: q goes through this thread's own LDS row so that
            // only the L accumulators stay live across the j loop
            const int Ls = lds_stride(L);
            T *qrow = lds + threadIdx.x * Ls;
#pragma unroll
            for (int j = 0; j < LMAX; ++j)
                if (j < L) qrow[j] = q[j];
#pragma unroll
            for (int i = 0; i < LMAX; ++i) P[i] = T(0);
            for (int j = 0; j < L; ++j) {
                const T qj = qrow[j];
#pragma unroll
                for (int i = 0; i < LMAX; ++i) P[i] += smu[i * LMAX + j] * qj;
            }
#pragma unroll
            for (int i = 0; i < LMAX; ++i)
                P[i] = (i < L) ? P[i] + (i == sa ? dself : T(0)) : T(0);
            __syncthreads();   // the tile buffer is reused by tile_load below
        }
        T y[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) y[j] = T(0);
        if (staged) {
            tile_rows<T, LMAX, TP>(np, L, fy, lds, y);
        } else if (early) {
            __syncthreads();
            tile_read_own<T, LMAX>(np, L, lds, y);
        } else {
            tile_load<T, LMAX, TP>(A.y, p0, np, L, lds, y);
        }
        if (act) {
#pragma unroll
            for (int j = 0; j < LMAX; ++j) {
                if (j < L) {
                    acc[0] += double(y[j]) * double(P[j]);
                    if (j == sa) acc[1] += double(P[j]);
                }
            }
        }
        tile_store<T, LMAX, TP>(A.Ps, p0, np, L, lds, P);
    }
    const double tot = block_sum_waves<kP2, TP>(acc, red);
    if (img >= 0 && threadIdx.x < kP2)
        unsafeAtomicAdd(&A.acc[acc_off(A.it & 1, tile & (kSets - 1), A.nimg, img) +
                               kP1 + threadIdx.x], tot);
    if (tile == 0)   // the other parity: read by this iteration's step 1 only
        for (int i = threadIdx.x; i < kSets * A.nimg * kPT; i += TP)
            A.acc[acc_off((A.it + 1) & 1, 0, A.nimg, 0) + i] = 0.0;
}

template <typename T, int LMAX, bool POTTS>
__global__ void __launch_bounds__(RowTile<T>::kPix, 3)
k_fw_slice_rows(FWSliceArgs<T> A, LatSet<T> ls) {
    constexpr int TP = RowTile<T>::kPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    __shared__ int32_t sid[TP * kCorners52];
    __shared__ T swc[TP * kCorners52];
    __shared__ T smu[POTTS ? 1 : LMAX * LMAX];
    __shared__ double red[kP2 * (TP / 64)];
    fw_slice_tile<T, LMAX, POTTS, TP>(A, ls, xcd_block(blockIdx.x, gridDim.x), lds, sid, swc,
                                      smu, red);
}

// ------------------------------------------- persistent Frank-Wolfe launch

// All iterations of a Frank-Wolfe solve in one cooperative launch (every
// block resident at once): the per-stage kernels' bodies run over virtual
// blocks (tiles of kPersistPix pixels, splat chunks, blur vectors) with a
// grid barrier between the stages: LMO | one-hot splat | blur group 1 |
// ... | blur group n (with the vertex checkpoint) | slice |. The step size
// still rides on the stage boundary between the slice and the next LMO. The
// barrier's wait is bounded: a block that waits longer than kBarrierSpins
// polls sets the timeout flag and goes on (the host then reports the solve
// as failed), so a broken co-residency cannot hang the device.
constexpr int kPersistPix = 256;
constexpr unsigned kBarrierSpins = 1u << 22;

__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned &gen, int *timeout) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&bar[0], 1u) == gridDim.x - 1) {
            atomicExch(&bar[0], 0u);
            __threadfence();
            atomicAdd(&bar[1], 1u);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (++spins > kBarrierSpins) {
                    atomicOr(timeout, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        ++gen;
        __threadfence();
    }
    __syncthreads();
}

template <typename T>
struct FWPersist {
    FWArgs<T> a;          // the LMO's arguments (it, first, s, sprev, saves set per iteration)
    FWSliceArgs<T> b;     // the slice's
    int iters, g1, g2;    // iterations; LMO and slice tiles of kPersistPix pixels
    int q, U;             // one-hot splat: chunks per block, entries per chunk
    long long splat_blocks, blur_vecs;
    int ngrp;             // blur groups (launches of the per-stage path)
    int32_t *s0, *s1;     // the label buffers, alternating by iteration
    T *ysv, *psv;         // checkpoints (or null): y_t and P_t per iteration,
    int32_t *ssv;         // s_t,
    T *vsv;               // and the blurred vertex values after each iteration's blur
    size_t NL, vblock;
    unsigned *bar;        // count, generation (both zero at launch)
    int *timeout;
};

template <typename T, int LMAX, bool POTTS>
__global__ void __launch_bounds__(kPersistPix, 2)
k_fw_persistent(FWPersist<T> P, LatSet<T> ls) {
    constexpr int TP = kPersistPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    __shared__ double red[kP1 * (TP / 64)];
    __shared__ double stot[kPT];
    __shared__ int32_t sid[TP * kCorners52];
    __shared__ T swc[TP * kCorners52];
    __shared__ T smu[POTTS ? 1 : LMAX * LMAX];
    __shared__ PairLds<T> sp[kSplatStage];
    __shared__ int4 scd[256];
    unsigned gen = 0;
    const int L = P.a.L;
    using V = typename Vec16<T>::type;
    constexpr int vw = Vec16<T>::n;
    for (int it = 0; it < P.iters; ++it) {
        int32_t *scur = (it & 1) ? P.s1 : P.s0;
        FWArgs<T> a = P.a;
        a.it = it;
        a.first = it == 0 ? 1 : 0;
        a.s = scur;
        a.sprev = (it & 1) ? P.s0 : P.s1;
        a.ysave = P.ysv ? P.ysv + (size_t)it * P.NL : nullptr;
        a.Psave = P.psv ? P.psv + (size_t)it * P.NL : nullptr;
        a.ssave = P.ssv ? P.ssv + (size_t)it * a.N : nullptr;
        for (int vb = blockIdx.x; vb < P.g1; vb += gridDim.x) {
            fw_lmo_tile<T, LMAX, 0, TP>(a, ls, vb, lds, red, stot);
            __syncthreads();
        }
        grid_barrier(P.bar, gen, P.timeout);
        for (long long vb = blockIdx.x; vb < P.splat_blocks; vb += gridDim.x) {
            splat_labels_block<T>(L, P.q, P.U, scur, ls, vb * 256, sp, scd);
            __syncthreads();
        }
        grid_barrier(P.bar, gen, P.timeout);
        for (int grp = 0; grp < P.ngrp; ++grp) {
            for (long long e = (long long)blockIdx.x * TP + threadIdx.x; e < P.blur_vecs;
                 e += (long long)gridDim.x * TP)
                blur_group_vector<T, 2>(ls, grp, e);
            grid_barrier(P.bar, gen, P.timeout);
        }
        if (P.ngrp == 1) {   // no second group cleared the splat target
            for (long long e = (long long)blockIdx.x * TP + threadIdx.x; e < P.blur_vecs;
                 e += (long long)gridDim.x * TP) {
                int m = 0;
                while (m + 1 < ls.nk && e >= ls.off[m + 1] / vw) ++m;
                V zero;
                for (int i = 0; i < vw; ++i) reinterpret_cast<T *>(&zero)[i] = T(0);
                reinterpret_cast<V *>(ls.l[m].V0)[e - ls.off[m] / vw] = zero;
            }
        }
        if (P.vsv) {   // blurred vertex values for the reverse sweep (slot it + 1)
            T *dst = P.vsv + (size_t)(it + 1) * P.vblock;
            for (long long e = (long long)blockIdx.x * TP + threadIdx.x; e < P.blur_vecs * vw;
                 e += (long long)gridDim.x * TP) {
                int m = 0;
                while (m + 1 < ls.nk && e >= ls.off[m + 1]) ++m;
                dst[e] = ls.l[m].Vf[e - ls.off[m]];
            }
        }
        FWSliceArgs<T> b = P.b;
        b.it = it;
        b.s = scur;
        for (int vb = blockIdx.x; vb < P.g2; vb += gridDim.x) {
            fw_slice_tile<T, LMAX, POTTS, TP>(b, ls, vb, lds, sid, swc, smu, red);
            __syncthreads();
        }
        grid_barrier(P.bar, gen, P.timeout);
    }
}

__global__ void k_fill_u32(unsigned *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// ------------------------------------------------- flat kernels (L > 32)

// (Psi + D) Y for a dense Y (or its K'Y given in `pre`), whole pixels per block
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_slice_qp_flat(int N, int L, const T *__restrict__ Y, const T *__restrict__ pre,
                LatSet<T> ls, T wsum, const T *__restrict__ mu,
                const T *__restrict__ mabs, const T *__restrict__ r,
                T *__restrict__ out) {
    __shared__ T sq[kThreads];
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int l = t - lp * L;
    for (int g = blockIdx.x; (long long)g * ppb < N; g += gridDim.x) {
        const long long a = (long long)g * ppb + lp;
        const bool act = lp < ppb && a < N;
        const size_t e = (size_t)a * L + l;
        T yv = T(0);
        if (act) {
            yv = Y[e];
            T q;
            if (pre) {
                q = pre[e];
            } else {
                q = T(0);
                for (int m = 0; m < ls.nk; ++m) {
                    const LatView<T> &Lt = ls.l[m];
                    const int D1 = Lt.d + 1;
                    for (int k = 0; k < D1; ++k) {
                        const int id = Lt.vid[a * D1 + k];
                        if (id >= 0)
                            q += Lt.wg * Lt.w[a * D1 + k] * Lt.Vf[(size_t)id * Lt.ld + l];
                    }
                }
                q -= wsum * yv;
            }
            sq[t] = q;
        }
        __syncthreads();
        if (act) {
            T p = T(0);
            const T *qrow = sq + lp * L;
            for (int j = 0; j < L; ++j) p += mu[(size_t)l * L + j] * qrow[j];
            out[e] = p + mabs[l] * r[a] * yv;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fw_lmo_flat(FWArgs<T> A) {
    __shared__ T sg[kThreads];
    __shared__ int sarg[kThreads];
    __shared__ double red[kP1 * kThreads];
    const int L = A.L;
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int l = t - lp * L;
    int lo, hi;
    const int img = tile_range(A.seg, A.nimg, ppb * kFlatGroups, blockIdx.x, lo, hi);
    __shared__ double stot[kPT];
    const T al = A.first ? T(0)
                         : T(fw_block_step(fw_load_sum(A.acc, A.it - 1, A.nimg, img),
                                           A.it - 1, A.nimg, img,
                                           img >= 0 && lo == A.seg[2 * img], A.trace,
                                           A.stats, stot));
    double acc[kP1];
#pragma unroll
    for (int i = 0; i < kP1; ++i) acc[i] = 0.0;
    for (int g0 = lo; g0 < hi; g0 += ppb) {
        const long long a = (long long)g0 + lp;
        const bool act = lp < ppb && a < hi;
        const size_t e = (size_t)a * L + l;
        T yv = T(0), pyv = T(0), cv = T(0), gv = T(0);
        int sp = -1;
        if (act) {
            yv = A.y[e];
            pyv = A.Py[e];
            sp = A.sprev[a];
            if (!A.first) {
                yv = yv + al * (T(l == sp ? 1 : 0) - yv);
                pyv = (T(1) - al) * pyv + al * A.Ps[e];
                A.y[e] = yv;
                A.Py[e] = pyv;
            }
            cv = A.c[e];
            gv = cv + T(2) * pyv;
            sg[t] = gv;
        }
        __syncthreads();
        if (act && l == 0) {
            int best = 0;
            T bv = sg[t];
            for (int j = 1; j < L; ++j) {
                const T v = sg[t + j];
                if (v < bv) {
                    bv = v;
                    best = j;
                }
            }
            sarg[lp] = best;
            A.s[a] = best;
            acc[6] += (best != sp) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (act) {
            const int sl = sarg[lp];
            acc[0] += double(yv) * double(pyv);
            acc[2] += double(cv) * double(yv);
            acc[4] += double(gv) * double(yv);
            if (l == sl) {
                acc[1] += double(pyv);
                acc[3] += double(cv);
                acc[5] += double(gv);
            }
        }
        __syncthreads();
    }
    block_sum<kP1, kThreads>(acc, red);
    if (img >= 0 && t < kP1)
        unsafeAtomicAdd(&A.acc[acc_off(A.it & 1, blockIdx.x & (kSets - 1), A.nimg, img) + t],
                        acc[t]);
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fw_slice_flat(FWSliceArgs<T> A, LatSet<T> ls) {
    __shared__ T sq[kThreads];
    __shared__ double red[kP2 * kThreads];
    const int L = A.L;
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int l = t - lp * L;
    double acc[kP2] = {0.0, 0.0};
    int lo, hi;
    const int img = tile_range(A.seg, A.nimg, ppb * kFlatGroups, blockIdx.x, lo, hi);
    for (int g0 = lo; g0 < hi; g0 += ppb) {
        const long long a = (long long)g0 + lp;
        const bool act = lp < ppb && a < hi;
        const size_t e = (size_t)a * L + l;
        int sa = 0;
        if (act) {
            sa = A.s[a];
            T q;
            if (A.pre) {
                q = A.pre[e];
            } else {
                q = T(0);
                for (int m = 0; m < ls.nk; ++m) {
                    const LatView<T> &Lt = ls.l[m];
                    const int D1 = Lt.d + 1;
                    for (int k = 0; k < D1; ++k) {
                        const int id = Lt.vid[a * D1 + k];
                        if (id >= 0)
                            q += Lt.wg * Lt.w[a * D1 + k] * Lt.Vf[(size_t)id * Lt.ld + l];
                    }
                }
                if (l == sa) q -= A.wsum;
            }
            sq[t] = q;
        }
        __syncthreads();
        if (act) {
            T p = T(0);
            const T *qrow = sq + lp * L;
            for (int j = 0; j < L; ++j) p += A.mu[(size_t)l * L + j] * qrow[j];
            if (l == sa) p += A.mabs[l] * A.r[a];
            A.Ps[e] = p;
            acc[0] += double(A.y[e]) * double(p);
            if (l == sa) acc[1] += double(p);
        }
        __syncthreads();
    }
    double v[kP2] = {acc[0], acc[1]};
    block_sum<kP2, kThreads>(v, red);
    if (img >= 0 && t < kP2)
        unsafeAtomicAdd(&A.acc[acc_off(A.it & 1, blockIdx.x & (kSets - 1), A.nimg, img) +
                               kP1 + t], v[t]);
    if (blockIdx.x == 0)
        for (int i = t; i < kSets * A.nimg * kPT; i += kThreads)
            A.acc[acc_off((A.it + 1) & 1, 0, A.nimg, 0) + i] = 0.0;
}

// ------------------------------------------------------------ the rest

// y <- y + alpha (s - y), P_y <- (1 - alpha) P_y + alpha P_s with the last
// step of each image (blockIdx.y), solved here from the accumulated sums of
// iteration `it`; block (0, img) records its trace and checkpoint entries
template <typename T>
__global__ void k_fw_final(int L, const int *__restrict__ seg, T *__restrict__ y,
                           T *__restrict__ Py, const T *__restrict__ Ps,
                           const int32_t *__restrict__ s, const double *__restrict__ acc,
                           int it, int nimg, double *__restrict__ trace,
                           double *__restrict__ stats) {
    __shared__ double stot[kPT];
    const int img = blockIdx.y;
    const size_t lo = (size_t)seg[2 * img] * L, hi = (size_t)seg[2 * img + 1] * L;
    const T al = T(fw_block_step(fw_load_sum(acc, it, nimg, img), it, nimg, img,
                                 blockIdx.x == 0, trace, stats, stot));
    for (size_t e = lo + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < hi;
         e += (size_t)gridDim.x * blockDim.x) {
        const int a = int(e / L);
        const int l = int(e - (size_t)a * L);
        y[e] = y[e] + al * (T(l == s[a] ? 1 : 0) - y[e]);
        Py[e] = (T(1) - al) * Py[e] + al * Ps[e];
    }
}

template <typename T>
__global__ void k_onehot(int N, int L, const int32_t *__restrict__ s,
                         T *__restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * L) return;
    const int a = int(e / L);
    out[e] = T(int(e - (size_t)a * L) == s[a] ? 1 : 0);
}

__global__ void k_check_labels(const int *__restrict__ seg, int nimg, int L,
                               const int32_t *__restrict__ x,
                               int *__restrict__ bad) {
    int lo, hi;
    tile_range(seg, nimg, 256, blockIdx.x, lo, hi);
    const int a = lo + threadIdx.x;
    if (a < hi && (x[a] < 0 || x[a] >= L)) atomicOr(bad, 1);
}

template <typename T>
__global__ void k_round(int N, int L, const T *__restrict__ y,
                        int32_t *__restrict__ labels) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    int best = 0;
    T bv = y[(size_t)a * L];
    for (int j = 1; j < L; ++j) {
        const T v = y[(size_t)a * L + j];
        if (v > bv) {
            bv = v;
            best = j;
        }
    }
    labels[a] = best;
}

// per-block partial sums of the energy of labels x (the pairwise part reads
// the sliced one-hot filter, or its K'S in `pre`)
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_energy(const int *__restrict__ seg, int nimg, int L,
         const T *__restrict__ phi, const int32_t *__restrict__ x,
         const T *__restrict__ pre, LatSet<T> ls, T wsum,
         const T *__restrict__ mu, double *__restrict__ part) {
    __shared__ double red[kThreads];
    const int ppb = kThreads / L;
    const int t = threadIdx.x;
    const int lp = t / L;
    const int l = t - lp * L;
    double acc[1] = {0.0};
    int lo, hi;
    tile_range(seg, nimg, ppb * kFlatGroups, blockIdx.x, lo, hi);
    for (int g0 = lo; g0 < hi; g0 += ppb) {
        const long long a = (long long)g0 + lp;
        if (lp < ppb && a < hi) {
            const size_t e = (size_t)a * L + l;
            const int xa = x[a];
            if (xa < 0 || xa >= L) continue;   // rejected by k_check_labels
            T q;
            if (pre) {
                q = pre[e];
            } else {
                q = T(0);
                for (int m = 0; m < ls.nk; ++m) {
                    const LatView<T> &Lt = ls.l[m];
                    const int D1 = Lt.d + 1;
                    for (int k = 0; k < D1; ++k) {
                        const int id = Lt.vid[a * D1 + k];
                        if (id >= 0)
                            q += Lt.wg * Lt.w[a * D1 + k] * Lt.Vf[(size_t)id * Lt.ld + l];
                    }
                }
                if (l == xa) q -= wsum;
            }
            acc[0] += double(mu[(size_t)xa * L + l]) * double(q);
            if (l == xa) acc[0] += double(phi[e]);
        }
    }
    block_sum<1, kThreads>(acc, red);
    if (t == 0) part[blockIdx.x] = acc[0];
}

// per-block partial sums of S(y) = phi^T y + y^T Psi y with Psi y = P_y - d*y
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_S_value(const int *__restrict__ seg, int nimg, int L,
          const T *__restrict__ phi, const T *__restrict__ y,
          const T *__restrict__ Py, const T *__restrict__ mabs,
          const T *__restrict__ r, double *__restrict__ part) {
    __shared__ double red[kThreads];
    double acc[1] = {0.0};
    int lo, hi;
    tile_range(seg, nimg, kThreads, blockIdx.x, lo, hi);
    for (size_t e = (size_t)lo * L + threadIdx.x; e < (size_t)hi * L;
         e += kThreads) {
        const int a = int(e / L);
        const int i = int(e - (size_t)a * L);
        const double yv = y[e];
        acc[0] += double(phi[e]) * yv + yv * double(Py[e]) -
                  double(mabs[i]) * double(r[a]) * yv * yv;
    }
    block_sum<1, kThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

int grid_flat(int N, int L) {
    const int ppb = kThreads / L;
    return std::max(1, std::min(kMaxGrid, ceil_div(N, ppb)));
}

double sum_partials(dcrf_ctx *ctx, const double *dpart, int n) {
    std::vector<double> h(n);
    DCRF_TRY_HIP(hipMemcpyAsync(h.data(), dpart, n * sizeof(double),
                                hipMemcpyDeviceToHost, ctx->stream));
    DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += h[i];
    return s;
}

// Tiles (pixels per block) of the two per-pixel Frank-Wolfe kernels: the row
// kernels for L <= 32, the flat kernels above.
template <typename T>
int lmo_tile(int L) {
    return L <= kRowMaxC ? LmoTile<T>::kPix : (kThreads / L) * kFlatGroups;
}
template <typename T>
int slice_tile(int L) {
    return L <= kRowMaxC ? RowTile<T>::kPix : (kThreads / L) * kFlatGroups;
}
int flat_tile(int L) { return (kThreads / L) * kFlatGroups; }

template <typename T>
struct Work {
    T *c, *Py, *Ps, *mabs;
    int32_t *s, *sprev;
    double *acc, *trace;
    int G1, G2;   // blocks (tiles) of k_fw_lmo and k_fw_slice
};

template <typename T>
Work<T> fw_workspace(dcrf_ctx *ctx, int L, int iters) {
    const hipStream_t st = ctx->stream;
    const size_t NL = (size_t)ctx->N * L;
    const int G1 = seg_tiles(ctx, lmo_tile<T>(L));
    const int G2 = seg_tiles(ctx, slice_tile<T>(L));
    // the partial sums of k_S_value (the solver's own sums go to fw_scal)
    const size_t np = std::max<size_t>((size_t)G1 * kP1 + (size_t)G2 * kP2,
                                       (size_t)seg_tiles(ctx, kThreads));
    ctx->fw_c.ensure(NL * sizeof(T), st);
    ctx->fw_Py.ensure(NL * sizeof(T), st);
    ctx->fw_Ps.ensure(NL * sizeof(T), st);
    ctx->fw_s.ensure((size_t)ctx->N * 4, st);
    ctx->fw_sprev.ensure((size_t)ctx->N * 4, st);
    ctx->fw_part.ensure(np * 8, st);
    ctx->fw_scal.ensure((size_t)2 * kSets * ctx->nimg * kPT * 8, st);   // accumulators
    ctx->fw_trace.ensure((size_t)std::max(iters, 1) * ctx->nimg * 4 * 8, st);
    ctx->fw_mu.ensure((size_t)L * sizeof(T), st);
    Work<T> w;
    w.G1 = G1;
    w.G2 = G2;
    w.c = ctx->fw_c.as<T>();
    w.Py = ctx->fw_Py.as<T>();
    w.Ps = ctx->fw_Ps.as<T>();
    w.mabs = ctx->fw_mu.as<T>();
    w.s = ctx->fw_s.as<int32_t>();
    w.sprev = ctx->fw_sprev.as<int32_t>();
    w.acc = ctx->fw_scal.as<double>();
    w.trace = ctx->fw_trace.as<double>();
    return w;
}

template <typename T>
void qp_apply_t(dcrf_ctx *ctx, const T *y, const T *mu, int L, const T *mabs,
                T *out) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N;
    const T *pre = nullptr;
    if (ctx->mode != DCRF_FILTER_LATTICE) {
        ctx->tmpA.ensure((size_t)N * L * sizeof(T), st);
        filter_apply(ctx, y, ctx->tmpA.p, L, false, ctx->mode);
        pre = ctx->tmpA.as<T>();
    } else {
        splat_dense(ctx, y, L);
        blur_all(ctx, L, false);
    }
    if (L <= kRowMaxC) {
        slice_into(ctx, y, pre, L, mu, mabs, out, true);
        return;
    }
    LatSet<T> ls = make_lat_set<T>(ctx, L);
    ProfScope ps(ctx, PROF_SLICE_QP);
    DCRF_PLAUNCH(ps, (k_slice_qp_flat<T>), dim3(grid_flat(N, L)),
                       dim3(kThreads), 0, st, N, L, y, pre, ls, T(ctx->wsum),
                       mu, mabs, ctx->r.as<T>(), out);
    DCRF_CHECK_LAUNCH();
}

// Whether mu is the Potts compatibility [i != j]: known without a host read
// for the context's own copy (a null mu at the boundary), else read once.
template <typename T>
bool is_potts(dcrf_ctx *ctx, const T *mu, int L) {
    if (is_internal_potts(ctx, mu)) return true;
    // up to 32 labels the copy lives on the stack (no host allocation)
    T small[kRowMaxC * kRowMaxC];
    std::vector<T> big;
    T *h = small;
    if (L > kRowMaxC) {
        big.resize((size_t)L * L);
        h = big.data();
    }
    DCRF_TRY_HIP(hipMemcpyAsync(h, mu, (size_t)L * L * sizeof(T),
                                hipMemcpyDeviceToHost, ctx->stream));
    DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j)
            if (h[(size_t)i * L + j] != T(i != j ? 1 : 0)) return false;
    return true;
}

template <typename T, int LMAX, bool POTTS>
void fw_persistent_go(dcrf_ctx *ctx, FWPersist<T> &P, LatSet<T> &ls) {
    const auto kern = k_fw_persistent<T, LMAX, POTTS>;
    int per_cu = 0, cus = 0;
    DCRF_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPersistPix, 0));
    DCRF_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                       ctx->device));
    if (per_cu < 1) fail(DCRF_EUNSUPPORTED, "the persistent solve does not fit a compute unit");
    long long need = std::max<long long>(P.g1, P.g2);
    need = std::max(need, P.splat_blocks);
    need = std::max(need, (P.blur_vecs + kPersistPix - 1) / kPersistPix);
    const int grid = int(std::max(1ll, std::min<long long>((long long)per_cu * cus, need)));
    void *args[] = {&P, &ls};
    DCRF_TRY_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(grid),
                                            dim3(kPersistPix), args, 0, ctx->stream));
}

// All iterations of the solve in one cooperative launch (k_fw_persistent),
// then a check that no grid barrier timed out.
template <typename T>
void fw_persistent_launch(dcrf_ctx *ctx, LatSet<T> ls, const Work<T> &w, T *y, const T *mu,
                          int L, int iters, const FWCheckpoint *save, size_t vblock,
                          bool potts) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N;
    blur_group_tables(ctx, 2);
    for (int m = 0; m < ctx->nk; ++m) ls.l[m].gt = ctx->lat[m].gtab[0].as<int32_t>();
    ctx->fw_bar.ensure(256, st);
    unsigned *bar = ctx->fw_bar.as<unsigned>();
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, bar, 3);
    FWPersist<T> P{};
    P.a = FWArgs<T>{N, L, y, w.Py, w.Ps, w.c, w.s, w.sprev, w.acc, w.trace,
                    save ? save->stats : nullptr, 0, 1, ctx->seg.as<int>(), ctx->nimg,
                    nullptr, nullptr, nullptr};
    P.b = FWSliceArgs<T>{N, L, y, w.s, w.Ps, mu, w.mabs, ctx->r.as<T>(), nullptr,
                         T(ctx->wsum), w.acc, 0, ctx->seg.as<int>(), ctx->nimg};
    P.iters = iters;
    P.g1 = P.g2 = seg_tiles(ctx, kPersistPix);
    P.q = dense_splat_q(ctx, L);
    P.U = ctx->dense_chunk;
    P.splat_blocks = ls.coff[ls.nk] / 256;
    P.blur_vecs = ls.off[ls.nk] / Vec16<T>::n;
    P.ngrp = 0;
    for (int m = 0; m < ls.nk; ++m) P.ngrp = std::max(P.ngrp, ls.l[m].ngrp);
    P.s0 = w.s;
    P.s1 = w.sprev;
    P.ysv = save ? static_cast<T *>(save->y) : nullptr;
    P.psv = save ? static_cast<T *>(save->P) : nullptr;
    P.ssv = save ? save->s : nullptr;
    P.vsv = save && vblock ? static_cast<T *>(save->V) : nullptr;
    P.NL = (size_t)N * L;
    P.vblock = vblock;
    P.bar = bar;
    P.timeout = reinterpret_cast<int *>(bar + 2);
    DCRF_CHECK_LAUNCH();
    if (potts)
        DCRF_DISPATCH_ROWS(L, (fw_persistent_go<T, LMAX, true>(ctx, P, ls)));
    else
        DCRF_DISPATCH_ROWS(L, (fw_persistent_go<T, LMAX, false>(ctx, P, ls)));
    int timed_out = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&timed_out, bar + 2, 4, hipMemcpyDeviceToHost, st));
    DCRF_TRY_HIP(hipStreamSynchronize(st));
    if (timed_out)
        fail(DCRF_EHIP, "a grid barrier of the persistent Frank-Wolfe launch timed out");
}

template <typename T>
void frank_wolfe_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, T *y,
                   int iters, dcrf_iter_trace *trace, int cmode, bool have_Py,
                   const FWCheckpoint *save = nullptr, int potts_known = -1) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N;
    const size_t NL = (size_t)N * L;
    Work<T> w = fw_workspace<T>(ctx, L, iters);
    const int gE = ceil_div((long long)NL, 256);
    hipLaunchKernelGGL((k_mu_abs<T>), dim3(1), dim3(256), 0, st, L, mu, w.mabs);
    // linear term: c = phi - d (convex QP) or phi - 2 d * y (CCCP step)
    hipLaunchKernelGGL((k_linear_term<T>), dim3(gE), dim3(256), 0, st, N, L,
                       phi, ctx->r.as<T>(), w.mabs, cmode == 1 ? y : nullptr,
                       T(cmode == 1 ? 2 : 1), w.c);
    if (!have_Py) qp_apply_t<T>(ctx, y, mu, L, w.mabs, w.Py);
    // blurred vertex values of every lattice, one block per checkpoint
    size_t vblock = 0;
    if (save && ctx->mode == DCRF_FILTER_LATTICE)
        for (int m = 0; m < ctx->nk; ++m)
            vblock += (size_t)ctx->lat[m].M * row_stride(L, sizeof(T));
    auto save_vertices = [&](int slot) {
        const LatSet<T> cur = make_lat_set<T>(ctx, L);
        T *dst = static_cast<T *>(save->V) + (size_t)slot * vblock;
        for (int m = 0; m < ctx->nk; ++m) {
            const size_t n = (size_t)ctx->lat[m].M * cur.l[m].ld;
            DCRF_TRY_HIP(hipMemcpyAsync(dst, cur.l[m].Vf, n * sizeof(T),
                                        hipMemcpyDeviceToDevice, st));
            dst += n;
        }
    };
    if (save && vblock) {
        if (have_Py) fail(DCRF_EINVAL, "checkpoints need the first filter of y");
        save_vertices(0);
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(N, 256)), dim3(256), 0, st,
                       w.sprev, (size_t)N, -1);
    {   // the step-size accumulators start at zero (a fill kernel, not a memset)
        const size_t n = (size_t)2 * kSets * ctx->nimg * kPT;
        hipLaunchKernelGGL((k_fill<double>), dim3(ceil_div((long long)n, 256)), dim3(256),
                           0, st, w.acc, n, 0.0);
    }
    DCRF_CHECK_LAUNCH();

    const bool exact = ctx->mode != DCRF_FILTER_LATTICE;   // K'S of a dense one-hot
    const bool rows = L <= kRowMaxC;
    if (!exact) ensure_vertex_buffers(ctx, L);
    if (exact) {
        ctx->tmpA.ensure(NL * sizeof(T), st);
        ctx->tmpB.ensure(NL * sizeof(T), st);
    }
    // one block per tile of an image (k_fw_lmo: G1 tiles, k_fw_slice: G tiles)
    const int G1 = w.G1, G = w.G2;
    const int nimg = ctx->nimg;
    const int *seg = ctx->seg.as<int>();
    const bool potts = potts_known >= 0 ? potts_known != 0 : is_potts<T>(ctx, mu, L);
    const LatSet<T> ls = exact ? LatSet<T>{} : make_lat_set<T>(ctx, L);
    // the one-hot splat inside the LMO kernel (the row kernels only)
    const int fuse = (!exact && rows && ctx->fw_splat) ? (ls.shape52 ? 2 : 1) : 0;
    // every iteration in one cooperative launch: the row kernels' lattice
    // path with the staged one-hot splat and two blur directions per group
    const bool persist = ctx->fw_persistent && !exact && rows && !fuse && iters > 0 &&
                         ctx->blur_group == 2 && !ctx->tile_mode && ctx->splat_lds;
    if (persist) {
        fw_persistent_launch<T>(ctx, ls, w, y, mu, L, iters, save, vblock, potts);
        if (iters & 1) std::swap(w.s, w.sprev);   // the last s where the loop leaves it
    }
    for (int it = 0; it < (persist ? 0 : iters); ++it) {
        // checkpoints are written by the row kernel itself; the flat kernel
        // (more than 32 labels) leaves them to copies below
        T *ysv = save && rows ? static_cast<T *>(save->y) + (size_t)it * NL : nullptr;
        T *psv = save && rows ? static_cast<T *>(save->P) + (size_t)it * NL : nullptr;
        int32_t *ssv = save && rows ? save->s + (size_t)it * N : nullptr;
        FWArgs<T> a{N, L, y, w.Py, w.Ps, w.c, w.s, w.sprev, w.acc, w.trace,
                    save ? save->stats : nullptr, it, it == 0 ? 1 : 0, seg, nimg,
                    ysv, psv, ssv};
        {
            ProfScope ps(ctx, PROF_FW_LMO);
            if (rows && fuse == 2) {
                DCRF_DISPATCH_ROWS(L, DCRF_PLAUNCH(ps, (k_fw_lmo_rows<T, LMAX, 2>),
                                                         dim3(G1), dim3(LmoTile<T>::kPix),
                                                         0, st, a, ls));
            } else if (rows && fuse == 1) {
                DCRF_DISPATCH_ROWS(L, DCRF_PLAUNCH(ps, (k_fw_lmo_rows<T, LMAX, 1>),
                                                         dim3(G1), dim3(LmoTile<T>::kPix),
                                                         0, st, a, ls));
            } else if (rows) {
                DCRF_DISPATCH_ROWS(L, DCRF_PLAUNCH(ps, (k_fw_lmo_rows<T, LMAX, 0>),
                                                         dim3(G1), dim3(LmoTile<T>::kPix),
                                                         0, st, a, ls));
            } else {
                DCRF_PLAUNCH(ps, (k_fw_lmo_flat<T>), dim3(G1), dim3(kThreads), 0,
                                   st, a);
            }
        }
        if (save && !rows) {   // y_t, P_t and s_t for the reverse sweep
            DCRF_TRY_HIP(hipMemcpyAsync(static_cast<T *>(save->y) + (size_t)it * NL, y,
                                        NL * sizeof(T), hipMemcpyDeviceToDevice, st));
            DCRF_TRY_HIP(hipMemcpyAsync(static_cast<T *>(save->P) + (size_t)it * NL, w.Py,
                                        NL * sizeof(T), hipMemcpyDeviceToDevice, st));
            DCRF_TRY_HIP(hipMemcpyAsync(save->s + (size_t)it * N, w.s, (size_t)N * 4,
                                        hipMemcpyDeviceToDevice, st));
        }
        const T *pre = nullptr;
        if (exact) {
            hipLaunchKernelGGL((k_onehot<T>), dim3(gE), dim3(256), 0, st, N, L,
                               w.s, ctx->tmpB.as<T>());
            filter_apply(ctx, ctx->tmpB.p, ctx->tmpA.p, L, false, ctx->mode);
            pre = ctx->tmpA.as<T>();
        } else {
            if (!fuse) splat_labels(ctx, w.s, L);
            blur_all(ctx, L, false);
            if (save && vblock) save_vertices(it + 1);
        }
        FWSliceArgs<T> b{N, L, y, w.s, w.Ps, mu, w.mabs, ctx->r.as<T>(), pre,
                         T(ctx->wsum), w.acc, it, seg, nimg};
        {
            ProfScope ps(ctx, PROF_FW_SLICE);
            if (rows) {
                if (potts)
                    DCRF_DISPATCH_ROWS(L, DCRF_PLAUNCH(ps, 
                        (k_fw_slice_rows<T, LMAX, true>), dim3(G),
                        dim3(RowTile<T>::kPix), 0, st, b, ls));
                else
                    DCRF_DISPATCH_ROWS(L, DCRF_PLAUNCH(ps, 
                        (k_fw_slice_rows<T, LMAX, false>), dim3(G),
                        dim3(RowTile<T>::kPix), 0, st, b, ls));
            } else {
                DCRF_PLAUNCH(ps, (k_fw_slice_flat<T>), dim3(G), dim3(kThreads),
                                   0, st, b, ls);
            }
        }
        DCRF_CHECK_LAUNCH();
        std::swap(w.s, w.sprev);
    }
    // the last conditional gradient is in sprev after the swap
    if (iters > 0) {
        int maxn = 1;
        for (int j = 0; j < nimg; ++j)
            maxn = std::max(maxn, ctx->seg_h[2 * j + 1] - ctx->seg_h[2 * j]);
        const int gx = std::min(4096, ceil_div((long long)maxn * L, 256));
        ProfScope ps(ctx, PROF_FW_FINAL);
        DCRF_PLAUNCH(ps, (k_fw_final<T>), dim3(gx, nimg), dim3(256), 0, st, L, seg, y,
                     w.Py, w.Ps, w.sprev, w.acc, iters - 1, nimg, w.trace,
                     save ? save->stats : nullptr);
        DCRF_CHECK_LAUNCH();
    }
    if (trace && iters > 0) {   // record it * nimg + image: (f, gap, alpha, changed)
        static_assert(sizeof(dcrf_iter_trace) == 4 * sizeof(double),
                      "a trace record is four doubles, as on the device");
        DCRF_TRY_HIP(hipMemcpyAsync(trace, w.trace, (size_t)iters * nimg * 4 * 8,
                                    hipMemcpyDeviceToHost, st));
        DCRF_TRY_HIP(hipStreamSynchronize(st));
    }
}

// the per-tile partial sums of S(y) = phi^T y + y^T Psi y (from P_y) into
// part[0, G), G = seg_tiles(ctx, kThreads)
template <typename T>
void S_partials_t(dcrf_ctx *ctx, const T *phi, const T *y, int L, double *part) {
    const int G = seg_tiles(ctx, kThreads);
    hipLaunchKernelGGL((k_S_value<T>), dim3(G), dim3(kThreads), 0, ctx->stream,
                       ctx->seg.as<int>(), ctx->nimg, L, phi, y, ctx->fw_Py.as<T>(),
                       ctx->fw_mu.as<T>(), ctx->r.as<T>(), part);
    DCRF_CHECK_LAUNCH();
}

// CCCP on the generic DC decomposition. The S history's partial sums stay on
// the device, one row per value, and are read back once at the end: a call
// waits for the stream only when S_hist is asked for, and then once.
template <typename T>
void dc_gen_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L, T *y, int outer,
              int inner, double *S_hist) {
    // P_y = (Psi + D) y for the starting point
    Work<T> w = fw_workspace<T>(ctx, L, inner);
    const int G = seg_tiles(ctx, kThreads);
    DevBuf &hp = ctx->hist;   // outer + 1 rows of G partial sums
    if (S_hist) hp.ensure((size_t)(outer + 1) * G * 8, ctx->stream);
    hipLaunchKernelGGL((k_mu_abs<T>), dim3(1), dim3(256), 0, ctx->stream, L, mu,
                       w.mabs);
    qp_apply_t<T>(ctx, y, mu, L, w.mabs, w.Py);
    if (S_hist) S_partials_t<T>(ctx, phi, y, L, hp.as<double>());
    const int potts = outer > 0 ? (is_potts<T>(ctx, mu, L) ? 1 : 0) : 0;
    for (int k = 0; k < outer; ++k) {
        frank_wolfe_t<T>(ctx, phi, mu, L, y, inner, nullptr, 1, true, nullptr, potts);
        if (S_hist) S_partials_t<T>(ctx, phi, y, L, hp.as<double>() + (size_t)(k + 1) * G);
    }
    if (S_hist) {
        std::vector<double> h((size_t)(outer + 1) * G);
        DCRF_TRY_HIP(hipMemcpyAsync(h.data(), hp.p, h.size() * 8,
                                    hipMemcpyDeviceToHost, ctx->stream));
        DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
        for (int k = 0; k <= outer; ++k) {
            double v = 0.0;
            for (int i = 0; i < G; ++i) v += h[(size_t)k * G + i];
            S_hist[k] = v;
        }
    }
}

template <typename T>
double energy_t(dcrf_ctx *ctx, const T *phi, const T *mu, int L,
                const int32_t *x) {
    const hipStream_t st = ctx->stream;
    const int N = ctx->N;
    {
        ctx->scratch.ensure(64, st);
        int *bad = ctx->scratch.as<int>() + 1;
        DCRF_TRY_HIP(hipMemsetAsync(bad, 0, 4, st));
        hipLaunchKernelGGL(k_check_labels, dim3(seg_tiles(ctx, 256)), dim3(256), 0,
                           st, ctx->seg.as<int>(), ctx->nimg, L, x, bad);
        int hbad = 0;
        DCRF_TRY_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
        DCRF_TRY_HIP(hipStreamSynchronize(st));
        if (hbad) fail(DCRF_EINVAL, "labels must lie in [0, L)");
    }
    const T *pre = nullptr;
    LatSet<T> ls{};
    if (ctx->mode != DCRF_FILTER_LATTICE) {
        ctx->tmpA.ensure((size_t)N * L * sizeof(T), st);
        ctx->tmpB.ensure((size_t)N * L * sizeof(T), st);
        hipLaunchKernelGGL((k_onehot<T>), dim3(ceil_div((long long)N * L, 256)),
                           dim3(256), 0, st, N, L, x, ctx->tmpB.as<T>());
        filter_apply(ctx, ctx->tmpB.p, ctx->tmpA.p, L, false, ctx->mode);
        pre = ctx->tmpA.as<T>();
    } else {
        splat_labels(ctx, x, L);
        blur_all(ctx, L, false);
        ls = make_lat_set<T>(ctx, L);
    }
    const int G = seg_tiles(ctx, flat_tile(L));
    ctx->fw_part.ensure((size_t)G * 8, st);
    hipLaunchKernelGGL((k_energy<T>), dim3(G), dim3(kThreads), 0, st,
                       ctx->seg.as<int>(), ctx->nimg, L, phi, x, pre, ls,
                       T(ctx->wsum), mu, ctx->fw_part.as<double>());
    DCRF_CHECK_LAUNCH();
    return sum_partials(ctx, ctx->fw_part.as<double>(), G);
}

// dcrf_qp_frank_wolfe with every buffer the solve takes borrowed from
// `base` (cap bytes): the same kernels on the same layouts, with the
// per-call state (linear term, P_y, P_s, conditional gradients, partial
// sums, step accumulators, trace, sum_j |mu_ij|, the Potts copy of mu, the
// input-error flag) and each lattice's three vertex-value arrays placed at
// 256-byte aligned offsets of base. Everything else the solve reads (the
// lattice tables, r, the blur path tables) was built by dcrf_set_image. While
// it runs, any other allocation fails with DCRF_ENOMEM instead of reaching
// the device allocator, and the context's own buffers are restored on exit.
template <typename T>
void fw_noalloc_t(dcrf_ctx *ctx, const T *phi, const void *mu, int L, T *y, int iters,
                  dcrf_iter_trace *trace, char *base, size_t cap) {
    if (ctx->mode != DCRF_FILTER_LATTICE)
        fail(DCRF_EUNSUPPORTED, "the allocation-free solve needs the lattice filter mode");
    if (L > kRowMaxC) fail(DCRF_EUNSUPPORTED, "the allocation-free solve takes L <= 32");
    if (iters > 4096) fail(DCRF_EINVAL, "the allocation-free solve takes iters <= 4096");
    const int nimg = ctx->nimg;
    const size_t N = ctx->N, NL = N * L, e = sizeof(T);
    const int G1 = seg_tiles(ctx, lmo_tile<T>(L)), G2 = seg_tiles(ctx, slice_tile<T>(L));
    const size_t np = std::max<size_t>((size_t)G1 * kP1 + (size_t)G2 * kP2,
                                       (size_t)seg_tiles(ctx, kThreads));
    const size_t ld = row_stride(L, e);
    struct Item { DevBuf *buf; size_t bytes; };
    constexpr int kItems = 11 + 3 * DCRF_MAXK;
    Item items[kItems];
    int n = 0;
    for (DevBuf *b : {&ctx->fw_c, &ctx->fw_Py, &ctx->fw_Ps}) items[n++] = {b, NL * e};
    items[n++] = {&ctx->fw_s, N * 4};
    items[n++] = {&ctx->fw_sprev, N * 4};
    items[n++] = {&ctx->fw_part, np * 8};
    items[n++] = {&ctx->fw_scal, (size_t)2 * kSets * nimg * kPT * 8};
    items[n++] = {&ctx->fw_trace, (size_t)std::max(iters, 1) * nimg * 4 * 8};
    items[n++] = {&ctx->fw_mu, (size_t)L * e};
    items[n++] = {&ctx->potts, (size_t)L * L * e};
    items[n++] = {&ctx->errflag, 4};
    for (int m = 0; m < ctx->nk; ++m)
        for (int b = 0; b < 3; ++b)
            items[n++] = {&ctx->lat[m].V[b], (size_t)std::max(ctx->lat[m].M, 1) * ld * e};
    size_t total = 0;
    for (int i = 0; i < n; ++i) total += (items[i].bytes + 255) / 256 * 256;
    if (total > cap)
        fail(DCRF_EINVAL, "this solve needs " + std::to_string(total) +
                              " bytes of scratch; the allocation-free entry point has " +
                              std::to_string(cap));
    // borrow, and put everything back however the solve ends
    struct Restore {
        dcrf_ctx *ctx;
        Item *items;
        int n;
        DevBuf saved[kItems];
        int potts_L, potts_dtype;
        bool prof;
        int persistent;
        Arena *arena;
        Arena refuse;
        ~Restore() {
            for (int i = 0; i < n; ++i) *items[i].buf = saved[i];
            ctx->potts_L = potts_L;
            ctx->potts_dtype = potts_dtype;
            ctx->prof.on = prof;
            ctx->fw_persistent = persistent;
            tl_arena = arena;
        }
    } rs{ctx, items, n, {}, ctx->potts_L, ctx->potts_dtype, ctx->prof.on,
         ctx->fw_persistent, tl_arena, {}};
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        rs.saved[i] = *items[i].buf;
        DevBuf b;
        b.p = base + off;
        b.bytes = (items[i].bytes + 255) / 256 * 256;
        b.borrowed = true;
        *items[i].buf = b;
        off += b.bytes;
    }
    ctx->potts_L = 0;       // the Potts copy is rebuilt in the scratch when asked for
    ctx->prof.on = false;   // profiling would create events
    // the per-stage launches: the persistent solve waits for the stream (its
    // barrier check) and keeps a buffer of its own
    ctx->fw_persistent = 0;
    rs.refuse.refuse = "the allocation-free solve would need device memory beyond its "
                       "scratch (e.g. blur tables for a launch shape not yet used)";
    tl_arena = &rs.refuse;
    const hipStream_t st = ctx->stream;
    // what must start at zero: the splat targets and the error flag
    for (int m = 0; m < ctx->nk; ++m) {
        const size_t cnt = (size_t)std::max(ctx->lat[m].M, 1) * ld;
        hipLaunchKernelGGL((k_fill<T>), dim3(ceil_div((long long)cnt, 256)), dim3(256), 0,
                           st, ctx->lat[m].V[0].as<T>(), cnt, T(0));
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, ctx->errflag.as<int32_t>(),
                       (size_t)1, 0);
    DCRF_CHECK_LAUNCH();
    const T *mu_eff = static_cast<const T *>(resolve_mu(ctx, mu, L));
    check_finite(ctx, phi, L);
    check_finite(ctx, y, L);
    frank_wolfe_t<T>(ctx, phi, mu_eff, L, y, iters, trace, 0, false);
    if (trace) raise_device_errors(ctx);
}

}  // namespace

// flag |= 1 if an element of an image's rows of x (N x L) is not finite;
// rows between the images of a batch are not read
template <typename T>
__global__ void __launch_bounds__(256)
k_check_finite(const int *__restrict__ seg, int nimg, int L, const T *__restrict__ x,
               int *__restrict__ flag) {
    int lo, hi;
    tile_range(seg, nimg, 256, blockIdx.x, lo, hi);
    bool bad = false;
    for (size_t e = (size_t)lo * L + threadIdx.x; e < (size_t)hi * L; e += 256)
        bad = bad || !isfinite(double(x[e]));
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

template <typename T>
__global__ void k_potts_fill(int L, T *__restrict__ mu) {
    for (int e = threadIdx.x; e < L * L; e += blockDim.x)
        mu[e] = (e / L != e % L) ? T(1) : T(0);
}

void check_finite(dcrf_ctx *ctx, const void *x, int L) {
    ctx->errflag.ensure(4, ctx->stream);
    const int G = seg_tiles(ctx, 256);
    if (ctx->dtype == DCRF_F64)
        hipLaunchKernelGGL((k_check_finite<double>), dim3(G), dim3(256), 0, ctx->stream,
                           ctx->seg.as<int>(), ctx->nimg, L,
                           static_cast<const double *>(x), ctx->errflag.as<int>());
    else
        hipLaunchKernelGGL((k_check_finite<float>), dim3(G), dim3(256), 0, ctx->stream,
                           ctx->seg.as<int>(), ctx->nimg, L,
                           static_cast<const float *>(x), ctx->errflag.as<int>());
    DCRF_CHECK_LAUNCH();
}

void raise_device_errors(dcrf_ctx *ctx) {
    if (!ctx->errflag.p) return;
    int h = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&h, ctx->errflag.p, 4, hipMemcpyDeviceToHost, ctx->stream));
    DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (!h) return;
    DCRF_TRY_HIP(hipMemsetAsync(ctx->errflag.p, 0, 4, ctx->stream));
    fail(DCRF_EINVAL, "a non-finite value in the unaries or marginals given to this "
                      "call or to an earlier call since the last check");
}

const void *resolve_mu(dcrf_ctx *ctx, const void *mu, int L) {
    if (mu) return mu;
    if (!(ctx->potts.p && ctx->potts_L == L && ctx->potts_dtype == ctx->dtype)) {
        ctx->potts.ensure((size_t)L * L * ctx->elt(), ctx->stream);
        if (ctx->dtype == DCRF_F64)
            hipLaunchKernelGGL((k_potts_fill<double>), dim3(1), dim3(256), 0, ctx->stream,
                               L, ctx->potts.as<double>());
        else
            hipLaunchKernelGGL((k_potts_fill<float>), dim3(1), dim3(256), 0, ctx->stream,
                               L, ctx->potts.as<float>());
        DCRF_CHECK_LAUNCH();
        ctx->potts_L = L;
        ctx->potts_dtype = ctx->dtype;
    }
    return ctx->potts.p;
}

void frank_wolfe_noalloc(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                         void *y, int iters, dcrf_iter_trace *trace, void *base,
                         size_t cap) {
    if (ctx->dtype == DCRF_F64)
        fw_noalloc_t<double>(ctx, static_cast<const double *>(unary), mu, L,
                             static_cast<double *>(y), iters, trace,
                             static_cast<char *>(base), cap);
    else
        fw_noalloc_t<float>(ctx, static_cast<const float *>(unary), mu, L,
                            static_cast<float *>(y), iters, trace,
                            static_cast<char *>(base), cap);
}

void fill_ones(dcrf_ctx *ctx, void *p, size_t n) {
    if (ctx->dtype == DCRF_F64)
        hipLaunchKernelGGL((k_fill<double>), dim3(ceil_div((long long)n, 256)),
                           dim3(256), 0, ctx->stream, static_cast<double *>(p), n,
                           1.0);
    else
        hipLaunchKernelGGL((k_fill<float>), dim3(ceil_div((long long)n, 256)),
                           dim3(256), 0, ctx->stream, static_cast<float *>(p), n,
                           1.0f);
    DCRF_CHECK_LAUNCH();
}

void qp_apply(dcrf_ctx *ctx, const void *y, const void *mu, int L, void *out) {
    const hipStream_t st = ctx->stream;
    ctx->fw_mu.ensure((size_t)L * ctx->elt(), st);
    if (ctx->dtype == DCRF_F64) {
        hipLaunchKernelGGL((k_mu_abs<double>), dim3(1), dim3(256), 0, st, L,
                           static_cast<const double *>(mu), ctx->fw_mu.as<double>());
        qp_apply_t<double>(ctx, static_cast<const double *>(y),
                           static_cast<const double *>(mu), L,
                           ctx->fw_mu.as<double>(), static_cast<double *>(out));
    } else {
        hipLaunchKernelGGL((k_mu_abs<float>), dim3(1), dim3(256), 0, st, L,
                           static_cast<const float *>(mu), ctx->fw_mu.as<float>());
        qp_apply_t<float>(ctx, static_cast<const float *>(y),
                          static_cast<const float *>(mu), L,
                          ctx->fw_mu.as<float>(), static_cast<float *>(out));
    }
}

void frank_wolfe(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                 void *y, int iters, dcrf_iter_trace *trace, const void *,
                 bool have_Py) {
    if (ctx->dtype == DCRF_F64)
        frank_wolfe_t<double>(ctx, static_cast<const double *>(unary),
                              static_cast<const double *>(mu), L,
                              static_cast<double *>(y), iters, trace, 0, have_Py);
    else
        frank_wolfe_t<float>(ctx, static_cast<const float *>(unary),
                             static_cast<const float *>(mu), L,
                             static_cast<float *>(y), iters, trace, 0, have_Py);
}

static_assert(kStats == kFWStats, "checkpoint layout");

void frank_wolfe_checkpointed(dcrf_ctx *ctx, const void *unary, const void *mu,
                              int L, void *y, int iters, const FWCheckpoint &save) {
    if (ctx->dtype == DCRF_F64)
        frank_wolfe_t<double>(ctx, static_cast<const double *>(unary),
                              static_cast<const double *>(mu), L,
                              static_cast<double *>(y), iters, nullptr, 0, false,
                              &save);
    else
        frank_wolfe_t<float>(ctx, static_cast<const float *>(unary),
                             static_cast<const float *>(mu), L,
                             static_cast<float *>(y), iters, nullptr, 0, false,
                             &save);
}

void dc_gen(dcrf_ctx *ctx, const void *unary, const void *mu, int L, void *y,
            int outer, int inner, double *S_hist) {
    if (ctx->dtype == DCRF_F64)
        dc_gen_t<double>(ctx, static_cast<const double *>(unary),
                         static_cast<const double *>(mu), L,
                         static_cast<double *>(y), outer, inner, S_hist);
    else
        dc_gen_t<float>(ctx, static_cast<const float *>(unary),
                        static_cast<const float *>(mu), L,
                        static_cast<float *>(y), outer, inner, S_hist);
}

void round_labels(dcrf_ctx *ctx, const void *y, int L, int32_t *labels) {
    if (ctx->dtype == DCRF_F64)
        hipLaunchKernelGGL((k_round<double>), dim3(ceil_div(ctx->N, 256)),
                           dim3(256), 0, ctx->stream, ctx->N, L,
                           static_cast<const double *>(y), labels);
    else
        hipLaunchKernelGGL((k_round<float>), dim3(ceil_div(ctx->N, 256)),
                           dim3(256), 0, ctx->stream, ctx->N, L,
                           static_cast<const float *>(y), labels);
    DCRF_CHECK_LAUNCH();
}

double energy(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
              const int32_t *labels) {
    if (ctx->dtype == DCRF_F64)
        return energy_t<double>(ctx, static_cast<const double *>(unary),
                                static_cast<const double *>(mu), L, labels);
    return energy_t<float>(ctx, static_cast<const float *>(unary),
                           static_cast<const float *>(mu), L, labels);
}

}  // namespace dcrf
