// The pairwise filter K' Y = sum_m w_m K_m Y - (sum_m w_m) Y (eq. fb summed
// over the kernels of eq. pairwise, without the b = a term of
// eq. labelling-energy), in two forms:
//
//  - permutohedral: K_m Y ~ gamma_d slice(blur(splat(Y))), with
//    gamma_d = (4 pi / 3)^{d/2} sqrt(d+1) so that the response to a uniform
//    density equals the Gaussian integral.
//      splat: a gather over each vertex's inverse index. The (pixel, weight)
//        pairs of a vertex are cut into chunks of at most `chunk` pairs; one
//        group of C lanes per chunk sums w * Y[pixel] and adds the sum to the
//        vertex row with one atomic per channel. Vertices shared by thousands
//        of pixels (flat colour regions of the bilateral lattice) cost one
//        atomic per chunk instead of one per pixel. A block stages its
//        chunks' pairs in LDS first, so the only scattered global loads left
//        are those of the input values (or, for a one-hot input, of the
//        labels).
//      blur: d+1 out-of-place passes V'[v] = V[v]/2 + (V[v+u_j] + V[v-u_j])/4
//        (missing neighbours read as 0) over all lattices, one or a group of
//        up to three directions per launch (through per-vertex path tables,
//        the same values as the sequential passes); the transpose runs the
//        directions in reverse order.
//      slice: one thread per pixel gathers its d+1 vertex rows with 16-byte
//        loads into registers; the tile's input rows and per-pixel vertex ids
//        and weights are staged in LDS with contiguous loads, and the output
//        rows leave through LDS, so the pixel-major arrays move coalesced.
//    Optional launch shape: the same splats and slices by 16x16 pixel tiles
//    (tiles.hip), with each tile's distinct vertices staged in LDS.
//  - exact: the O(N^2) sum on the vector ALU, tiled through LDS (reference
//    mode for small images and for measuring the lattice's error).
//
// Vertex values are M x ld (ld = C rounded up to 16 bytes, zero padding).
// V[0] is the splat target and is kept all-zero between calls: the second
// blur launch clears it while the launches ping-pong between V[1] and V[2].

#include <algorithm>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

// ------------------------------------------------------------------ splat


// lane (chunk, c): V0[v][c] += sum w * Y[pix][c]; block b of a lattice takes
// its chunks b q .. b q + q - 1 (q = dense_splat_q: chunks of C lanes)
template <typename T>
__global__ void __launch_bounds__(256)
k_splat_gather(int C, int q, const T *__restrict__ Y, LatSet<T> ls) {
    const long long b0 = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x;
    int m = 0;   // uniform: each lattice's blocks start at a multiple of 256 lanes
    while (m + 1 < ls.nk && b0 >= ls.coff[m + 1]) ++m;
    const LatView<T> &L = ls.l[m];
    const int k = threadIdx.x / C;
    const int ch = int((b0 - ls.coff[m]) / 256) * q + k;
    if (k >= q || ch >= L.ndchunks) return;
    const int c = threadIdx.x - k * C;
    const int4 cd = L.dchunks[ch];
    T acc0 = T(0), acc1 = T(0), acc2 = T(0), acc3 = T(0);
    int i = cd.y;
    for (; i + 4 <= cd.z; i += 4) {   // four independent loads in flight
        acc0 += L.ent_w[i + 0] * Y[(size_t)L.ent_pix[i + 0] * C + c];
        acc1 += L.ent_w[i + 1] * Y[(size_t)L.ent_pix[i + 1] * C + c];
        acc2 += L.ent_w[i + 2] * Y[(size_t)L.ent_pix[i + 2] * C + c];
        acc3 += L.ent_w[i + 3] * Y[(size_t)L.ent_pix[i + 3] * C + c];
    }
    for (; i < cd.z; ++i) acc0 += L.ent_w[i] * Y[(size_t)L.ent_pix[i] * C + c];
    const T acc = (acc0 + acc1) + (acc2 + acc3);
    if (acc != T(0)) atomic_add(&L.V0[(size_t)cd.x * L.ld + c], acc);
}

// The same with the block's chunks staged in LDS: block b takes q <= 256 / C
// consecutive chunks (lane = chunk * C + channel, q U <= kSplatStage). Their (pixel, weight)
// pairs are copied to LDS with contiguous loads first, so that the only
// per-lane global loads left are those of the input values; the C lanes of a
// chunk would otherwise each load the same pair. With two lattices
// (pq0 + pq1 > 0) the blocks follow xcd_pair_block, 8 pq_m blocks for
// lattice m (the chunks are in first-pixel order), so that each XCD gathers
// one stretch of input rows for both lattices; blocks past a lattice's
// chunks do nothing.
template <typename T>
__global__ void __launch_bounds__(256)
k_splat_gather_lds(int C, int q, int U, const T *__restrict__ Y, LatSet<T> ls, int pq0,
                   int pq1) {
    __shared__ PairLds<T> sp[kSplatStage];
    __shared__ int4 scd[256];
    int m = 0, lb = 0;
    if (pq0 + pq1 > 0) {
        m = xcd_pair_block(blockIdx.x, pq0, pq1, lb);
    } else {
        const long long b0 = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x;
        while (m + 1 < ls.nk && b0 >= ls.coff[m + 1]) ++m;   // uniform
        lb = int((b0 - ls.coff[m]) / 256);
    }
    const LatView<T> &L = ls.l[m];
    const int ch0 = lb * q;
    const int nq = min(q, L.ndchunks - ch0);
    if (nq <= 0) return;   // uniform, before any barrier
    const int t = threadIdx.x;
    if (t < nq) scd[t] = L.dchunks[ch0 + t];
    const size_t base = (size_t)ch0 * U;   // the block's entries: one contiguous range
    for (int i = t; i < nq * U; i += 256) sp[i] = PairLds<T>{L.dpix[base + i], L.dw[base + i]};
    __syncthreads();
    const int k = t / C, c = t - (t / C) * C;
    if (k >= nq) return;
    const int4 cd = scd[k];
    const int n = cd.z - cd.y;
    const PairLds<T> *pk = sp + k * U;
    T acc0 = T(0), acc1 = T(0), acc2 = T(0), acc3 = T(0);
    int j = 0;
    for (; j + 4 <= n; j += 4) {
        const PairLds<T> e0 = pk[j], e1 = pk[j + 1], e2 = pk[j + 2], e3 = pk[j + 3];
        acc0 += e0.w * Y[(size_t)e0.i * C + c];
        acc1 += e1.w * Y[(size_t)e1.i * C + c];
        acc2 += e2.w * Y[(size_t)e2.i * C + c];
        acc3 += e3.w * Y[(size_t)e3.i * C + c];
    }
    for (; j < n; ++j) acc0 += pk[j].w * Y[(size_t)pk[j].i * C + c];
    const T acc = (acc0 + acc1) + (acc2 + acc3);
    if (acc != T(0)) atomic_add(&L.V0[(size_t)cd.x * L.ld + c], acc);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_splat_labels_lds(int C, int q, int U, const int32_t *__restrict__ labels,
                   LatSet<T> ls) {
    __shared__ PairLds<T> sp[kSplatStage];
    __shared__ int4 scd[256];
    splat_labels_block<T>(C, q, U, labels, ls,
                          (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x, sp, scd);
}

// One-hot input (pixel a is 1 at channel labels[a]): one wave per inverse-
// index chunk (all entries of one vertex v). Each lane takes an entry and
// adds its weight to an LDS histogram over the labels; the wave then adds
// the non-zero bins to V0[v][label], one global atomic per label present.
constexpr int kLabelBins = 256;   // labels per chunk histogram (L <= 256)

template <typename T>
__global__ void __launch_bounds__(256)
k_splat_labels_chunks(int C, const int32_t *__restrict__ labels, LatSet<T> ls) {
    __shared__ T bins[4][kLabelBins];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const long long chg = (long long)xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
    T *b = bins[wave];
    for (int l = lane; l < C; l += 64) b[l] = T(0);
    __syncthreads();
    const bool valid = chg < ls.choff[ls.nk];
    int m = 0;
    while (m + 1 < ls.nk && chg >= ls.choff[m + 1]) ++m;
    const LatView<T> &L = ls.l[m];
    int4 cd = make_int4(0, 0, 0, 0);
    if (valid) {
        cd = L.chunks[chg - ls.choff[m]];
        for (int i = cd.y + lane; i < cd.z; i += 64) {
            const int lab = labels[L.ent_pix[i]];
            if (lab >= 0 && lab < C) atomicAdd(&b[lab], L.ent_w[i]);
        }
    }
    __syncthreads();
    if (valid)
        for (int l = lane; l < C; l += 64) {
            const T s = b[l];
            if (s != T(0)) atomic_add(&L.V0[(size_t)cd.x * L.ld + l], s);
        }
}

// ------------------------------------------------------------------- blur

__device__ __forceinline__ float4 blur3(float4 c, float4 p, float4 q) {
    return make_float4(0.5f * c.x + 0.25f * (p.x + q.x), 0.5f * c.y + 0.25f * (p.y + q.y),
                       0.5f * c.z + 0.25f * (p.z + q.z), 0.5f * c.w + 0.25f * (p.w + q.w));
}
__device__ __forceinline__ double2 blur3(double2 c, double2 p, double2 q) {
    return make_double2(0.5 * c.x + 0.25 * (p.x + q.x), 0.5 * c.y + 0.25 * (p.y + q.y));
}

// pass p of every lattice with d >= p, over 16-byte vectors of the vertex
// rows flattened over sum_m M_m x ld / (16 / sizeof(T)); a block covers
// blockDim * vpt consecutive vectors, thread t taking t, t + blockDim, ...
// so that every access stays coalesced and vpt loads are in flight per thread
template <typename T>
__device__ __forceinline__ void blur_vector(const LatSet<T> &ls, int pass,
                                            int reverse, long long e) {
    using V = typename Vec16<T>::type;
    constexpr int vw = Vec16<T>::n;
    int m = 0;
    while (m + 1 < ls.nk && e >= ls.off[m + 1] / vw) ++m;
    const LatView<T> &L = ls.l[m];
    const unsigned G = unsigned(L.ld / vw);
    const unsigned r = unsigned(e - ls.off[m] / vw);
    V zero;
    for (int i = 0; i < vw; ++i) reinterpret_cast<T *>(&zero)[i] = T(0);
    if (pass > L.d) {
        if (pass == 1) reinterpret_cast<V *>(L.V0)[r] = zero;
        return;
    }
    const int v = int(r / G);
    const int g = int(r - unsigned(v) * G);
    const int j = reverse ? (L.d - pass) : pass;
    const V *src = reinterpret_cast<const V *>((pass == 0) ? L.V0 : ((pass & 1) ? L.V1 : L.V2));
    V *dst = reinterpret_cast<V *>((pass & 1) ? L.V2 : L.V1);
    const int np = L.nbr[((size_t)j * L.M + v) * 2 + 0];
    const int nm = L.nbr[((size_t)j * L.M + v) * 2 + 1];
    const V vp = np >= 0 ? src[(size_t)np * G + g] : zero;
    const V vm = nm >= 0 ? src[(size_t)nm * G + g] : zero;
    dst[r] = blur3(src[r], vp, vm);
    if (pass == 1) reinterpret_cast<V *>(L.V0)[r] = zero;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_blur_pass(LatSet<T> ls, int pass, int reverse, long long total, int vpt) {
    // XCD-contiguous ranges of vertex rows: the rows a block reads around its
    // own (lattice neighbours of nearby vertices) stay in one XCD's L2
    const long long base =
        (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x * vpt + threadIdx.x;
    for (int q = 0; q < vpt; ++q) {
        const long long e = base + (long long)q * blockDim.x;
        if (e >= total) return;
        blur_vector<T>(ls, pass, reverse, e);
    }
}

// Grouped blur: G consecutive directions in one launch. For the directions
// j_1..j_G of a group (in the order they are applied) the output is
//   out[v] = sum over a in {0, +1, -1}^G of prod_k c(a_k) V[x_0],
//   x_G = v, x_{k-1} = x_k + a_k u_{j_k},  c(0) = 1/2, c(+-1) = 1/4,
// over the paths whose points x_k all exist: exactly the G sequential passes
// (a point missing in between reads as 0 there). The endpoints x_0 of the 3^G
// paths of every vertex are tabulated once per lattice (k_group_table); a
// group of the last launch that has fewer than G directions tabulates only
// the staying path for the missing ones, and the launch rescales by 2 per
// missing direction.

__global__ void k_group_table(int M, const int32_t *__restrict__ nbr, int G,
                              int j1, int j2, int j3, int npass,
                              int32_t *__restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= M) return;
    int P = 1;
    for (int k = 0; k < G; ++k) P *= 3;
    const int js[3] = {j1, j2, j3};
    for (int path = 0; path < P; ++path) {
        int x = v, code = path, pw = P / 3;
        bool ok = true;
        // digit k (k = G..1, most significant first) is the step along j_k
        for (int k = G; k >= 1 && ok; --k) {
            const int a = code / pw;
            code -= a * pw;
            pw /= 3;
            if (a == 0) continue;
            if (k > npass) {
                ok = false;
                break;
            }
            x = nbr[((size_t)js[k - 1] * M + x) * 2 + (a - 1)];
            ok = x >= 0;
        }
        out[(size_t)v * P + path] = ok ? x : -1;
    }
}


template <typename T, int G>
__global__ void __launch_bounds__(256)
k_blur_group(LatSet<T> ls, int grp, long long total, int vpt) {
    const long long base =
        (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x * vpt + threadIdx.x;
    for (int q = 0; q < vpt; ++q) {
        const long long e = base + (long long)q * blockDim.x;
        if (e >= total) return;
        blur_group_vector<T, G>(ls, grp, e);
    }
}

template <typename T>
__global__ void k_zero_rows(LatSet<T> ls, long long total) {
    using V = typename Vec16<T>::type;
    constexpr int vw = Vec16<T>::n;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int m = 0;
    while (m + 1 < ls.nk && e >= ls.off[m + 1] / vw) ++m;
    V zero;
    for (int i = 0; i < vw; ++i) reinterpret_cast<T *>(&zero)[i] = T(0);
    reinterpret_cast<V *>(ls.l[m].V0)[e - ls.off[m] / vw] = zero;
}

// ------------------------------------------------------------------ slice

enum { kSliceRaw = 0, kSliceQP = 1 };

// One thread per pixel.
//   raw: out = K'Y            = slice - wsum * Y
//   qp:  out = (Psi + D) Y    = (K'Y) mu^T + d * Y, d_a(i) = mabs_i r_a
// `pre` (optional) holds K'Y already (exact mode): then no lattice is read.
template <typename T, int LMAX, int MODE>
__global__ void __launch_bounds__(RowTile<T>::kPix, 2)
k_slice_rows(int N, int C, const T *__restrict__ Y, const T *__restrict__ pre,
             LatSet<T> ls, T wsum, const T *__restrict__ mu,
             const T *__restrict__ mabs, const T *__restrict__ r,
             T *__restrict__ out) {
    constexpr int TP = RowTile<T>::kPix;
    __shared__ __align__(16) T lds[TP * (LMAX | 1)];
    __shared__ int32_t sid[TP * kCorners52];
    __shared__ T swc[TP * kCorners52];
    __shared__ T smu[MODE == kSliceQP ? LMAX * LMAX : 1];
    if (MODE == kSliceQP) {
        for (int i = threadIdx.x; i < C * C; i += TP)
            smu[(i / C) * LMAX + (i % C)] = mu[i];
        __syncthreads();
    }
    for (long long p0 = (long long)xcd_block(blockIdx.x, gridDim.x) * TP; p0 < N;
         p0 += (long long)gridDim.x * TP) {
        const int np = (int)min((long long)TP, N - p0);
        const long long a = p0 + threadIdx.x;
        const bool act = (int)threadIdx.x < np;
        T y[LMAX], q[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) y[j] = T(0), q[j] = T(0);
        if (pre) {
            tile_load<T, LMAX, TP>(pre, p0, np, C, lds, q);
            tile_load<T, LMAX, TP>(Y, p0, np, C, lds, y);
        } else {
            // the tile of Y goes to LDS first, while few registers are live,
            // and its loads overlap the gathers of the slice
            if (ls.shape52) stage_corners52<T, TP>(ls, p0, np, sid, swc);
            tile_copy_in<T, TP, LMAX>(Y + p0 * C, np * C, C, lds);
            if (ls.shape52) {
                __syncthreads();
                if (act) slice_pixel52_staged<T, LMAX, TP>(ls, threadIdx.x, C, sid, swc, q);
            } else if (act) {
                slice_pixel<T, LMAX>(ls, a, C, q);
            }
            __syncthreads();
            tile_read_own<T, LMAX>(np, C, lds, y);   // each thread its own row
        }
        if (!pre) {
#pragma unroll
            for (int j = 0; j < LMAX; ++j) q[j] -= wsum * y[j];
        }
        if (MODE == kSliceRaw) {
            tile_store<T, LMAX, TP>(out, p0, np, C, lds, q);
        } else {
            T o[LMAX];
            const T ra = act ? r[a] : T(0);
#pragma unroll
            for (int i = 0; i < LMAX; ++i) {
                T p = T(0);
#pragma unroll
                for (int j = 0; j < LMAX; ++j)
                    if (i < C && j < C) p += smu[i * LMAX + j] * q[j];
                o[i] = (i < C) ? p + mabs[i] * ra * y[i] : T(0);
            }
            tile_store<T, LMAX, TP>(out, p0, np, C, lds, o);
        }
    }
}

// generic slice for C > kRowMaxC: one lane per (pixel, channel)
template <typename T>
__global__ void __launch_bounds__(256)
k_slice_raw_flat(int N, int C, const T *__restrict__ in, T *__restrict__ out,
                 LatSet<T> ls, T wsum) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * C) return;
    const long long a = (long long)(e / C);
    const int c = int(e - (size_t)a * C);
    T acc = T(0);
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int D1 = L.d + 1;
        for (int k = 0; k < D1; ++k) {
            const int id = L.vid[a * D1 + k];
            if (id >= 0)
                acc += L.wg * L.w[a * D1 + k] * L.Vf[(size_t)id * L.ld + c];
        }
    }
    out[e] = acc - wsum * in[e];
}

// ------------------------------------------------------------------ exact

constexpr int kExactTile = 128;
constexpr int kExactMaxF = 16;   // sum of feature dimensions over the kernels
constexpr int kExactCB = 8;      // channels per pass

// out_a[c0 .. c0+CB) = sum_{b != a} sum_m w_m exp(-|f_a - f_b|^2/2) in_b
template <typename T>
__global__ void __launch_bounds__(kExactTile)
k_exact(int N, int C, int c0, const T *__restrict__ in, T *__restrict__ out,
        ExactSet<T> ex) {
    __shared__ T sf[kExactTile][kExactMaxF];
    __shared__ T sv[kExactTile][kExactCB];
    const int a = blockIdx.x * kExactTile + threadIdx.x;
    T fa[kExactMaxF];
    for (int j = 0; j < kExactMaxF; ++j) fa[j] = T(0);
    if (a < N)
        for (int m = 0; m < ex.nk; ++m)
            for (int j = 0; j < ex.d[m]; ++j)
                fa[ex.off[m] + j] = ex.f[m][(size_t)a * ex.d[m] + j];
    T acc[kExactCB];
#pragma unroll
    for (int c = 0; c < kExactCB; ++c) acc[c] = T(0);
    const int cn = min(kExactCB, C - c0);
    for (int b0 = 0; b0 < N; b0 += kExactTile) {
        const int b = b0 + threadIdx.x;
        if (b < N) {
            for (int m = 0; m < ex.nk; ++m)
                for (int j = 0; j < ex.d[m]; ++j)
                    sf[threadIdx.x][ex.off[m] + j] = ex.f[m][(size_t)b * ex.d[m] + j];
            for (int c = 0; c < kExactCB; ++c)
                sv[threadIdx.x][c] = c < cn ? in[(size_t)b * C + c0 + c] : T(0);
        }
        __syncthreads();
        const int nb = min(kExactTile, N - b0);
        for (int t = 0; t < nb; ++t) {
            if (b0 + t == a) continue;
            T kab = T(0);
            for (int m = 0; m < ex.nk; ++m) {
                T r2 = T(0);
                for (int j = ex.off[m]; j < ex.off[m + 1]; ++j) {
                    const T df = fa[j] - sf[t][j];
                    r2 += df * df;
                }
                kab += ex.w[m] * exp(T(-0.5) * r2);
            }
#pragma unroll
            for (int c = 0; c < kExactCB; ++c) acc[c] += kab * sv[t][c];
        }
        __syncthreads();
    }
    if (a < N)
        for (int c = 0; c < cn; ++c) out[(size_t)a * C + c0 + c] = acc[c];
}

// ------------------------------------------------------- tile kernels

// Tile splats: one block per 2-D pixel tile. Per lattice, the tile's
// pixel-vertex pairs grouped by slot (each slot one distinct vertex of the
// tile) are staged in LDS together with the slot boundaries; lane task
// (slot, c) sums its slot's pairs from LDS and adds the sum to the vertex row
// with one global atomic. Each input value is read from global memory once.

// pairs of one lattice in one tile: at most d + 1 <= kMaxD1 per pixel
constexpr int kTilePairs = kTilePix * kMaxD1;

// Stage the pairs [e0, e0 + ne) of one lattice and its slot offsets (ns + 1,
// relative to e0) in LDS. Loads of a thread are issued before its stores.
template <typename T>
__device__ __forceinline__ void tile_stage_pairs(const LatView<T> &L, int s0, int ns,
                                                 int e0, int ne, uint8_t *spx, T *sw,
                                                 int *sof) {
    constexpr int K = kTilePairs / kTilePix;
    uint8_t px[K];
    T w[K];
    int of[K + 1];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = (int)threadIdx.x + k * kTilePix;
        const int ic = i < ne ? i : 0;
        px[k] = ne > 0 ? L.sr_pix[e0 + ic] : uint8_t(0);
        w[k] = ne > 0 ? L.sr_w[e0 + ic] : T(0);
    }
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        const int i = (int)threadIdx.x + k * kTilePix;
        of[k] = L.sr_off[s0 + (i <= ns ? i : ns)];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = (int)threadIdx.x + k * kTilePix;
        if (i < ne) {
            spx[i] = px[k];
            sw[i] = w[k];
        }
    }
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        const int i = (int)threadIdx.x + k * kTilePix;
        if (i <= ns) sof[i] = of[k] - e0;
    }
}

// LDS of the tile splats: staged values (kTilePix rows of stride C | 1, or
// one label per pixel), then pair weights, slot offsets and pair pixels
template <typename T>
size_t tile_splat_lds(int C) {
    return (size_t)kTilePix * (C | 1) * sizeof(T) + (size_t)kTilePairs * sizeof(T) +
           (size_t)(kTilePairs + 1) * 4 + kTilePairs;
}

template <typename T>
__global__ void __launch_bounds__(kTilePix)
k_tile_splat(int C, const T *__restrict__ Y, LatSet<T> ls,
             const int4 *__restrict__ tiles) {
    extern __shared__ __align__(16) unsigned char tile_smem[];
    const int LS = C | 1;
    T *ys = reinterpret_cast<T *>(tile_smem);
    T *sw = ys + kTilePix * LS;
    int *sof = reinterpret_cast<int *>(sw + kTilePairs);
    uint8_t *spx = reinterpret_cast<uint8_t *>(sof + kTilePairs + 1);
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const int4 td = tiles[t];
    tile2_in<T, kTilePix>(Y, td, C, ys, LS);
    const float invC = 1.0f / float(C);
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int s0 = L.ts_off[t], ns = L.ts_off[t + 1] - s0;
        const int e0 = L.sr_off[s0], ne = L.sr_off[s0 + ns] - e0;
        tile_stage_pairs<T>(L, s0, ns, e0, ne, spx, sw, sof);
        __syncthreads();
        for (int task = threadIdx.x; task < ns * C; task += kTilePix) {
            const int sl = int((float(task) + 0.5f) * invC);
            const int c = task - sl * C;
            const int b = sof[sl], e = sof[sl + 1];
            T acc0 = T(0), acc1 = T(0);
            int j = b;
            for (; j + 2 <= e; j += 2) {
                acc0 += sw[j] * ys[spx[j] * LS + c];
                acc1 += sw[j + 1] * ys[spx[j + 1] * LS + c];
            }
            if (j < e) acc0 += sw[j] * ys[spx[j] * LS + c];
            const T acc = acc0 + acc1;
            if (acc != T(0)) atomic_add(&L.V0[(size_t)L.ts_vid[s0 + sl] * L.ld + c], acc);
        }
        __syncthreads();
    }
}

// One-hot input: the tile's labels are staged instead of rows, and lane task
// (slot, c) adds up the weights of its slot's pairs whose pixel has label c.
template <typename T>
__global__ void __launch_bounds__(kTilePix)
k_tile_labels(int C, const int32_t *__restrict__ labels, LatSet<T> ls,
              const int4 *__restrict__ tiles) {
    extern __shared__ __align__(16) unsigned char tile_smem[];
    int *labs = reinterpret_cast<int *>(tile_smem);
    T *sw = reinterpret_cast<T *>(tile_smem + kTilePix * 8);
    int *sof = reinterpret_cast<int *>(sw + kTilePairs);
    uint8_t *spx = reinterpret_cast<uint8_t *>(sof + kTilePairs + 1);
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const int4 td = tiles[t];
    {
        const int i = threadIdx.x / kTileW, px = threadIdx.x % kTileW;
        labs[threadIdx.x] = (i < td.z && px < td.w)
                                ? labels[(size_t)td.x + (size_t)i * td.y + px] : -1;
    }
    const float invC = 1.0f / float(C);
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int s0 = L.ts_off[t], ns = L.ts_off[t + 1] - s0;
        const int e0 = L.sr_off[s0], ne = L.sr_off[s0 + ns] - e0;
        tile_stage_pairs<T>(L, s0, ns, e0, ne, spx, sw, sof);
        __syncthreads();
        for (int task = threadIdx.x; task < ns * C; task += kTilePix) {
            const int sl = int((float(task) + 0.5f) * invC);
            const int c = task - sl * C;
            const int b = sof[sl], e = sof[sl + 1];
            T acc0 = T(0), acc1 = T(0);
            int j = b;
            for (; j + 2 <= e; j += 2) {
                acc0 += labs[spx[j]] == c ? sw[j] : T(0);
                acc1 += labs[spx[j + 1]] == c ? sw[j + 1] : T(0);
            }
            if (j < e) acc0 += labs[spx[j]] == c ? sw[j] : T(0);
            const T acc = acc0 + acc1;
            if (acc != T(0)) atomic_add(&L.V0[(size_t)L.ts_vid[s0 + sl] * L.ld + c], acc);
        }
        __syncthreads();
    }
}

// The slice of pixel a from a tile's slot rows staged in LDS, for two
// lattices of compile-time dimensions DA and DB: the slots and weights of
// all pairs are loaded first, then every row is read (slots beyond the
// staged ones from global memory).
template <typename T, int LMAX, int DA, int DB>
__device__ __forceinline__ void tile_slice_pixel(const LatSet<T> &ls, size_t a, int C,
                                                 const T *rows, int ld, const int *base,
                                                 const int *nin, const int *s0,
                                                 T (&q)[LMAX]) {
    int sa[DA + 1], sb[DB + 1];
    T wa[DA + 1], wb[DB + 1];
    const LatView<T> &A = ls.l[0];
    const LatView<T> &B = ls.l[1];
#pragma unroll
    for (int k = 0; k <= DA; ++k) {
        sa[k] = A.tr_slot[a * (DA + 1) + k];
        wa[k] = A.wg * A.w[a * (DA + 1) + k];
    }
#pragma unroll
    for (int k = 0; k <= DB; ++k) {
        sb[k] = B.tr_slot[a * (DB + 1) + k];
        wb[k] = B.wg * B.w[a * (DB + 1) + k];
    }
#pragma unroll
    for (int k = 0; k <= DA; ++k) {
        if (sa[k] == 0xffff) continue;
        if (sa[k] < nin[0])
            axpy_row<LMAX>(q, wa[k], rows + (size_t)(base[0] + sa[k]) * ld, C);
        else
            axpy_row<LMAX>(q, wa[k], A.Vf + (size_t)A.ts_vid[s0[0] + sa[k]] * ld, C);
    }
#pragma unroll
    for (int k = 0; k <= DB; ++k) {
        if (sb[k] == 0xffff) continue;
        if (sb[k] < nin[1])
            axpy_row<LMAX>(q, wb[k], rows + (size_t)(base[1] + sb[k]) * ld, C);
        else
            axpy_row<LMAX>(q, wb[k], B.Vf + (size_t)B.ts_vid[s0[1] + sb[k]] * ld, C);
    }
}

// Slice (raw or QP) of one tile per block, one thread per pixel. The tile's
// slot rows of every lattice are staged in LDS first (at most `cap` rows;
// slots beyond them are read from global memory) together with the tile's
// rows of Y; each pixel then adds its d+1 rows per lattice from LDS, and the
// results leave through LDS, coalesced.
template <typename T, int LMAX, int MODE>
__global__ void __launch_bounds__(kTilePix)
k_tile_slice(int C, const T *__restrict__ Y, LatSet<T> ls,
             const int4 *__restrict__ tiles, int cap, T wsum,
             const T *__restrict__ mu, const T *__restrict__ mabs,
             const T *__restrict__ r, T *__restrict__ out) {
    using V = typename Vec16<T>::type;
    constexpr int vw = Vec16<T>::n;
    extern __shared__ __align__(16) unsigned char tile_smem[];
    const int LS = C | 1;
    T *py = reinterpret_cast<T *>(tile_smem);   // kTilePix x LS: Y, then out
    T *rows = py + kTilePix * LS;                // cap x ld
    rows = reinterpret_cast<T *>((reinterpret_cast<uintptr_t>(rows) + 15) & ~uintptr_t(15));
    __shared__ T smu[MODE == kSliceQP ? LMAX * LMAX : 1];
    if (MODE == kSliceQP)
        for (int i = threadIdx.x; i < C * C; i += kTilePix)
            smu[(i / C) * LMAX + (i % C)] = mu[i];
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const int4 td = tiles[t];
    const int ld = ls.l[0].ld;
    int base[DCRF_MAXK], nin[DCRF_MAXK], s0[DCRF_MAXK];
    int used = 0;
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        s0[m] = L.ts_off[t];
        const int ns = L.ts_off[t + 1] - s0[m];
        nin[m] = min(ns, cap - used);
        base[m] = used;
        used += nin[m];
    }
    {
        // batches of kB vectors per thread: every vertex id of a batch is
        // loaded, then every row vector, then all are stored
        constexpr int kB = 8;
        const int G = ld / vw;
        for (int m = 0; m < ls.nk; ++m) {
            const LatView<T> &L = ls.l[m];
            const int cnt = nin[m] * G;
            for (int i0 = 0; i0 < cnt; i0 += kTilePix * kB) {
                int vid[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int idx = i0 + u * kTilePix + (int)threadIdx.x;
                    vid[u] = idx < cnt ? L.ts_vid[s0[m] + idx / G] : -1;
                }
                V v[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int idx = i0 + u * kTilePix + (int)threadIdx.x;
                    if (vid[u] >= 0)
                        v[u] = reinterpret_cast<const V *>(L.Vf)[(size_t)vid[u] * G +
                                                                 (idx - (idx / G) * G)];
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int idx = i0 + u * kTilePix + (int)threadIdx.x;
                    if (vid[u] >= 0)
                        reinterpret_cast<V *>(rows)[(size_t)base[m] * G + idx] = v[u];
                }
            }
        }
    }
    tile2_in<T, kTilePix>(Y, td, C, py, LS);
    __syncthreads();
    const int i = threadIdx.x / kTileW, px = threadIdx.x % kTileW;
    const bool act = i < td.z && px < td.w;
    if (act) {
        const size_t a = (size_t)td.x + (size_t)i * td.y + px;
        T *prow = py + threadIdx.x * LS;
        T q[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) q[j] = T(0);
        if (ls.shape52) {
            tile_slice_pixel<T, LMAX, 5, 2>(ls, a, C, rows, ld, base, nin, s0, q);
        } else {
            for (int m = 0; m < ls.nk; ++m) {
                const LatView<T> &L = ls.l[m];
                const int D1 = L.d + 1;
                for (int k = 0; k < D1; ++k) {
                    const int sl = L.tr_slot[a * D1 + k];
                    if (sl == 0xffff) continue;
                    const T w = L.wg * L.w[a * D1 + k];
                    if (sl < nin[m])
                        axpy_row<LMAX>(q, w, rows + (size_t)(base[m] + sl) * ld, C);
                    else
                        axpy_row<LMAX>(q, w, L.Vf + (size_t)L.ts_vid[s0[m] + sl] * ld, C);
                }
            }
        }
        T y[LMAX];
#pragma unroll
        for (int j = 0; j < LMAX; ++j) y[j] = (j < C) ? prow[j] : T(0);
#pragma unroll
        for (int j = 0; j < LMAX; ++j) q[j] -= wsum * y[j];
        if (MODE == kSliceRaw) {
#pragma unroll
            for (int j = 0; j < LMAX; ++j)
                if (j < C) prow[j] = q[j];
        } else {
            const T ra = r[a];
#pragma unroll
            for (int i2 = 0; i2 < LMAX; ++i2) {
                if (i2 < C) {
                    T p = T(0);
#pragma unroll
                    for (int j = 0; j < LMAX; ++j)
                        if (j < C) p += smu[i2 * LMAX + j] * q[j];
                    prow[i2] = p + mabs[i2] * ra * y[i2];
                }
            }
        }
    }
    __syncthreads();
    tile2_out<T, kTilePix>(out, td, C, py, LS);
}

int row_grid(dcrf_ctx *ctx, int tp) {
    return std::max(1, std::min(ceil_div(ctx->N, tp), 4096));
}

template <typename T>
void exact_t(dcrf_ctx *ctx, const T *in, T *out, int C) {
    ExactSet<T> ex = make_exact_set<T>(ctx);
    if (ex.off[ex.nk] > kExactMaxF)
        fail(DCRF_EUNSUPPORTED, "exact filter supports at most 16 feature "
                                "dimensions over all kernels");
    for (int c0 = 0; c0 < C; c0 += kExactCB)
        hipLaunchKernelGGL((k_exact<T>), dim3(ceil_div(ctx->N, kExactTile)),
                           dim3(kExactTile), 0, ctx->stream, ctx->N, C, c0, in,
                           out, ex);
    DCRF_CHECK_LAUNCH();
}

// sum over b != a of k_m(a, b) in_b for kernel m alone (weight 1)
template <typename T>
void exact_kernel_t(dcrf_ctx *ctx, int m, const T *in, T *out, int C) {
    const ExactSet<T> all = make_exact_set<T>(ctx);
    ExactSet<T> ex{};
    ex.nk = 1;
    ex.f[0] = all.f[m];
    ex.d[0] = all.d[m];
    ex.off[0] = 0;
    ex.off[1] = all.d[m];
    ex.w[0] = T(1);
    for (int c0 = 0; c0 < C; c0 += kExactCB)
        hipLaunchKernelGGL((k_exact<T>), dim3(ceil_div(ctx->N, kExactTile)),
                           dim3(kExactTile), 0, ctx->stream, ctx->N, C, c0, in,
                           out, ex);
    DCRF_CHECK_LAUNCH();
}

constexpr size_t kTileLds = 56 * 1024;   // dynamic LDS of the tile slices

// whether the per-tile kernels serve C channels: each lattice's slots of a
// tile must fit the splat's LDS partial rows
template <typename T>
bool use_tiles(const dcrf_ctx *ctx, int C) {
    if (!(ctx->tile_mode && ctx->ntiles > 0 && C <= kRowMaxC)) return false;
    // the slice stages the tile's pixel rows and at least one slot row
    const size_t slice = (size_t)kTilePix * (C | 1) * sizeof(T) + 16 +
                         (size_t)row_stride(C, sizeof(T)) * sizeof(T);
    return tile_splat_lds<T>(C) <= kTileLds && slice <= kTileLds;
}

// splat of the dense N x C input into V0 of every lattice of ls
template <typename T>
void splat_set(dcrf_ctx *ctx, const LatSet<T> &ls, const T *in, int C) {
    const hipStream_t s = ctx->stream;
    ProfScope ps(ctx, PROF_SPLAT);
    if (use_tiles<T>(ctx, C)) {
        DCRF_PLAUNCH(ps, (k_tile_splat<T>), dim3(ctx->ntiles), dim3(kTilePix),
                     tile_splat_lds<T>(C), s, C, in, ls, ctx->tiles.as<int4>());
        DCRF_CHECK_LAUNCH();
        return;
    }
    const long long total = ls.coff[ls.nk];
    if (total == 0) return;
    if (C > 256) fail(DCRF_EUNSUPPORTED, "the dense splat takes at most 256 channels");
    const dim3 grid(ceil_div(total, 256));
    const int q = dense_splat_q(ctx, C);
    if (ctx->splat_lds && ls.nk == 2) {
        int pq[2];
        for (int m = 0; m < 2; ++m)
            pq[m] = (int)ceil_div(ceil_div((long long)ls.l[m].ndchunks, (long long)q), 8ll);
        DCRF_PLAUNCH(ps, (k_splat_gather_lds<T>), dim3(8 * (pq[0] + pq[1])), dim3(256), 0,
                     s, C, q, ctx->dense_chunk, in, ls, pq[0], pq[1]);
    } else if (ctx->splat_lds)
        DCRF_PLAUNCH(ps, (k_splat_gather_lds<T>), grid, dim3(256), 0, s, C, q,
                           ctx->dense_chunk, in, ls, 0, 0);
    else
        DCRF_PLAUNCH(ps, (k_splat_gather<T>), grid, dim3(256), 0, s, C, q, in, ls);
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void splat_dense_t(dcrf_ctx *ctx, const T *in, int C) {
    ensure_vertex_buffers(ctx, C);
    LatSet<T> ls = make_lat_set<T>(ctx, C);
    splat_set<T>(ctx, ls, in, C);
}

template <typename T>
void splat_labels_t(dcrf_ctx *ctx, const int32_t *labels, int L) {
    if (L > kLabelBins) fail(DCRF_EUNSUPPORTED, "more than 256 labels");
    ensure_vertex_buffers(ctx, L);
    LatSet<T> ls = make_lat_set<T>(ctx, L);
    ProfScope ps(ctx, PROF_SPLAT_LABELS);
    if (use_tiles<T>(ctx, 1)) {
        DCRF_PLAUNCH(ps, (k_tile_labels<T>), dim3(ctx->ntiles), dim3(kTilePix),
                     (size_t)kTilePix * 8 + tile_splat_lds<T>(1) - (size_t)kTilePix * sizeof(T),
                     ctx->stream, L, labels, ls, ctx->tiles.as<int4>());
        DCRF_CHECK_LAUNCH();
        return;
    }
    if (ctx->splat_lds) {
        const long long total = ls.coff[ls.nk];
        if (total == 0) return;
        DCRF_PLAUNCH(ps, (k_splat_labels_lds<T>), dim3(ceil_div(total, 256)), dim3(256),
                           0, ctx->stream, L, dense_splat_q(ctx, L), ctx->dense_chunk,
                           labels, ls);
        DCRF_CHECK_LAUNCH();
        return;
    }
    const long long total = ls.choff[ls.nk];
    if (total == 0) return;
    DCRF_PLAUNCH(ps, (k_splat_labels_chunks<T>), dim3(ceil_div(total, 4)),
                       dim3(256), 0, ctx->stream, L, labels, ls);
    DCRF_CHECK_LAUNCH();
}

// path tables of the grouped blur for the context's group size
void ensure_group_tables(dcrf_ctx *ctx, int G, bool adjoint) {
    const int dir = adjoint ? 1 : 0;
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &L = ctx->lat[m];
        if (L.gtab_G[dir] == G || L.M == 0) continue;
        int P = 1;
        for (int k = 0; k < G; ++k) P *= 3;
        const int ng = blur_launches(L.d, G);
        L.gtab[dir].ensure((size_t)ng * L.M * P * 4, ctx->stream);
        for (int grp = 0; grp < ng; ++grp) {
            int js[3] = {0, 0, 0};
            int np = 0;
            for (int k = 0; k < G; ++k) {
                const int pass = grp * G + k;   // position in the blur order
                if (pass > L.d) break;
                js[k] = adjoint ? (L.d - pass) : pass;
                ++np;
            }
            hipLaunchKernelGGL(k_group_table, dim3(ceil_div(L.M, 256)), dim3(256), 0,
                               ctx->stream, L.M, L.nbr.as<int32_t>(), G, js[0], js[1],
                               js[2], np,
                               L.gtab[dir].as<int32_t>() + (size_t)grp * L.M * P);
        }
        DCRF_CHECK_LAUNCH();
        L.gtab_G[dir] = G;
    }
}

// The blur of every lattice of `ls` (its views index the context's lattices
// lat[first], lat[first+1], ...), one launch per direction or per group of
// ctx->blur_group directions.
template <typename T>
void blur_launch(dcrf_ctx *ctx, LatSet<T> &ls, int first, bool adjoint) {
    const long long total = ls.off[ls.nk] / Vec16<T>::n;
    if (total == 0) return;
    const int bs = ctx->blur_block, vpt = ctx->blur_vpt, G = ctx->blur_group;
    const dim3 grid(ceil_div(total, (long long)bs * vpt));
    int nl = 0;
    for (int m = 0; m < ls.nk; ++m) nl = std::max(nl, ls.l[m].ngrp);
    if (G == 1) {
        for (int p = 0; p < nl; ++p) {
            ProfScope ps(ctx, PROF_BLUR);
            DCRF_PLAUNCH(ps, (k_blur_pass<T>), grid, dim3(bs), 0, ctx->stream, ls, p,
                               adjoint ? 1 : 0, total, vpt);
        }
    } else {
        ensure_group_tables(ctx, G, adjoint);
        for (int m = 0; m < ls.nk; ++m)
            ls.l[m].gt = ctx->lat[first + m].gtab[adjoint ? 1 : 0].as<int32_t>();
        for (int grp = 0; grp < nl; ++grp) {
            ProfScope ps(ctx, PROF_BLUR);
            if (G == 2)
                DCRF_PLAUNCH(ps, (k_blur_group<T, 2>), grid, dim3(bs), 0, ctx->stream,
                                   ls, grp, total, vpt);
            else
                DCRF_PLAUNCH(ps, (k_blur_group<T, 3>), grid, dim3(bs), 0, ctx->stream,
                                   ls, grp, total, vpt);
        }
    }
    if (nl == 1)   // no second launch cleared the splat target
        hipLaunchKernelGGL((k_zero_rows<T>), dim3(ceil_div(total, 256)), dim3(256), 0,
                           ctx->stream, ls, total);
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void blur_all_t(dcrf_ctx *ctx, int C, bool adjoint) {
    LatSet<T> ls = make_lat_set<T>(ctx, C);
    blur_launch<T>(ctx, ls, 0, adjoint);
}

// LDS rows for the slot rows of one tile in the tile slices
template <typename T>
int tile_slice_cap(const dcrf_ctx *ctx, const LatSet<T> &ls, int first, int C) {
    int mx = 0;
    for (int m = 0; m < ls.nk; ++m) mx += ctx->lat[first + m].max_tile_slots;
    const int ld = row_stride(C, sizeof(T));
    const size_t pix = (size_t)kTilePix * (C | 1) * sizeof(T) + 16;
    const size_t room = kTileLds > pix ? kTileLds - pix : 0;
    return std::max(1, std::min<int>(mx, int(room / (ld * sizeof(T)))));
}

template <typename T>
void slice_set(dcrf_ctx *ctx, const LatSet<T> &ls, int first, const T *Y,
               const T *pre, int C, T wsum, const T *mu, const T *mabs, T *out,
               bool qp) {
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    const T *r = ctx->r.as<T>();
    constexpr int TP = RowTile<T>::kPix;
    if (!pre && use_tiles<T>(ctx, C)) {
        ProfScope ps(ctx, qp ? PROF_SLICE_QP : PROF_SLICE);
        const int cap = tile_slice_cap<T>(ctx, ls, first, C);
        const size_t lds = (size_t)kTilePix * (C | 1) * sizeof(T) + 16 +
                           (size_t)cap * row_stride(C, sizeof(T)) * sizeof(T);
        DCRF_DISPATCH_ROWS(C, {
            if (qp)
                DCRF_PLAUNCH(ps, (k_tile_slice<T, LMAX, kSliceQP>), dim3(ctx->ntiles),
                                   dim3(kTilePix), lds, s, C, Y, ls,
                                   ctx->tiles.as<int4>(), cap, wsum, mu, mabs, r, out);
            else
                DCRF_PLAUNCH(ps, (k_tile_slice<T, LMAX, kSliceRaw>), dim3(ctx->ntiles),
                                   dim3(kTilePix), lds, s, C, Y, ls,
                                   ctx->tiles.as<int4>(), cap, wsum, mu, mabs, r, out);
        });
        DCRF_CHECK_LAUNCH();
        return;
    }
    if (C <= kRowMaxC) {
        ProfScope ps(ctx, qp ? PROF_SLICE_QP : PROF_SLICE);
        DCRF_DISPATCH_ROWS(C, {
            if (qp)
                DCRF_PLAUNCH(ps, (k_slice_rows<T, LMAX, kSliceQP>),
                                   dim3(row_grid(ctx, TP)), dim3(TP), 0, s, N, C,
                                   Y, pre, ls, wsum, mu, mabs, r, out);
            else
                DCRF_PLAUNCH(ps, (k_slice_rows<T, LMAX, kSliceRaw>),
                                   dim3(row_grid(ctx, TP)), dim3(TP), 0, s, N, C,
                                   Y, pre, ls, wsum, mu, mabs, r, out);
        });
        DCRF_CHECK_LAUNCH();
        return;
    }
    if (qp) fail(DCRF_EUNSUPPORTED, "more than 32 labels");
    if (pre) {
        DCRF_TRY_HIP(hipMemcpyAsync(out, pre, (size_t)N * C * sizeof(T),
                                    hipMemcpyDeviceToDevice, s));
        return;
    }
    ProfScope ps(ctx, PROF_SLICE);
    DCRF_PLAUNCH(ps, (k_slice_raw_flat<T>), dim3(ceil_div((long long)N * C, 256)),
                       dim3(256), 0, s, N, C, Y, out, ls, wsum);
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void slice_t(dcrf_ctx *ctx, const T *Y, const T *pre, int C, const T *mu,
             const T *mabs, T *out, bool qp) {
    const LatSet<T> ls = make_lat_set<T>(ctx, C);
    slice_set<T>(ctx, ls, 0, Y, pre, C, T(ctx->wsum), mu, mabs, out, qp);
}

template <typename T>
void filter_t(dcrf_ctx *ctx, const T *in, T *out, int C, bool adjoint,
              int kind) {
    if (kind == DCRF_FILTER_EXACT) {
        exact_t<T>(ctx, in, out, C);
        return;
    }
    if (kind == DCRF_FILTER_SEPARABLE) {
        filter_separable(ctx, in, out, C, adjoint);
        return;
    }
    splat_dense_t<T>(ctx, in, C);
    blur_all_t<T>(ctx, C, adjoint);
    slice_t<T>(ctx, in, nullptr, C, nullptr, nullptr, out, false);
}

// K~_m X alone: lattice m with weight 1 and no self-term subtraction
template <typename T>
void filter_kernel_t(dcrf_ctx *ctx, int m, const T *in, T *out, int C,
                     bool adjoint) {
    const hipStream_t s = ctx->stream;
    ensure_vertex_buffers(ctx, C);
    const LatSet<T> all = make_lat_set<T>(ctx, C);
    LatSet<T> ls{};
    ls.nk = 1;
    ls.l[0] = all.l[m];
    ls.l[0].wg = T(ctx->lat[m].gamma);
    ls.off[1] = all.off[m + 1] - all.off[m];
    ls.coff[1] = all.coff[m + 1] - all.coff[m];
    ls.eoff[1] = all.eoff[m + 1] - all.eoff[m];
    ls.choff[1] = all.choff[m + 1] - all.choff[m];
    ls.soff[1] = all.soff[m + 1] - all.soff[m];
    ls.shape52 = 0;
    (void)s;
    splat_set<T>(ctx, ls, in, C);
    blur_launch<T>(ctx, ls, m, adjoint);
    slice_set<T>(ctx, ls, m, in, nullptr, C, T(0), nullptr, nullptr, out, false);
}

}  // namespace

void exact_kernel(dcrf_ctx *ctx, int m, const void *in, void *out, int C) {
    if (ctx->dtype == DCRF_F64)
        exact_kernel_t<double>(ctx, m, static_cast<const double *>(in),
                               static_cast<double *>(out), C);
    else
        exact_kernel_t<float>(ctx, m, static_cast<const float *>(in),
                              static_cast<float *>(out), C);
}

void filter_kernel(dcrf_ctx *ctx, int m, const void *in, void *out, int C,
                   bool adjoint) {
    if (ctx->dtype == DCRF_F64)
        filter_kernel_t<double>(ctx, m, static_cast<const double *>(in),
                                static_cast<double *>(out), C, adjoint);
    else
        filter_kernel_t<float>(ctx, m, static_cast<const float *>(in),
                               static_cast<float *>(out), C, adjoint);
}

void ensure_vertex_buffers(dcrf_ctx *ctx, int C) {
    const int ld = row_stride(C, ctx->elt());
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &L = ctx->lat[m];
        const size_t bytes = (size_t)(L.M > 0 ? L.M : 1) * ld * ctx->elt();
        for (int b = 0; b < 3; ++b) L.V[b].ensure(bytes, ctx->stream);
    }
}

void splat_dense(dcrf_ctx *ctx, const void *in, int C) {
    if (ctx->dtype == DCRF_F64)
        splat_dense_t<double>(ctx, static_cast<const double *>(in), C);
    else
        splat_dense_t<float>(ctx, static_cast<const float *>(in), C);
}

void blur_group_tables(dcrf_ctx *ctx, int G) { ensure_group_tables(ctx, G, false); }

void splat_labels(dcrf_ctx *ctx, const int32_t *labels, int L) {
    if (ctx->dtype == DCRF_F64)
        splat_labels_t<double>(ctx, labels, L);
    else
        splat_labels_t<float>(ctx, labels, L);
}

void blur_all(dcrf_ctx *ctx, int C, bool adjoint) {
    if (ctx->dtype == DCRF_F64)
        blur_all_t<double>(ctx, C, adjoint);
    else
        blur_all_t<float>(ctx, C, adjoint);
}

void slice_into(dcrf_ctx *ctx, const void *Y, const void *pre, int C,
                const void *mu, const void *mabs, void *out, bool qp) {
    if (ctx->dtype == DCRF_F64)
        slice_t<double>(ctx, static_cast<const double *>(Y),
                        static_cast<const double *>(pre), C,
                        static_cast<const double *>(mu),
                        static_cast<const double *>(mabs),
                        static_cast<double *>(out), qp);
    else
        slice_t<float>(ctx, static_cast<const float *>(Y),
                       static_cast<const float *>(pre), C,
                       static_cast<const float *>(mu),
                       static_cast<const float *>(mabs),
                       static_cast<float *>(out), qp);
}

void filter_apply(dcrf_ctx *ctx, const void *in, void *out, int C,
                  bool adjoint, int kind) {
    if (ctx->dtype == DCRF_F64)
        filter_t<double>(ctx, static_cast<const double *>(in),
                         static_cast<double *>(out), C, adjoint, kind);
    else
        filter_t<float>(ctx, static_cast<const float *>(in),
                        static_cast<float *>(out), C, adjoint, kind);
}

void compute_row_sums(dcrf_ctx *ctx) {
    const size_t e = ctx->elt();
    ctx->r.ensure((size_t)ctx->N * e, ctx->stream);
    ctx->tmpA.ensure((size_t)ctx->N * e, ctx->stream);
    fill_ones(ctx, ctx->tmpA.p, ctx->N);
    filter_apply(ctx, ctx->tmpA.p, ctx->r.p, 1, false, ctx->mode);
}

}  // namespace dcrf
