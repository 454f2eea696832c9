// Device-side views of the lattices and helpers shared by the kernels.
#pragma once

#include "dcrf_internal.h"

namespace dcrf {

// One lattice as the splat / blur / slice kernels see it.
template <typename T>
struct LatView {
    const int32_t *vid;  // N x (d+1) vertex ids (-1: weight 0)
    const T *w;          // N x (d+1) barycentric weights
    const int32_t *nbr;  // (d+1) x M x 2
    T *V0, *V1, *V2;     // M x ld: splat target, ping, pong
    const T *Vf;         // the buffer that holds the blurred values
    const int4 *chunks;  // inverse-index chunks (vertex, begin, end, 0)
    const int4 *dchunks; // the chunks of the dense splat
    const int32_t *dpix; // their entries at a stride of the chunk length
    const T *dw;
    const int32_t *ent_pix;
    const T *ent_w;
    const int32_t *ent_v;
    int d, M, ld, nchunks, ndchunks;
    T wg;                // w_m * gamma_m
    const int32_t *gt;   // grouped-blur path table of the direction in use
    int ngrp;            // blur launches of this lattice
    // per-tile vertex slots
    const int32_t *ts_off, *ts_vid, *sr_off, *vs_off, *vs_slot;
    const uint16_t *tr_slot, *sr_slot;
    const uint8_t *sr_pix;
    const T *sr_w;
    int nslots;
};

template <typename T>
struct LatSet {
    LatView<T> l[DCRF_MAXK];
    long long off[DCRF_MAXK + 1];   // prefix sums of M_m * ld (blur)
    long long coff[DCRF_MAXK + 1];  // dense splat: prefix sums of 256 lanes per
                                    // block of 256 / C chunks (one lattice a block)
    long long eoff[DCRF_MAXK + 1];  // prefix sums of the entries
    long long choff[DCRF_MAXK + 1]; // prefix sums of nchunks_m (label splat)
    long long soff[DCRF_MAXK + 1];  // prefix sums of nslots_m (tile splat)
    int nk;
    int shape52;                    // two lattices with d = 5 and d = 2
};

template <typename T>
struct ExactSet {
    const T *f[DCRF_MAXK];
    int d[DCRF_MAXK];
    int off[DCRF_MAXK + 1];
    T w[DCRF_MAXK];
    int nk;
};

// Pairs staged in LDS per block by the staged gather splat.
constexpr int kSplatStage = 1024;

// Chunks per block of 256 lanes in the dense splat (C lanes per chunk); the
// staged splat keeps their pairs within kSplatStage.
inline int dense_splat_q(const dcrf_ctx *ctx, int C) {
    int q = C <= 256 ? 256 / C : 1;
    if (ctx->splat_lds) q = std::min(q, std::max(1, kSplatStage / ctx->dense_chunk));
    return q;
}

// C: channels of the call; the vertex rows have stride row_stride(C).
template <typename T>
inline LatSet<T> make_lat_set(dcrf_ctx *ctx, int C) {
    LatSet<T> s{};
    s.nk = ctx->nk;
    s.off[0] = 0;
    s.coff[0] = 0;
    s.eoff[0] = 0;
    s.choff[0] = 0;
    s.soff[0] = 0;
    const int ld = row_stride(C, sizeof(T));
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &L = ctx->lat[m];
        LatView<T> &v = s.l[m];
        v.vid = L.pix_vid.as<int32_t>();
        v.w = L.pix_w.as<T>();
        v.nbr = L.nbr.as<int32_t>();
        v.V0 = L.V[0].as<T>();
        v.V1 = L.V[1].as<T>();
        v.V2 = L.V[2].as<T>();
        const int nl = blur_launches(L.d, ctx->blur_group);
        v.ngrp = nl;
        v.Vf = L.V[final_buffer_after(nl)].as<T>();
        v.gt = nullptr;
        v.ts_off = L.ts_off.as<int32_t>();
        v.ts_vid = L.ts_vid.as<int32_t>();
        v.sr_off = L.sr_off.as<int32_t>();
        v.vs_off = L.vs_off.as<int32_t>();
        v.vs_slot = L.vs_slot.as<int32_t>();
        v.tr_slot = L.tr_slot.as<uint16_t>();
        v.sr_slot = L.sr_slot.as<uint16_t>();
        v.sr_pix = L.sr_pix.as<uint8_t>();
        v.sr_w = L.sr_w.as<T>();
        v.nslots = L.nslots;
        v.chunks = L.chunks.as<int4>();
        v.dchunks = L.dchunks.as<int4>();
        v.dpix = L.dpix.as<int32_t>();
        v.dw = L.dw.as<T>();
        v.ent_pix = L.ent_pix.as<int32_t>();
        v.ent_w = L.ent_w.as<T>();
        v.ent_v = L.ent_v.as<int32_t>();
        v.d = L.d;
        v.M = L.M;
        v.ld = ld;
        v.nchunks = L.nchunks;
        v.ndchunks = L.ndchunks;
        v.wg = T(ctx->kern[m].weight * L.gamma);
        s.off[m + 1] = s.off[m] + (long long)L.M * ld;
        const long long q = dense_splat_q(ctx, C);
        s.coff[m + 1] = s.coff[m] + ((long long)L.ndchunks + q - 1) / q * 256;
        s.eoff[m + 1] = s.eoff[m] + (long long)L.nent;
        s.choff[m + 1] = s.choff[m] + (long long)L.nchunks;
        s.soff[m + 1] = s.soff[m] + (long long)L.nslots;
    }
    s.shape52 = (ctx->nk == 2 && ctx->lat[0].d == 5 && ctx->lat[1].d == 2) ? 1 : 0;
    return s;
}

template <typename T>
inline ExactSet<T> make_exact_set(dcrf_ctx *ctx) {
    ExactSet<T> s{};
    s.nk = ctx->nk;
    s.off[0] = 0;
    for (int m = 0; m < ctx->nk; ++m) {
        s.f[m] = ctx->lat[m].feat.as<T>();
        s.d[m] = ctx->lat[m].d;
        s.off[m + 1] = s.off[m] + s.d[m];
        s.w[m] = T(ctx->kern[m].weight);
    }
    return s;
}

__device__ __forceinline__ void atomic_add(float *p, float v) {
    unsafeAtomicAdd(p, v);
}
__device__ __forceinline__ void atomic_add(double *p, double v) {
    unsafeAtomicAdd(p, v);
}

void fill_ones(dcrf_ctx *ctx, void *p, size_t n);

// ------------------------------------------------------- row kernels

// Pixels per block of the row kernels (one thread per pixel).
template <typename T> struct RowTile;
template <> struct RowTile<float> { static constexpr int kPix = 128; };
template <> struct RowTile<double> { static constexpr int kPix = 64; };

// The workgroups of a launch are dealt to the chip's 8 XCDs round-robin
// (block b runs on XCD b % 8, each XCD with its own L2). This maps the
// hardware block index to a logical one such that every XCD receives one
// contiguous range of logical blocks: neighbouring work (adjacent pixel
// tiles, inverse-index chunks ordered by pixel) then shares an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb - q * X;
    const int x = b % X, i = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Block b of a launch over two lattices of 8 q0 and 8 q1 blocks, whose
// blocks walk each lattice's work in pixel order: the hardware sends block b
// to XCD b mod 8, and XCD x takes blocks [x q_m, (x + 1) q_m) of both
// lattices, interleaved in proportion, so that it covers the same stretch of
// pixels in both lattices at the same time and the rows they gather meet in
// its L2. Returns the lattice and sets lb, the block within it.
__device__ __forceinline__ int xcd_pair_block(int b, int q0, int q1, int &lb) {
    const int x = b & 7, i = b >> 3, T = q0 + q1;
    const int c = int((long long)(i + 1) * q0 / T);   // lattice-0 blocks among the first i + 1
    if (c > int((long long)i * q0 / T)) {
        lb = x * q0 + c - 1;
        return 0;
    }
    lb = x * q1 + (i - c);
    return 1;
}

// Tile `tile` of the per-image tilings of TP pixels, images taken in order
// (see dcrf_ctx::seg): returns the image and sets [lo, hi), its pixel rows.
// Images start at multiples of 64 pixels, so a tile's rows start 16-byte
// aligned like those of a single image.
__device__ __forceinline__ int tile_range(const int *__restrict__ seg, int nimg,
                                          int TP, int tile, int &lo, int &hi) {
    int t = tile;
    for (int j = 0; j < nimg; ++j) {
        const int s = seg[2 * j], e = seg[2 * j + 1];
        const int nt = (e - s + TP - 1) / TP;
        if (t < nt) {
            lo = s + t * TP;
            hi = min(lo + TP, e);
            return j;
        }
        t -= nt;
    }
    lo = hi = 0;
    return -1;
}

// Copy a 2-D pixel tile of a pixel-major N x C array to or from LDS rows
// of stride LS (pixel (i, px) of the tile at row i * kTileW + px). td holds
// the tile's first pixel row, the image's row stride in pixels, and the
// tile's rows and columns. Consecutive threads move consecutive elements of
// a tile row, which is one contiguous range in global memory. Every thread
// of the block must call these; the caller synchronises.
template <typename T, int NT>
__device__ __forceinline__ void tile2_in(const T *__restrict__ g, int4 td, int C,
                                         T *lds, int LS) {
    // flattened elements t, t + NT, ... of the tile; each batch of kB loads is
    // issued before any of them is stored, one round trip per batch
    constexpr int kB = 16;
    const int wC = td.w * C;
    const int E = td.z * wC;
    const float invw = 1.0f / float(wC), invc = 1.0f / float(C);
    for (int f0 = 0; f0 < E; f0 += NT * kB) {
        T v[kB];
        int dst[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int f = f0 + u * NT + (int)threadIdx.x;
            dst[u] = -1;
            v[u] = T(0);
            if (f < E) {
                const int i = int((float(f) + 0.5f) * invw);
                const int k = f - i * wC;
                const int px = int((float(k) + 0.5f) * invc);
                v[u] = g[((size_t)td.x + (size_t)i * td.y) * C + k];
                dst[u] = (i * kTileW + px) * LS + (k - px * C);
            }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u)
            if (dst[u] >= 0) lds[dst[u]] = v[u];
    }
}

template <typename T, int NT>
__device__ __forceinline__ void tile2_out(T *__restrict__ g, int4 td, int C,
                                          const T *lds, int LS) {
    const int wC = td.w * C;
    const float inv = 1.0f / float(C);
    for (int i = 0; i < td.z; ++i) {
        T *dst = g + ((size_t)td.x + (size_t)i * td.y) * C;
        const T *src = lds + i * kTileW * LS;
        for (int k = threadIdx.x; k < wC; k += NT) {
            const int px = int((float(k) + 0.5f) * inv);
            dst[k] = src[px * LS + (k - px * C)];
        }
    }
}

// Largest channel count handled with per-thread register rows.
constexpr int kRowMaxC = 32;

// LDS row stride of a staged tile: odd, so that threads reading row t at
// stride Ls hit distinct banks.
__device__ __forceinline__ int lds_stride(int C) { return C | 1; }

// 16-byte vector of T
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int n = 2; };

// Move np pixel rows of C values between global memory (contiguous rows) and
// per-thread registers through LDS so that the global side is coalesced.
// For odd C the LDS tile is the contiguous global block and moves with
// 16-byte accesses (tiles start at multiples of TP pixels, so 16-byte
// aligned); for even C rows are padded to an odd stride. A thread moves at
// most ceil(CMAX / 4) vectors (np <= TP, C <= CMAX): all of its loads are
// issued before the first store, so a copy costs one memory round trip.
// Every thread of the block must call these (they synchronise).
template <typename T, int TP, int CMAX>
__device__ __forceinline__ void tile_copy_in(const T *__restrict__ src, int n,
                                             int C, T *lds) {
    if (C & 1) {
        using V = typename Vec16<T>::type;
        constexpr int w = Vec16<T>::n;
        constexpr int K = (CMAX + w - 1) / w;
        const int nv = n / w;
        const V *s = reinterpret_cast<const V *>(src);
        V *l = reinterpret_cast<V *>(lds);
        // indices past the end repeat the last vector (loaded and stored
        // again, same value): with no condition on a load or its store, the
        // compiler keeps every load in flight instead of sinking each one
        // into a branch of its own
        if (nv > 0) {
            V v[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] = s[min((int)threadIdx.x + k * TP, nv - 1)];
            // an empty statement that uses every loaded vector: all of them
            // are live at once here, so the compiler issues all the loads
            // before the first wait instead of pairing each with its store
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < w; ++e)
                    __asm__ __volatile__("" ::"v"(reinterpret_cast<const T *>(&v[k])[e]));
#pragma unroll
            for (int k = 0; k < K; ++k) l[min((int)threadIdx.x + k * TP, nv - 1)] = v[k];
        }
        const int i = nv * w + (int)threadIdx.x;
        if (i < n) lds[i] = src[i];
    } else {
        const int Ls = C | 1;
        const float inv = 1.0f / float(C);
        if (n > 0) {
            T v[CMAX];
#pragma unroll
            for (int k = 0; k < CMAX; ++k) v[k] = src[min((int)threadIdx.x + k * TP, n - 1)];
#pragma unroll
            for (int k = 0; k < CMAX; ++k) __asm__ __volatile__("" ::"v"(v[k]));
#pragma unroll
            for (int k = 0; k < CMAX; ++k) {
                const int i = min((int)threadIdx.x + k * TP, n - 1);
                const int p = int((float(i) + 0.5f) * inv);
                lds[p * Ls + (i - p * C)] = v[k];
            }
        }
    }
}

template <typename T, int TP, int CMAX>
__device__ __forceinline__ void tile_copy_out(T *__restrict__ dst, int n, int C,
                                              const T *lds) {
    if (C & 1) {
        using V = typename Vec16<T>::type;
        constexpr int w = Vec16<T>::n;
        constexpr int K = (CMAX + w - 1) / w;
        const int nv = n / w;
        V *d = reinterpret_cast<V *>(dst);
        const V *l = reinterpret_cast<const V *>(lds);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = (int)threadIdx.x + k * TP;
            if (i < nv) d[i] = l[i];
        }
        const int i = nv * w + (int)threadIdx.x;
        if (i < n) dst[i] = lds[i];
    } else {
        const int Ls = C | 1;
        const float inv = 1.0f / float(C);
#pragma unroll
        for (int k = 0; k < CMAX; ++k) {
            const int i = (int)threadIdx.x + k * TP;
            if (i < n) {
                const int p = int((float(i) + 0.5f) * inv);
                dst[i] = lds[p * Ls + (i - p * C)];
            }
        }
    }
}

// tile_copy_in in two halves, so that the loads of several tiles (or of a
// tile and other data) are in flight together: tile_fetch issues a thread's
// loads into a TileRegs, tile_put stores them into the LDS tile in
// tile_copy_in's layout. Every thread calls both; neither synchronises.
// Odd C: v[k] is the tile's 16-byte vector threadIdx.x + k TP (clamped to the
// last whole one), `tail` element nv w + threadIdx.x; even C: element k of v
// (viewed as K w values of T) is the tile's element threadIdx.x + k TP.
template <typename T, int TP, int CMAX>
struct TileRegs {
    using V = typename Vec16<T>::type;
    static constexpr int w = Vec16<T>::n;
    static constexpr int K = (CMAX + w - 1) / w;
    V v[K];
    T tail;
    __device__ __forceinline__ T &el(int k) { return reinterpret_cast<T *>(v)[k]; }
    __device__ __forceinline__ const T &el(int k) const {
        return reinterpret_cast<const T *>(v)[k];
    }
};

template <typename T, int TP, int CMAX>
__device__ __forceinline__ void tile_fetch(const T *__restrict__ src, int n, int C,
                                           TileRegs<T, TP, CMAX> &r) {
    using R = TileRegs<T, TP, CMAX>;
    if (C & 1) {
        const int nv = n / R::w;
        const auto *s = reinterpret_cast<const typename R::V *>(src);
        if (nv > 0) {
#pragma unroll
            for (int k = 0; k < R::K; ++k) r.v[k] = s[min((int)threadIdx.x + k * TP, nv - 1)];
        }
        const int i = nv * R::w + (int)threadIdx.x;
        r.tail = i < n ? src[i] : T(0);
    } else if (n > 0) {
#pragma unroll
        for (int k = 0; k < CMAX; ++k) r.el(k) = src[min((int)threadIdx.x + k * TP, n - 1)];
    }
}

template <typename T, int TP, int CMAX>
__device__ __forceinline__ void tile_put(int n, int C, const TileRegs<T, TP, CMAX> &r,
                                         T *lds) {
    using R = TileRegs<T, TP, CMAX>;
    if (C & 1) {
        const int nv = n / R::w;
        auto *l = reinterpret_cast<typename R::V *>(lds);
        if (nv > 0) {
#pragma unroll
            for (int k = 0; k < R::K; ++k) l[min((int)threadIdx.x + k * TP, nv - 1)] = r.v[k];
        }
        const int i = nv * R::w + (int)threadIdx.x;
        if (i < n) lds[i] = r.tail;
    } else if (n > 0) {
        const int Ls = C | 1;
        const float inv = 1.0f / float(C);
#pragma unroll
        for (int k = 0; k < CMAX; ++k) {
            const int i = min((int)threadIdx.x + k * TP, n - 1);
            const int p = int((float(i) + 0.5f) * inv);
            lds[p * Ls + (i - p * C)] = r.el(k);
        }
    }
}

// Row threadIdx.x of a tile staged by tile_copy_in, into registers (no
// synchronisation: the caller has synchronised after the copy, and a thread
// that later overwrites only its own row needs none either).
template <typename T, int LMAX>
__device__ __forceinline__ void tile_read_own(int np, int C, const T *lds, T (&r)[LMAX]) {
    const int Ls = lds_stride(C);
    if ((int)threadIdx.x < np) {
#pragma unroll
        for (int j = 0; j < LMAX; ++j)
            if (j < C) r[j] = lds[threadIdx.x * Ls + j];
    }
}

template <typename T, int LMAX, int TP>
__device__ __forceinline__ void tile_load(const T *__restrict__ g, long long p0,
                                          int np, int C, T *lds, T (&r)[LMAX]) {
    const int Ls = lds_stride(C);
    tile_copy_in<T, TP, LMAX>(g + p0 * C, np * C, C, lds);
    __syncthreads();
    if ((int)threadIdx.x < np) {
#pragma unroll
        for (int j = 0; j < LMAX; ++j)
            if (j < C) r[j] = lds[threadIdx.x * Ls + j];
    }
    __syncthreads();
}

// tile_load's second half for a tile fetched by tile_fetch (np rows of C)
template <typename T, int LMAX, int TP>
__device__ __forceinline__ void tile_rows(int np, int C, const TileRegs<T, TP, LMAX> &f,
                                          T *lds, T (&r)[LMAX]) {
    tile_put<T, TP, LMAX>(np * C, C, f, lds);
    __syncthreads();
    tile_read_own<T, LMAX>(np, C, lds, r);
    __syncthreads();
}

template <typename T, int LMAX, int TP>
__device__ __forceinline__ void tile_store(T *__restrict__ g, long long p0,
                                           int np, int C, T *lds,
                                           const T (&r)[LMAX]) {
    const int Ls = lds_stride(C);
    if ((int)threadIdx.x < np) {
#pragma unroll
        for (int j = 0; j < LMAX; ++j)
            if (j < C) lds[threadIdx.x * Ls + j] = r[j];
    }
    __syncthreads();
    tile_copy_out<T, TP, LMAX>(g + p0 * C, np * C, C, lds);
    __syncthreads();
}

// acc[j] += s * row[j] for j < C, with 16-byte loads (rows are 16-byte
// aligned and padded with zeros to a multiple of 16 bytes)
template <int LMAX>
__device__ __forceinline__ void axpy_row(float (&acc)[LMAX], float s,
                                         const float *__restrict__ row, int C) {
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
    for (int q = 0; q < LMAX / 4; ++q) {
        if (4 * q < C) {
            const float4 v = r4[q];
            acc[4 * q + 0] += s * v.x;
            acc[4 * q + 1] += s * v.y;
            acc[4 * q + 2] += s * v.z;
            acc[4 * q + 3] += s * v.w;
        }
    }
}

template <int LMAX>
__device__ __forceinline__ void axpy_row(double (&acc)[LMAX], double s,
                                         const double *__restrict__ row, int C) {
    const double2 *r2 = reinterpret_cast<const double2 *>(row);
#pragma unroll
    for (int q = 0; q < LMAX / 2; ++q) {
        if (2 * q < C) {
            const double2 v = r2[q];
            acc[2 * q + 0] += s * v.x;
            acc[2 * q + 1] += s * v.y;
        }
    }
}

// The slice of pixel a for two lattices of compile-time dimensions DA, DB:
// all vertex ids and weights are loaded first, then every row load is issued
// unconditionally (a missing vertex reads row 0 with weight 0), so that all
// of them can be in flight together.
template <typename T, int LMAX, int DA, int DB>
__device__ __forceinline__ void slice_pixel_fixed(const LatSet<T> &ls,
                                                  long long a, int C,
                                                  T (&acc)[LMAX]) {
    const LatView<T> &A = ls.l[0];
    const LatView<T> &B = ls.l[1];
    int ia[DA + 1], ib[DB + 1];
    T wa[DA + 1], wb[DB + 1];
#pragma unroll
    for (int k = 0; k <= DA; ++k) {
        const int id = A.vid[a * (DA + 1) + k];
        wa[k] = id >= 0 ? A.wg * A.w[a * (DA + 1) + k] : T(0);
        ia[k] = id >= 0 ? id : 0;
    }
#pragma unroll
    for (int k = 0; k <= DB; ++k) {
        const int id = B.vid[a * (DB + 1) + k];
        wb[k] = id >= 0 ? B.wg * B.w[a * (DB + 1) + k] : T(0);
        ib[k] = id >= 0 ? id : 0;
    }
#pragma unroll
    for (int k = 0; k <= DA; ++k)
        axpy_row<LMAX>(acc, wa[k], A.Vf + (size_t)ia[k] * A.ld, C);
#pragma unroll
    for (int k = 0; k <= DB; ++k)
        axpy_row<LMAX>(acc, wb[k], B.Vf + (size_t)ib[k] * B.ld, C);
}

// The per-pixel vertex ids and weights of the two lattices of a 5-D + 2-D
// set (ls.shape52) for the pixels [p0, p0 + np) of a row tile, moved to LDS
// with contiguous loads (all issued before the first store): lattice 0 at
// sid/sw[0, 6 TP), lattice 1 at [6 TP, 9 TP). Every thread of the block calls
// this; the caller synchronises before reading. np >= 1.
constexpr int kCorners52 = 9;
template <typename T, int TP>
__device__ __forceinline__ void stage_corners52(const LatSet<T> &ls, long long p0,
                                                int np, int32_t *sid, T *sw) {
    const LatView<T> &A = ls.l[0];
    const LatView<T> &B = ls.l[1];
    const int na = np * 6, nb = np * 3;
    const int32_t *va = A.vid + p0 * 6, *vb = B.vid + p0 * 3;
    const T *wa = A.w + p0 * 6, *wb = B.w + p0 * 3;
    int ia[6], ib[3];
    T fa[6], fb[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int i = min((int)threadIdx.x + k * TP, na - 1);
        ia[k] = va[i];
        fa[k] = wa[i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = min((int)threadIdx.x + k * TP, nb - 1);
        ib[k] = vb[i];
        fb[k] = wb[i];
    }
    // every loaded value is live here, so all the loads are issued first
#pragma unroll
    for (int k = 0; k < 6; ++k) __asm__ __volatile__("" ::"v"(ia[k]), "v"(fa[k]));
#pragma unroll
    for (int k = 0; k < 3; ++k) __asm__ __volatile__("" ::"v"(ib[k]), "v"(fb[k]));
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int i = min((int)threadIdx.x + k * TP, na - 1);
        sid[i] = ia[k];
        sw[i] = fa[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = min((int)threadIdx.x + k * TP, nb - 1);
        sid[6 * TP + i] = ib[k];
        sw[6 * TP + i] = fb[k];
    }
}

// The slice of the tile's pixel t (ls.shape52) from the corners staged by
// stage_corners52; as slice_pixel_fixed otherwise.
template <typename T, int LMAX, int TP>
__device__ __forceinline__ void slice_pixel52_staged(const LatSet<T> &ls, int t, int C,
                                                     const int32_t *sid, const T *sw,
                                                     T (&acc)[LMAX]) {
    const LatView<T> &A = ls.l[0];
    const LatView<T> &B = ls.l[1];
    int ia[6], ib[3];
    T wa[6], wb[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int id = sid[t * 6 + k];
        wa[k] = id >= 0 ? A.wg * sw[t * 6 + k] : T(0);
        ia[k] = id >= 0 ? id : 0;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int id = sid[6 * TP + t * 3 + k];
        wb[k] = id >= 0 ? B.wg * sw[6 * TP + t * 3 + k] : T(0);
        ib[k] = id >= 0 ? id : 0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) axpy_row<LMAX>(acc, wa[k], A.Vf + (size_t)ia[k] * A.ld, C);
#pragma unroll
    for (int k = 0; k < 3; ++k) axpy_row<LMAX>(acc, wb[k], B.Vf + (size_t)ib[k] * B.ld, C);
}

// The slice of a whole tile from the corners staged by stage_corners52, into
// the LDS tile qt (row stride lds_stride(C)): one task per (pixel, 16-byte
// chunk of its row), consecutive lanes taking consecutive chunks of one
// pixel, so that a wave's loads of one corner cover a few rows instead of one
// row per lane. A thread takes its tasks U at a time with the loads of all U
// issued together (a task past the end repeats the last one and stores
// nothing), so that 9 U rows are in flight per lane. All threads of the block
// call it; the caller synchronises before reading qt.
template <typename T, int LMAX, int TP, int U = 2>
__device__ __forceinline__ void slice_tile52_coop(const LatSet<T> &ls, int np, int C,
                                                  const int32_t *sid, const T *sw,
                                                  T *qt) {
    using V = typename Vec16<T>::type;
    constexpr int w = Vec16<T>::n;
    constexpr int KQ = (LMAX + w - 1) / w;   // tasks per thread
    const LatView<T> &A = ls.l[0];
    const LatView<T> &B = ls.l[1];
    const int nq = (C + w - 1) / w;
    const int Ls = lds_stride(C);
    const int ntask = np * nq;
#pragma unroll
    for (int i0 = 0; i0 < KQ; i0 += U) {
        if ((int)threadIdx.x + i0 * TP >= ntask) break;
        int p[U], qc[U];
        V va[U][6], vb[U][3];
        T fa[U][6], fb[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int task = min((int)threadIdx.x + (i0 + u) * TP, ntask - 1);
            p[u] = task / nq;
            qc[u] = task - p[u] * nq;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int id = sid[p[u] * 6 + k];
                fa[u][k] = id >= 0 ? A.wg * sw[p[u] * 6 + k] : T(0);
                va[u][k] = *reinterpret_cast<const V *>(
                    A.Vf + (size_t)(unsigned)(id >= 0 ? id : 0) * (unsigned)A.ld + qc[u] * w);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int id = sid[6 * TP + p[u] * 3 + k];
                fb[u][k] = id >= 0 ? B.wg * sw[6 * TP + p[u] * 3 + k] : T(0);
                vb[u][k] = *reinterpret_cast<const V *>(
                    B.Vf + (size_t)(unsigned)(id >= 0 ? id : 0) * (unsigned)B.ld + qc[u] * w);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T ac[w];
#pragma unroll
            for (int e = 0; e < w; ++e) ac[e] = T(0);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const T *x = reinterpret_cast<const T *>(&va[u][k]);
#pragma unroll
                for (int e = 0; e < w; ++e) ac[e] += fa[u][k] * x[e];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T *x = reinterpret_cast<const T *>(&vb[u][k]);
#pragma unroll
                for (int e = 0; e < w; ++e) ac[e] += fb[u][k] * x[e];
            }
            if ((int)threadIdx.x + (i0 + u) * TP < ntask) {
#pragma unroll
                for (int e = 0; e < w; ++e)
                    if (qc[u] * w + e < C) qt[p[u] * Ls + qc[u] * w + e] = ac[e];
            }
        }
    }
}

// ------------------------------------ label splat and grouped blur bodies

// (pixel or label, weight) of one inverse-index entry, one LDS word
template <typename T> struct alignas(2 * sizeof(T) > 8 ? 16 : 8) PairLds {
    int i;
    T w;
};

// One-hot input in the layout of the staged dense splat: block b takes q
// chunks of C = L lanes (chunk, label); the labels of the chunks' pixels and
// the weights are staged in LDS, then lane (chunk, c) adds up the weights of
// the entries labelled c, and adds the sum to V0[v][c] if it is not zero.
// Labels outside [0, L) add nothing.
// The block of 256 threads that takes lanes [b0, b0 + 256); sp holds
// kSplatStage pairs, scd 256 chunk descriptors.
template <typename T>
__device__ __forceinline__ void splat_labels_block(int C, int q, int U,
                                                   const int32_t *__restrict__ labels,
                                                   const LatSet<T> &ls, long long b0,
                                                   PairLds<T> *sp, int4 *scd) {
    int m = 0;
    while (m + 1 < ls.nk && b0 >= ls.coff[m + 1]) ++m;
    const LatView<T> &L = ls.l[m];
    const int ch0 = int((b0 - ls.coff[m]) / 256) * q;
    const int nq = min(q, L.ndchunks - ch0);
    const int t = threadIdx.x;
    if (t < nq) scd[t] = L.dchunks[ch0 + t];
    const size_t base = (size_t)ch0 * U;   // the block's entries: one contiguous range
    for (int i = t; i < nq * U; i += 256)
        sp[i] = PairLds<T>{labels[L.dpix[base + i]], L.dw[base + i]};
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
        acc0 += e0.i == c ? e0.w : T(0);
        acc1 += e1.i == c ? e1.w : T(0);
        acc2 += e2.i == c ? e2.w : T(0);
        acc3 += e3.i == c ? e3.w : T(0);
    }
    for (; j < n; ++j) acc0 += pk[j].i == c ? pk[j].w : T(0);
    const T acc = (acc0 + acc1) + (acc2 + acc3);
    if (acc != T(0)) atomic_add(&L.V0[(size_t)cd.x * L.ld + c], acc);
}


template <int G> struct Pow3 { static constexpr int v = 3 * Pow3<G - 1>::v; };
template <> struct Pow3<0> { static constexpr int v = 1; };

template <typename T, int G>
__device__ __forceinline__ void blur_group_vector(const LatSet<T> &ls, int grp,
                                                  long long e) {
    using V = typename Vec16<T>::type;
    constexpr int vw = Vec16<T>::n;
    constexpr int P = Pow3<G>::v;
    int m = 0;
    while (m + 1 < ls.nk && e >= ls.off[m + 1] / vw) ++m;
    const LatView<T> &L = ls.l[m];
    const unsigned Gv = unsigned(L.ld / vw);
    const unsigned r = unsigned(e - ls.off[m] / vw);
    V zero;
    for (int i = 0; i < vw; ++i) reinterpret_cast<T *>(&zero)[i] = T(0);
    if (grp >= L.ngrp) {
        if (grp == 1) reinterpret_cast<V *>(L.V0)[r] = zero;
        return;
    }
    const int v = int(r / Gv);
    const int g = int(r - unsigned(v) * Gv);
    const V *src = reinterpret_cast<const V *>((grp == 0) ? L.V0 : ((grp & 1) ? L.V1 : L.V2));
    V *dst = reinterpret_cast<V *>((grp & 1) ? L.V2 : L.V1);
    const int32_t *ids = L.gt + ((size_t)grp * L.M + v) * P;
    int id[P];
#pragma unroll
    for (int p = 0; p < P; ++p) id[p] = ids[p];
    T acc[vw];
#pragma unroll
    for (int i = 0; i < vw; ++i) acc[i] = T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        // coefficient: 1/2 per staying step, 1/4 per move (digits of p)
        T c = T(1);
        int code = p;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            c *= (code % 3 == 0) ? T(0.5) : T(0.25);
            code /= 3;
        }
        const V x = src[(size_t)(id[p] >= 0 ? id[p] : 0) * Gv + g];
        if (id[p] < 0) c = T(0);
#pragma unroll
        for (int i = 0; i < vw; ++i) acc[i] += c * reinterpret_cast<const T *>(&x)[i];
    }
    if (grp == L.ngrp - 1) {
        const int missing = L.ngrp * G - (L.d + 1);
        const T sc = T(1 << missing);
#pragma unroll
        for (int i = 0; i < vw; ++i) acc[i] *= sc;
    }
    V o;
#pragma unroll
    for (int i = 0; i < vw; ++i) reinterpret_cast<T *>(&o)[i] = acc[i];
    dst[r] = o;
    if (grp == 1) reinterpret_cast<V *>(L.V0)[r] = zero;
}

// ------------------------------------------- one-hot splat, pixel-major

// Every lane of the wave holds one term: v to be added at row `id` (< 0: no
// term), column `lab` of V (row stride ld). Consecutive lanes hold
// consecutive pixels, whose terms often share their (row, column): such runs
// are summed inside the wave first (a segmented scan over lanes), and the
// last lane of each run adds the run's sum to V with one atomic. All lanes of
// the wave call it together.
template <typename T>
__device__ __forceinline__ void wave_run_add(T *V, int ld, int id, int lab, T v) {
    const int lane = (int)(threadIdx.x & 63);
    const int pid = __shfl_up(id, 1), plab = __shfl_up(lab, 1);
    const bool head = lane == 0 || pid != id || plab != lab;
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const int start = 63 - __clzll(hm & upto);   // the first lane of this run
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T up = __shfl_up(v, d);
        if (lane - d >= start) v += up;
    }
    const bool last = lane == 63 || ((hm >> (lane + 1)) & 1ull);
    if (last && id >= 0 && lab >= 0) atomic_add(V + (size_t)(unsigned)id * (unsigned)ld + lab, v);
}

// The corners of one pixel in a 5-D + 2-D lattice pair (ls.shape52), loaded
// ahead of their use; id -1 for a missing vertex or an inactive lane.
template <typename T>
struct Corners52 {
    int id[kCorners52];
    T w[kCorners52];
};

template <typename T>
__device__ __forceinline__ void load_corners52(const LatSet<T> &ls, long long a, bool act,
                                               Corners52<T> &c) {
    const long long i = act ? a : 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        c.id[k] = ls.l[0].vid[i * 6 + k];
        c.w[k] = ls.l[0].w[i * 6 + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c.id[6 + k] = ls.l[1].vid[i * 3 + k];
        c.w[6 + k] = ls.l[1].w[i * 3 + k];
    }
    if (!act)
#pragma unroll
        for (int k = 0; k < kCorners52; ++k) c.id[k] = -1;
}

// The splat of the one-hot rows of the wave's pixels: pixel a (label lab,
// < 0 or an inactive lane: nothing) adds w_m(a, k) to V0_m[v_m(a, k)][lab]
// for every corner k of every lattice, the terms of a run of lanes with the
// same vertex and label summed first (wave_run_add). The caller's targets
// V0 hold zeros before the first wave adds to them.
template <typename T>
__device__ __forceinline__ void splat_onehot52(const LatSet<T> &ls, const Corners52<T> &c,
                                               int lab) {
#pragma unroll
    for (int k = 0; k < kCorners52; ++k) {
        const LatView<T> &L = ls.l[k < 6 ? 0 : 1];
        wave_run_add<T>(L.V0, L.ld, c.id[k], lab, c.w[k]);
    }
}

template <typename T>
__device__ __forceinline__ void splat_onehot(const LatSet<T> &ls, long long a, bool act,
                                             int lab) {
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int D1 = L.d + 1;
        for (int k = 0; k < D1; ++k) {
            const int id = act ? L.vid[a * D1 + k] : -1;
            const T wv = act ? L.w[a * D1 + k] : T(0);
            wave_run_add<T>(L.V0, L.ld, id, lab, wv);
        }
    }
}

// sum over the lattices of w_m gamma_m sum_k b_k V_m[v_k]  (the slice of
// pixel a into acc, which the caller has zeroed)
template <typename T, int LMAX>
__device__ __forceinline__ void slice_pixel(const LatSet<T> &ls, long long a,
                                            int C, T (&acc)[LMAX]) {
    if (ls.shape52) {
        slice_pixel_fixed<T, LMAX, 5, 2>(ls, a, C, acc);
        return;
    }
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int D1 = L.d + 1;
        for (int k = 0; k < D1; ++k) {
            const int id = L.vid[a * D1 + k];
            if (id >= 0)
                axpy_row<LMAX>(acc, L.wg * L.w[a * D1 + k],
                               L.Vf + (size_t)id * L.ld, C);
        }
    }
}

// block-wide sum of NV doubles per thread (NT threads); every thread returns
// the totals
template <int NV, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[i * NT + t] = v[i];
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int i = 0; i < NV; ++i) lds[i * NT + t] += lds[i * NT + t + off];
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = lds[i * NT];
    __syncthreads();
}

// Block-wide sums of NV doubles per thread: a shuffle reduction inside each
// 64-lane wave, then the waves' sums through LDS (NV x NT/64 doubles). Thread
// i < NV returns the total of component i (fixed summation order).
template <int NV, int NT>
__device__ __forceinline__ double block_sum_waves(const double (&v)[NV], double *lds) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) lds[i * NW + w] = x;
    }
    __syncthreads();
    double s = 0.0;
    if ((int)threadIdx.x < NV)
        for (int k = 0; k < NW; ++k) s += lds[threadIdx.x * NW + k];
    return s;
}

// Euclidean projection of v (register row, C valid entries) onto the simplex:
// sort descending with a bitonic network, cumulative sums in sorted order,
// rho = last j with u_j - (css_j - 1) / j > 0, tau = (css_rho - 1) / rho.
template <typename T, int P>
__device__ __forceinline__ T simplex_tau(const T (&v)[P], int C) {
    T u[P];
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = (i < C) ? v[i] : -INFINITY;
#pragma unroll
    for (int k = 2; k <= P; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool desc = (i & k) == 0;
                    const T x = u[i], y = u[l];
                    const bool sw = desc ? (x < y) : (x > y);
                    u[i] = sw ? y : x;
                    u[l] = sw ? x : y;
                }
            }
    T css = T(0), tau = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (j < C) {
            css += u[j];
            const T t = (css - T(1)) / T(j + 1);
            if (u[j] - t > T(0)) tau = t;
        }
    }
    return tau;
}

template <int C> struct Pow2 { static constexpr int v = C <= 4 ? 4 : C <= 8 ? 8 : C <= 16 ? 16 : 32; };

// Calls BODY with LMAX bound to the smallest register-row size >= C.
#define DCRF_DISPATCH_ROWS(C, BODY)                                 \
    do {                                                           \
        if ((C) <= 4) { constexpr int LMAX = 4; BODY; }            \
        else if ((C) <= 8) { constexpr int LMAX = 8; BODY; }       \
        else if ((C) <= 16) { constexpr int LMAX = 16; BODY; }     \
        else if ((C) <= 24) { constexpr int LMAX = 24; BODY; }     \
        else { constexpr int LMAX = 32; BODY; }                    \
    } while (0)

}  // namespace dcrf
