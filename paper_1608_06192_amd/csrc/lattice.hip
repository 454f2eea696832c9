// Device construction of the permutohedral lattices of an image.
//
// The paper computes every pairwise message with the filter of Adams et al.
// (Sec. 3 "Filter-based Method", App. A) and gives no details of it. The
// lattice built here: each pixel's feature vector f (dimension d) is mapped
// onto the hyperplane sum(x) = 0 of R^{d+1} by an orthonormal basis scaled by
// s = (d+1) sqrt(2/3); the simplex of the lattice (d+1)A*_d that contains the
// point is found from the nearest remainder-0 point (round every coordinate
// to a multiple of d+1, then fix the coordinate sum by moving the coordinates
// that were rounded the farthest); its d+1 vertices and barycentric weights
// are stored per pixel. Vertices with weight 0 are not created, so the vertex
// set does not depend on how exact ties between coordinates are broken.
//
// The coordinates are computed in FP64 without contraction of multiply-adds
// (this file is compiled with -ffp-contract=off): which vertices exist is a
// discrete decision, and it has to be the same decision a plain IEEE
// evaluation of the same formulas takes.
//
// Vertices live in an open-addressing hash table of packed 64-bit keys
// (remainder in 3 bits, the first d coordinates divided by d+1 in the rest),
// filled with atomicCAS. Occupied slots are compacted into dense vertex ids
// by a block scan, and a neighbour table stores, for each vertex and blur
// direction u_j = (d+1) e_j - 1, the ids of v + u_j and v - u_j.

#include <algorithm>
#include <cmath>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "dcrf_internal.h"
#include "hash_scan.h"

namespace dcrf {
namespace {

constexpr int kFlagRange = 1;
constexpr int kFlagCapacity = 2;
constexpr int kFlagNonFinite = 4;

template <int D>
struct Codec {
    static constexpr int kBits = (64 - 3) / D;
    static constexpr long long kBias = 1ll << (kBits - 1);
    static constexpr unsigned long long kMask = (1ull << kBits) - 1;

    // coords: the first D coordinates of a vertex, all congruent to rem
    __device__ static bool encode(const int (&coord)[D], int rem,
                                  uint64_t &key) {
        uint64_t k = uint64_t(rem);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            long long q = (long long)(coord[i] - rem) / (D + 1) + kBias;
            if (q < 0 || q > (long long)kMask) return false;
            k |= uint64_t(q) << (3 + kBits * i);
        }
        key = k;
        return true;
    }
    __device__ static void decode(uint64_t key, int (&coord)[D], int &rem) {
        rem = int(key & 7u);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            long long q = (long long)((key >> (3 + kBits * i)) & kMask) - kBias;
            coord[i] = int(q * (D + 1) + rem);
        }
    }
};


// Elevation matrix (d+1 x d), scaled, passed by value.
template <int D>
struct Elev {
    double e[D + 1][D];
};

template <int D>
Elev<D> make_elevation() {
    Elev<D> E;
    const double s = double(D + 1) * std::sqrt(2.0 / 3.0);
    for (int j = 0; j < D; ++j) {
        const double cj = s / std::sqrt(double((j + 1) * (j + 2)));
        for (int i = 0; i <= D; ++i)
            E.e[i][j] = (i <= j) ? cj : (i == j + 1 ? -double(j + 1) * cj : 0.0);
    }
    return E;
}

// rank[i]: position of coordinate i in descending order of delta, equal
// values ordered by lower index first
template <int D>
__device__ __forceinline__ void ranks(const double (&delta)[D + 1],
                                      int (&rank)[D + 1]) {
#pragma unroll
    for (int i = 0; i <= D; ++i) {
        int r = 0;
#pragma unroll
        for (int j = 0; j <= D; ++j)
            r += (delta[j] > delta[i] || (delta[j] == delta[i] && j < i)) ? 1 : 0;
        rank[i] = r;
    }
}

// One thread per pixel: features -> elevated point -> enclosing simplex ->
// insert the vertices with positive weight into the hash table.
template <int D, typename T>
__global__ void __launch_bounds__(256)
k_lattice_points(int N, int W, const float *__restrict__ rgb, double theta_pos,
                 double theta_rgb, Elev<D> E, uint64_t *__restrict__ hkeys,
                 uint64_t capmask, uint32_t *__restrict__ pix_slot,
                 T *__restrict__ pix_w, int *__restrict__ flags) {
#pragma clang fp contract(off)
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    constexpr int D1 = D + 1;
    const int row = a / W;
    const int col = a - row * W;
    double f[D];
    f[0] = double(col) / theta_pos;
    f[1] = double(row) / theta_pos;
    if constexpr (D == 5) {
        f[2] = double(rgb[3 * (size_t)a + 0]) / theta_rgb;
        f[3] = double(rgb[3 * (size_t)a + 1]) / theta_rgb;
        f[4] = double(rgb[3 * (size_t)a + 2]) / theta_rgb;
    }
    double x[D1];
#pragma unroll
    for (int i = 0; i < D1; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) acc += E.e[i][j] * f[j];
        x[i] = acc;
    }
    // non-finite colours, and coordinates too large for the integer vertex
    // coordinates (a tiny theta), are reported, not used
    bool fin = true, finite = true;
#pragma unroll
    for (int j = 0; j < D; ++j) fin = fin && isfinite(f[j]);
#pragma unroll
    for (int i = 0; i < D1; ++i) finite = finite && (fabs(x[i]) < 1.0e9);
    if (!fin || !finite) {
        atomicOr(flags, fin ? kFlagRange : kFlagNonFinite);
#pragma unroll
        for (int k = 0; k < D1; ++k) {
            pix_w[(size_t)a * D1 + k] = T(0);
            pix_slot[(size_t)a * D1 + k] = 0xffffffffu;
        }
        return;
    }
    double c[D1], delta[D1];
    int rank[D1];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < D1; ++i) {
        c[i] = double(D1) * floor(x[i] / double(D1) + 0.5);
        sum += int(llrint(c[i])) / D1;
    }
#pragma unroll
    for (int i = 0; i < D1; ++i) delta[i] = x[i] - c[i];
    ranks<D>(delta, rank);
    if (sum != 0) {
#pragma unroll
        for (int i = 0; i < D1; ++i) {
            if (sum > 0 && rank[i] >= D1 - sum) c[i] -= double(D1);
            if (sum < 0 && rank[i] < -sum) c[i] += double(D1);
        }
#pragma unroll
        for (int i = 0; i < D1; ++i) delta[i] = x[i] - c[i];
        ranks<D>(delta, rank);
    }
    // sorted offsets y_0 >= ... >= y_D, selected without dynamic indexing
    double y[D1];
#pragma unroll
    for (int p = 0; p < D1; ++p) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < D1; ++i) v = (rank[i] == p) ? delta[i] : v;
        y[p] = v;
    }
    double b[D1];
    b[0] = 1.0 - (y[0] - y[D]) / double(D1);
#pragma unroll
    for (int p = 0; p < D; ++p) b[D - p] = (y[p] - y[p + 1]) / double(D1);

    int ci[D1];
#pragma unroll
    for (int i = 0; i < D1; ++i) ci[i] = int(llrint(c[i]));

#pragma unroll
    for (int k = 0; k < D1; ++k) {
        const size_t e = (size_t)a * D1 + k;
        pix_w[e] = T(b[k] > 0.0 ? b[k] : 0.0);
        uint32_t slot = 0xffffffffu;
        if (b[k] > 0.0) {
            int coord[D];
#pragma unroll
            for (int i = 0; i < D; ++i)
                coord[i] = ci[i] + k - (rank[i] > D - k ? D1 : 0);
            uint64_t key;
            if (!Codec<D>::encode(coord, k, key)) {
                atomicOr(flags, kFlagRange);
            } else {
                uint64_t h = mix64(key) & capmask;
                uint64_t probe = 0;
                for (; probe <= capmask; ++probe) {
                    unsigned long long prev = atomicCAS(
                        (unsigned long long *)&hkeys[h],
                        (unsigned long long)kEmpty, (unsigned long long)key);
                    if (prev == kEmpty || prev == key) break;
                    h = (h + 1) & capmask;
                }
                if (probe > capmask)
                    atomicOr(flags, kFlagCapacity);
                else
                    slot = uint32_t(h);
            }
        }
        pix_slot[e] = slot;
    }
}

// ---- per-vertex inverse index: the (pixel, weight) pairs of each vertex ----

__global__ void k_csr_count(size_t cnt, const int *__restrict__ pix_vid,
                            int *__restrict__ counts) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    const int v = pix_vid[e];
    if (v >= 0) atomicAdd(&counts[v], 1);
}

// sort keys of the pixel-vertex pairs: the vertex id, or the largest key of
// `bits` bits where the weight is 0 (those sort last and are dropped)
__global__ void k_ref_keys(size_t cnt, const int *__restrict__ pix_vid,
                           uint32_t none, uint32_t *__restrict__ keys,
                           uint32_t *__restrict__ refs) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    const int v = pix_vid[e];
    keys[e] = v >= 0 ? uint32_t(v) : none;
    refs[e] = uint32_t(e);
}

// entries from the pairs sorted by vertex (stable, so each vertex's pixels
// stay in raster order)
template <typename T>
__global__ void k_entries(int nent, int D1, const uint32_t *__restrict__ keys,
                          const uint32_t *__restrict__ refs,
                          const T *__restrict__ pix_w, int *__restrict__ ent_pix,
                          T *__restrict__ ent_w, int *__restrict__ ent_v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nent) return;
    const uint32_t ref = refs[i];
    ent_pix[i] = int(ref / uint32_t(D1));
    ent_w[i] = pix_w[ref];
    ent_v[i] = int(keys[i]);
}

__global__ void k_chunk_keys(int n, const int4 *__restrict__ chunks,
                             const int *__restrict__ ent_pix,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = uint32_t(ent_pix[chunks[i].y]);
    idx[i] = uint32_t(i);
}

__global__ void k_chunk_permute(int n, const uint32_t *__restrict__ idx,
                                const int4 *__restrict__ in, int4 *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[idx[i]];
}

int key_bits(unsigned long long maxval) {
    int b = 1;
    while (b < 32 && (1ull << b) <= maxval) ++b;
    return b;
}

// stable LSD radix sort of (key, value) pairs of u32 on the stream, keys
// using their low `bits` bits
void sort_pairs(dcrf_ctx *ctx, const uint32_t *kin, uint32_t *kout,
                const uint32_t *vin, uint32_t *vout, int n, int bits,
                DevBuf &temp) {
    size_t bytes = 0;
    DCRF_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin,
                                                   vout, n, 0, bits, ctx->stream));
    temp.ensure(bytes, ctx->stream);
    DCRF_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, bytes, kin, kout, vin,
                                                   vout, n, 0, bits, ctx->stream));
}

__global__ void k_chunk_count(int M, const int *__restrict__ off, int chunk,
                              int *__restrict__ nch) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= M) return;
    const int len = off[v + 1] - off[v];
    nch[v] = (len + chunk - 1) / chunk;
}

__global__ void k_chunk_fill(int M, const int *__restrict__ off,
                             const int *__restrict__ choff, int chunk,
                             int4 *__restrict__ chunks) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= M) return;
    const int b = off[v], e = off[v + 1];
    int c = choff[v];
    for (int s = b; s < e; s += chunk, ++c)
        chunks[c] = make_int4(v, s, min(e, s + chunk), 0);
}

__global__ void k_pixel_ids(size_t count, const uint32_t *__restrict__ pix_slot,
                            const int *__restrict__ slot_vid,
                            int *__restrict__ pix_vid) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    uint32_t s = pix_slot[e];
    pix_vid[e] = (s == 0xffffffffu) ? -1 : slot_vid[s];
}

// ---- vertex order: by the first pixel-vertex pair that touches the vertex --
//
// Compaction numbers the vertices in hash-slot order, which scatters the
// vertices of neighbouring pixels over the whole vertex array. Renumbering
// them by their first pair (pixel a, simplex corner k: index a (d+1) + k,
// unique per vertex) puts the vertices of nearby pixels at nearby ids: the
// vertex rows gathered by a wave of neighbouring pixels share cache lines,
// and the pixel band that one XCD works on maps to one range of rows. The
// order does not depend on the hash table's layout.

__global__ void k_first_pair(size_t cnt, const uint32_t *__restrict__ pix_slot,
                             const int *__restrict__ slot_vid,
                             uint32_t *__restrict__ first) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    const uint32_t sl = pix_slot[e];
    if (sl != 0xffffffffu) atomicMin(&first[slot_vid[sl]], uint32_t(e));
}

__global__ void k_iota_u32(int n, uint32_t *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = uint32_t(i);
}

// order[i]: old id of the vertex that becomes id i
__global__ void k_renumber(int M, const uint32_t *__restrict__ order,
                           const uint64_t *__restrict__ vkeys_old,
                           uint64_t *__restrict__ vkeys_new, int *__restrict__ newid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const uint32_t v = order[i];
    newid[v] = i;
    vkeys_new[i] = vkeys_old[v];
}

__global__ void k_remap_slots(size_t cap, const int *__restrict__ newid,
                              int *__restrict__ slot_vid) {
    const size_t sl = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= cap) return;
    const int v = slot_vid[sl];
    if (v >= 0) slot_vid[sl] = newid[v];
}

template <int D>
__device__ int hash_lookup(const uint64_t *__restrict__ hkeys, uint64_t capmask,
                           const int *__restrict__ slot_vid, uint64_t key) {
    uint64_t h = mix64(key) & capmask;
    for (uint64_t probe = 0; probe <= capmask; ++probe) {
        uint64_t k = hkeys[h];
        if (k == key) return slot_vid[h];
        if (k == kEmpty) return -1;
        h = (h + 1) & capmask;
    }
    return -1;
}

template <int D>
__global__ void __launch_bounds__(256)
k_neighbours(int M, const uint64_t *__restrict__ vkeys,
             const uint64_t *__restrict__ hkeys, uint64_t capmask,
             const int *__restrict__ slot_vid, int *__restrict__ nbr) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= M) return;
    constexpr int D1 = D + 1;
    int coord[D], rem;
    Codec<D>::decode(vkeys[v], coord, rem);
#pragma unroll
    for (int j = 0; j < D1; ++j) {
#pragma unroll
        for (int sgn = 0; sgn < 2; ++sgn) {
            const int s = sgn == 0 ? 1 : -1;
            int cn[D];
#pragma unroll
            for (int i = 0; i < D; ++i) cn[i] = coord[i] + s * (i == j ? D : -1);
            const int rn = (rem - s + D1) % D1;
            uint64_t key;
            int id = -1;
            if (Codec<D>::encode(cn, rn, key))
                id = hash_lookup<D>(hkeys, capmask, slot_vid, key);
            nbr[((size_t)j * M + v) * 2 + sgn] = id;
        }
    }
}

template <typename T>
__global__ void k_features(int N, int W, const float *__restrict__ rgb,
                           int use_rgb, double theta_pos, double theta_rgb,
                           T *__restrict__ feat) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int row = a / W;
    const int col = a - row * W;
    const int d = use_rgb ? 5 : 2;
    T *f = feat + (size_t)a * d;
    f[0] = T(double(col) / theta_pos);
    f[1] = T(double(row) / theta_pos);
    if (use_rgb) {
        for (int c = 0; c < 3; ++c)
            f[2 + c] = T(double(rgb[3 * (size_t)a + c]) / theta_rgb);
    }
}

// Inverse index of lattice m: for each vertex the (pixel, weight) pairs that
// splat into it, split into chunks of at most `chunk` pairs; the gather splat
// runs one group of lanes per chunk.
void chunk_index(dcrf_ctx *ctx, int m);

template <typename T>
void build_inverse_index(dcrf_ctx *ctx, int m) {
    Lattice &L = ctx->lat[m];
    const hipStream_t s = ctx->stream;
    const int M = L.M, D1 = L.d + 1;
    const size_t cnt = (size_t)ctx->N * D1;
    L.chunk = ctx->splat_chunk;
    L.dchunk = ctx->dense_chunk;
    L.csr_off.ensure((size_t)(M + 1) * 4, s);
    L.csr_tmp.ensure((size_t)(M + 1) * 4, s);
    L.ent_pix.ensure(cnt * 4, s);
    L.ent_w.ensure(cnt * sizeof(T), s);
    L.ent_v.ensure(cnt * 4, s);
    int *counts = L.csr_tmp.as<int>();
    DCRF_TRY_HIP(hipMemsetAsync(counts, 0, (size_t)(M + 1) * 4, s));
    hipLaunchKernelGGL(k_csr_count, dim3(ceil_div((long long)cnt, 256)), dim3(256),
                       0, s, cnt, L.pix_vid.as<int>(), counts);
    scan_ints(ctx, counts, M, L.csr_off.as<int>());
    DCRF_TRY_HIP(hipMemcpyAsync(&L.nent, L.csr_off.as<int>() + M, 4,
                                hipMemcpyDeviceToHost, s));
    // entries: the pixel-vertex pairs stably sorted by vertex
    DevBuf k0, k1, v0, v1, temp;
    struct Free {
        DevBuf *b[5];
        ~Free() { for (DevBuf *x : b) x->release(); }
    } fr{{&k0, &k1, &v0, &v1, &temp}};
    for (DevBuf *b : {&k0, &k1, &v0, &v1}) b->ensure(cnt * 4, s);
    const int bits = key_bits((unsigned long long)M);
    hipLaunchKernelGGL(k_ref_keys, dim3(ceil_div((long long)cnt, 256)), dim3(256), 0,
                       s, cnt, L.pix_vid.as<int>(), uint32_t((1ull << bits) - 1),
                       k0.as<uint32_t>(), v0.as<uint32_t>());
    sort_pairs(ctx, k0.as<uint32_t>(), k1.as<uint32_t>(), v0.as<uint32_t>(),
               v1.as<uint32_t>(), int(cnt), bits, temp);
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    if (L.nent > 0)
        hipLaunchKernelGGL((k_entries<T>), dim3(ceil_div(L.nent, 256)), dim3(256), 0,
                           s, L.nent, D1, k1.as<uint32_t>(), v1.as<uint32_t>(),
                           L.pix_w.as<T>(), L.ent_pix.as<int>(), L.ent_w.as<T>(),
                           L.ent_v.as<int>());
    DCRF_CHECK_LAUNCH();
    chunk_index(ctx, m);
    DCRF_TRY_HIP(hipStreamSynchronize(s));
}

// chunk list of lattice m from its inverse index (csr_off) and L.chunk
// a chunk list of lattice m from its inverse index (csr_off): chunks of at
// most `len` entries, ordered by their first pixel (the splats then walk the
// image roughly in raster order, and with the XCD mapping of their blocks
// each L2 sees one band of the image's rows)
void chunk_list(dcrf_ctx *ctx, int m, int len, DevBuf &out, int &count) {
    Lattice &L = ctx->lat[m];
    const hipStream_t s = ctx->stream;
    const int M = L.M;
    int *counts = L.csr_tmp.as<int>();
    if (M > 0)
        hipLaunchKernelGGL(k_chunk_count, dim3(ceil_div(M, 256)), dim3(256), 0, s,
                           M, L.csr_off.as<int>(), len, counts);
    L.chunk_off.ensure((size_t)(M + 1) * 4, s);
    scan_ints(ctx, counts, M, L.chunk_off.as<int>());
    int nch = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&nch, L.chunk_off.as<int>() + M, 4,
                                hipMemcpyDeviceToHost, s));
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    count = nch;
    out.ensure((size_t)std::max(nch, 1) * sizeof(int4), s);
    if (M > 0)
        hipLaunchKernelGGL(k_chunk_fill, dim3(ceil_div(M, 256)), dim3(256), 0, s,
                           M, L.csr_off.as<int>(), L.chunk_off.as<int>(), len,
                           out.as<int4>());
    DCRF_CHECK_LAUNCH();
    if (nch <= 1) return;
    DevBuf k0, k1, v0, v1, temp, tmp;
    struct Free {
        DevBuf *b[6];
        ~Free() { for (DevBuf *x : b) x->release(); }
    } fr{{&k0, &k1, &v0, &v1, &temp, &tmp}};
    for (DevBuf *b : {&k0, &k1, &v0, &v1}) b->ensure((size_t)nch * 4, s);
    tmp.ensure((size_t)nch * sizeof(int4), s);
    hipLaunchKernelGGL(k_chunk_keys, dim3(ceil_div(nch, 256)), dim3(256), 0, s, nch,
                       out.as<int4>(), L.ent_pix.as<int>(), k0.as<uint32_t>(),
                       v0.as<uint32_t>());
    sort_pairs(ctx, k0.as<uint32_t>(), k1.as<uint32_t>(), v0.as<uint32_t>(),
               v1.as<uint32_t>(), nch, key_bits((unsigned long long)ctx->N), temp);
    DCRF_TRY_HIP(hipMemcpyAsync(tmp.p, out.p, (size_t)nch * sizeof(int4),
                                hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_chunk_permute, dim3(ceil_div(nch, 256)), dim3(256), 0, s, nch,
                       v1.as<uint32_t>(), tmp.as<int4>(), out.as<int4>());
    DCRF_CHECK_LAUNCH();
    DCRF_TRY_HIP(hipStreamSynchronize(s));
}

// the entries of each dense chunk at a stride of U (the staged splats then
// load a block's entries as one contiguous range, without waiting for the
// chunk descriptors)
template <typename T>
__global__ void k_dense_pad(long long n, int U, const int4 *__restrict__ chunks,
                            const int *__restrict__ ent_pix, const T *__restrict__ ent_w,
                            int32_t *__restrict__ dpix, T *__restrict__ dw) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long c = i / U;
    const int j = int(i - c * U);
    const int4 cd = chunks[c];
    const int e = cd.y + j;
    dpix[i] = e < cd.z ? ent_pix[e] : 0;
    dw[i] = e < cd.z ? ent_w[e] : T(0);
}

// both chunk lists of lattice m: for the one-hot splat (L.chunk entries) and
// for the dense splat (L.dchunk entries), and the dense chunks' entries
void chunk_index(dcrf_ctx *ctx, int m) {
    Lattice &L = ctx->lat[m];
    chunk_list(ctx, m, L.chunk, L.chunks, L.nchunks);
    chunk_list(ctx, m, L.dchunk, L.dchunks, L.ndchunks);
    const long long n = (long long)L.ndchunks * L.dchunk;
    const hipStream_t s = ctx->stream;
    L.dpix.ensure((size_t)std::max(n, 1ll) * 4, s);
    L.dw.ensure((size_t)std::max(n, 1ll) * ctx->elt(), s);
    if (n > 0) {
        if (ctx->dtype == DCRF_F64)
            hipLaunchKernelGGL((k_dense_pad<double>), dim3(ceil_div(n, 256ll)), dim3(256), 0,
                               s, n, L.dchunk, L.dchunks.as<int4>(), L.ent_pix.as<int>(),
                               L.ent_w.as<double>(), L.dpix.as<int32_t>(), L.dw.as<double>());
        else
            hipLaunchKernelGGL((k_dense_pad<float>), dim3(ceil_div(n, 256ll)), dim3(256), 0,
                               s, n, L.dchunk, L.dchunks.as<int4>(), L.ent_pix.as<int>(),
                               L.ent_w.as<float>(), L.dpix.as<int32_t>(), L.dw.as<float>());
        DCRF_CHECK_LAUNCH();
    }
}

template <int D, typename T>
void build_one(dcrf_ctx *ctx, int m, const float *rgb, int *flags_dev) {
    Lattice &L = ctx->lat[m];
    const dcrf_kernel &k = ctx->kern[m];
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    constexpr int D1 = D + 1;
    L.d = D;
    L.gamma = std::pow(4.0 * M_PI / 3.0, 0.5 * D) * std::sqrt(double(D1));
    const size_t cap = hash_slots(ctx, (size_t)N * D1);
    L.cap = cap;
    L.hkeys.ensure(cap * 8, s);
    L.slot_vid.ensure(cap * 4, s);
    L.pix_slot.ensure((size_t)N * D1 * 4, s);
    L.pix_vid.ensure((size_t)N * D1 * 4, s);
    L.pix_w.ensure((size_t)N * D1 * sizeof(T), s);
    DCRF_TRY_HIP(hipMemsetAsync(L.hkeys.p, 0xff, cap * 8, s));

    hipLaunchKernelGGL((k_lattice_points<D, T>), dim3(ceil_div(N, 256)),
                       dim3(256), 0, s, N, ctx->W, rgb, k.theta_pos,
                       k.theta_rgb, make_elevation<D>(), L.hkeys.as<uint64_t>(),
                       uint64_t(cap - 1), L.pix_slot.as<uint32_t>(),
                       L.pix_w.as<T>(), flags_dev);
    DCRF_CHECK_LAUNCH();

    // the caller sized the scratch for the largest lattice (see build_all)
    const int ntiles = ceil_div((long long)cap, kScanTile);
    int *tiles = reinterpret_cast<int *>(ctx->scratch.as<char>() + 64);
    hipLaunchKernelGGL(k_count_occupied, dim3(ntiles), dim3(kScanThreads), 0,
                       s, L.hkeys.as<uint64_t>(), cap, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, tiles,
                       ntiles);
    int M = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&M, tiles + ntiles, 4, hipMemcpyDeviceToHost, s));
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    L.M = M;
    L.vkeys.ensure((size_t)(M > 0 ? M : 1) * 8, s);
    hipLaunchKernelGGL(k_assign_ids, dim3(ntiles), dim3(kScanThreads), 0, s,
                       L.hkeys.as<uint64_t>(), cap, tiles,
                       L.slot_vid.as<int>(), L.vkeys.as<uint64_t>());
    const size_t cnt = (size_t)N * D1;
    if (M > 1) {
        DevBuf first, k1, v0, v1, newid, vk, temp;
        struct Free {
            DevBuf *b[7];
            ~Free() { for (DevBuf *x : b) x->release(); }
        } fr{{&first, &k1, &v0, &v1, &newid, &vk, &temp}};
        for (DevBuf *b : {&first, &k1, &v0, &v1, &newid}) b->ensure((size_t)M * 4, s);
        vk.ensure((size_t)M * 8, s);
        DCRF_TRY_HIP(hipMemsetAsync(first.p, 0xff, (size_t)M * 4, s));
        hipLaunchKernelGGL(k_first_pair, dim3(ceil_div((long long)cnt, 256)), dim3(256),
                           0, s, cnt, L.pix_slot.as<uint32_t>(), L.slot_vid.as<int>(),
                           first.as<uint32_t>());
        hipLaunchKernelGGL(k_iota_u32, dim3(ceil_div(M, 256)), dim3(256), 0, s, M,
                           v0.as<uint32_t>());
        DCRF_CHECK_LAUNCH();
        sort_pairs(ctx, first.as<uint32_t>(), k1.as<uint32_t>(), v0.as<uint32_t>(),
                   v1.as<uint32_t>(), M, key_bits((unsigned long long)cnt), temp);
        hipLaunchKernelGGL(k_renumber, dim3(ceil_div(M, 256)), dim3(256), 0, s, M,
                           v1.as<uint32_t>(), L.vkeys.as<uint64_t>(), vk.as<uint64_t>(),
                           newid.as<int>());
        hipLaunchKernelGGL(k_remap_slots, dim3(ceil_div((long long)cap, 256)), dim3(256),
                           0, s, cap, newid.as<int>(), L.slot_vid.as<int>());
        DCRF_CHECK_LAUNCH();
        std::swap(L.vkeys, vk);
        DCRF_TRY_HIP(hipStreamSynchronize(s));
    }
    hipLaunchKernelGGL(k_pixel_ids, dim3(ceil_div((long long)cnt, 256)),
                       dim3(256), 0, s, cnt, L.pix_slot.as<uint32_t>(),
                       L.slot_vid.as<int>(), L.pix_vid.as<int>());
    L.nbr.ensure((size_t)D1 * (M > 0 ? M : 1) * 2 * 4, s);
    if (M > 0)
        hipLaunchKernelGGL((k_neighbours<D>), dim3(ceil_div(M, 256)), dim3(256),
                           0, s, M, L.vkeys.as<uint64_t>(),
                           L.hkeys.as<uint64_t>(), uint64_t(cap - 1),
                           L.slot_vid.as<int>(), L.nbr.as<int>());
    L.feat.ensure((size_t)N * D * sizeof(T), s);
    hipLaunchKernelGGL((k_features<T>), dim3(ceil_div(N, 256)), dim3(256), 0,
                       s, N, ctx->W, rgb, k.use_rgb, k.theta_pos, k.theta_rgb,
                       L.feat.as<T>());
    DCRF_CHECK_LAUNCH();
    build_inverse_index<T>(ctx, m);
}

template <typename T>
void build_all(dcrf_ctx *ctx, const float *rgb) {
    const hipStream_t s = ctx->stream;
    // scratch: 64 bytes of flags, then the tile counts of the compaction scan
    // of the largest hash table; sized once so no pointer into it goes stale
    size_t maxcap = 1024;
    for (int m = 0; m < ctx->nk; ++m) {
        const int D1 = (ctx->kern[m].use_rgb ? 5 : 2) + 1;
        maxcap = std::max(maxcap, hash_slots(ctx, (size_t)ctx->N * D1));
    }
    ctx->scratch.ensure(64 + (size_t)(ceil_div((long long)maxcap, kScanTile) + 1) * 4,
                        s);
    int *flags = ctx->scratch.as<int>();
    DCRF_TRY_HIP(hipMemsetAsync(flags, 0, 4, s));
    for (int m = 0; m < ctx->nk; ++m) {
        if (ctx->kern[m].use_rgb)
            build_one<5, T>(ctx, m, rgb, flags);
        else
            build_one<2, T>(ctx, m, rgb, flags);
    }
    int hflags = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, s));
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    if (hflags & kFlagNonFinite) fail(DCRF_EINVAL, "a colour value is not finite");
    if (hflags & kFlagRange)
        fail(DCRF_ERANGE,
             "lattice coordinates exceed the 64-bit vertex key range "
             "(theta too small for the image extent)");
    if (hflags & kFlagCapacity)
        fail(DCRF_ECAPACITY, "lattice hash table full: a lattice has more vertices "
                             "than hash slots");
}

}  // namespace

void build_lattices(dcrf_ctx *ctx, const float *rgb) {
    if (ctx->dtype == DCRF_F64)
        build_all<double>(ctx, rgb);
    else
        build_all<float>(ctx, rgb);
}

void rechunk(dcrf_ctx *ctx, int chunk, int dense_chunk) {
    int maxM = 0;
    for (int m = 0; m < ctx->nk; ++m) maxM = std::max(maxM, ctx->lat[m].M);
    // flags, then the tile sums of the scan over M + 1 counts
    ctx->scratch.ensure(64 + (size_t)(ceil_div((long long)maxM + 1, kScanTile) + 2) * 4,
                        ctx->stream);
    ctx->splat_chunk = chunk;
    ctx->dense_chunk = dense_chunk;
    for (int m = 0; m < ctx->nk; ++m) {
        ctx->lat[m].chunk = chunk;
        ctx->lat[m].dchunk = dense_chunk;
        chunk_index(ctx, m);
    }
}

void lattice_export(dcrf_ctx *ctx, int m, int32_t *keys, int32_t *vid,
                    double *w) {
    Lattice &L = ctx->lat[m];
    const hipStream_t s = ctx->stream;
    const int D = L.d, D1 = L.d + 1;
    const size_t cnt = (size_t)ctx->N * D1;
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    if (keys) {
        std::vector<uint64_t> k(L.M);
        DCRF_TRY_HIP(hipMemcpy(k.data(), L.vkeys.p, (size_t)L.M * 8,
                               hipMemcpyDeviceToHost));
        const int bits = (64 - 3) / D;
        const long long bias = 1ll << (bits - 1);
        const unsigned long long mask = (1ull << bits) - 1;
        for (int v = 0; v < L.M; ++v) {
            const int rem = int(k[v] & 7u);
            for (int i = 0; i < D; ++i) {
                long long q = (long long)((k[v] >> (3 + bits * i)) & mask) - bias;
                keys[(size_t)v * D + i] = int32_t(q * D1 + rem);
            }
        }
    }
    if (vid)
        DCRF_TRY_HIP(hipMemcpy(vid, L.pix_vid.p, cnt * 4, hipMemcpyDeviceToHost));
    if (w) {
        if (ctx->dtype == DCRF_F64) {
            DCRF_TRY_HIP(hipMemcpy(w, L.pix_w.p, cnt * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> wf(cnt);
            DCRF_TRY_HIP(hipMemcpy(wf.data(), L.pix_w.p, cnt * 4,
                                   hipMemcpyDeviceToHost));
            for (size_t i = 0; i < cnt; ++i) w[i] = wf[i];
        }
    }
}

}  // namespace dcrf
