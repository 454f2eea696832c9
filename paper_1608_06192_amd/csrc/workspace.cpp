// Upper bound of the device memory a context needs, for the workspace a
// caller hands to dcrf_set_image / dcrf_set_images (see include/dcrf.h).
//
// The bound mirrors every buffer the library keeps or takes for a while, at
// the largest size the inputs allow: a lattice of kernel m over N pixels has
// at most N (d_m + 1) vertices (every vertex holds at least one pixel), the
// inverse index at most N (d_m + 1) entries. Each block is counted with its
// 256-byte rounding plus one granule for the allocator's fragmentation, and
// the transient buffers of the lattice build (sort keys, renumbering tables,
// sort scratch) once, at their largest. The limits under which the bound
// holds are those stated in the header: filter calls of at most L channels,
// dense splat chunks of at most 64 entries, traces, histories and unrolled
// iterations of at most 4096 steps.

#include <algorithm>
#include <cstddef>

#include "dcrf_internal.h"

namespace dcrf {
namespace {

constexpr size_t kMaxSteps = 4096;     // traces, histories, unrolled iterations
constexpr size_t kMaxDenseChunk = 64;  // dense splat chunk length with a workspace
constexpr size_t kScanTileB = 256 * 16;  // items per tile of the device scans

struct Sum {
    size_t total = 0;
    void add(size_t bytes) {
        const size_t b = std::max<size_t>(bytes, 256);
        total += (b + 255) / 256 * 256 + 256;
    }
};

size_t pow2_slots(size_t n) {
    size_t cap = 1024;
    while (cap < 2 * n) cap <<= 1;
    return cap;
}

// scratch of the device radix sort of n (key, value) pairs of 32 bits:
// alternate key and value buffers, digit histograms and look-back state
size_t sort_scratch(size_t n) { return 16 * n + n + (1u << 20); }

size_t row_stride_b(int C, size_t e) {
    const size_t q = 16 / e;
    return (size_t(C) + q - 1) / q * q;
}

// the lattice arrays kept for one lattice over N pixel rows (n pairs)
void lattice_kept(Sum &s, size_t N, int d, size_t n, size_t cap, int L, size_t e) {
    const size_t D1 = size_t(d) + 1, M = n;
    s.add(cap * 8);                          // hash keys
    s.add(cap * 4);                          // slot -> vertex id
    s.add(n * 4);                            // per-pair hash slot
    s.add(n * 4);                            // per-pair vertex id
    s.add(n * e);                            // per-pair weight
    s.add(M * 8);                            // vertex keys
    s.add(D1 * M * 8);                       // neighbour table
    s.add(N * size_t(d) * e);                // features (exact mode)
    for (int i = 0; i < 3; ++i) s.add((M + 1) * 4);   // CSR offsets, counts, chunk scan
    s.add(n * 4);                            // entry pixels
    s.add(n * e);                            // entry weights
    s.add(n * 4);                            // entry vertices
    const size_t nch = M + n / 16 + 1;       // chunks of at least 16 entries
    s.add(nch * 16);                         // one-hot splat chunks
    s.add(nch * 16);                         // dense splat chunks
    const size_t dent = M * kMaxDenseChunk + n;
    s.add(dent * 4);                         // dense chunk pixels (padded)
    s.add(dent * e);                         // dense chunk weights (padded)
    const size_t ld = row_stride_b(std::max(L, 1), e);
    for (int i = 0; i < 3; ++i) s.add(M * ld * e);      // vertex values
    const size_t g2 = (D1 + 1) / 2 * 9, g3 = (D1 + 2) / 3 * 27;
    for (int i = 0; i < 2; ++i) s.add(std::max(g2, g3) * M * 4);   // blur path tables
    // per-tile vertex slots (tile launch shape)
    const size_t nt = N / 256 + 64;
    s.add(n * 4);                            // slot vertices
    s.add((n + 1) * 4);                      // slot pair offsets
    s.add((nt + 1) * 4);                     // tile slot offsets
    s.add(n * 2);                            // pair -> slot
    s.add(n);                                // slot pairs: pixel
    s.add(n * e);                            // slot pairs: weight
    s.add(n * 2);                            // slot pairs: slot
    s.add((M + 1) * 4);                      // vertex slot offsets
    s.add(n * 4);                            // vertex slots
}

// transient buffers of building one lattice (the largest of its stages)
size_t lattice_transient(size_t N, size_t n) {
    const size_t M = n, nch = M + n / 16 + 1;
    const size_t renumber = 5 * M * 4 + M * 8 + sort_scratch(M);
    const size_t inverse = 4 * n * 4 + sort_scratch(n);
    const size_t chunks = 4 * nch * 4 + nch * 16 + sort_scratch(nch);
    const size_t tiles = 2 * n * 8 + 2 * n * 4 + sort_scratch(n) + 2 * (n + 1) * 4 +
                         (M + 1) * 4 + N * 5 + (N / 256 + 65) * 4;
    return std::max({renumber, inverse, chunks, tiles}) + 16 * 256;
}

}  // namespace

size_t workspace_bound(int B, const int *H, const int *W, int L,
                       const dcrf_kernel *k, int nk, int dtype) {
    const size_t e = dtype == DCRF_F64 ? 8 : 4;
    // pixel rows: images start at multiples of 64 rows in a batch
    size_t N = 0, Nmax = 0;
    for (int j = 0; j < B; ++j) {
        const size_t n = size_t(H[j]) * size_t(W[j]);
        N = (B > 1) ? (N + n + 63) / 64 * 64 : n;
        Nmax = std::max(Nmax, n);
    }
    const size_t NL = N * size_t(L);
    Sum s;
    size_t transient = 0, nmax_pairs = 0, maxcap = 1024;
    for (int m = 0; m < nk; ++m) {
        const int d = k[m].use_rgb ? 5 : 2;
        const size_t n = N * size_t(d + 1);
        const size_t cap = pow2_slots(n);
        lattice_kept(s, N, d, n, cap, L, e);
        transient = std::max(transient, lattice_transient(N, n));
        nmax_pairs = std::max(nmax_pairs, n);
        maxcap = std::max(maxcap, cap);
        if (B > 1) {
            // the batch keeps every image's build (pairs, weights, neighbours,
            // keys, offsets, entries) until it concatenates them, and builds
            // the images in a scratch context one by one
            for (int j = 0; j < B; ++j) {
                const size_t nj = size_t(H[j]) * size_t(W[j]) * size_t(d + 1);
                s.add(nj * 4);
                s.add(nj * e);
                s.add(size_t(d + 1) * nj * 8);
                s.add(nj * 8);
                s.add((nj + 1) * 4);
                s.add(nj * 4);
                s.add(nj * e);
                s.add(nj * 4);
            }
            const size_t nj = Nmax * size_t(d + 1);
            lattice_kept(s, Nmax, d, nj, pow2_slots(nj), 1, e);
        }
    }
    s.add(transient);
    // context arrays
    s.add(size_t(2 * B) * 4 + 64);                     // image segments
    s.add(64 + 4 * ((maxcap + 2 * nmax_pairs) / kScanTileB + 8));   // flags, scans
    s.add(N * e);                                      // r = K'1
    s.add(NL * e);                                     // scratch arrays A, B
    s.add(NL * e);
    s.add((N / 256 + 64) * 16);                        // pixel tiles
    s.add(size_t(B + 1) * 4);
    s.add(4);                                          // input error flag
    s.add(size_t(L) * L * e);                          // Potts copy of mu
    s.add(4096);                                       // per-call flags and tables
    s.add(256);                                        // persistent solve's grid barrier
    // separable mode: taps (at most the larger image side) and three N x L arrays
    size_t side = 1;
    for (int j = 0; j < B; ++j) side = std::max<size_t>(side, std::max(H[j], W[j]));
    s.add(side * e);
    for (int i = 0; i < 3; ++i) s.add(NL * e);
    for (int i = 0; i < 3; ++i) s.add(NL * e);         // the LP on a label subset
    for (int i = 0; i < 3; ++i) s.add(NL * e);         // packed per-image arguments
    // Frank-Wolfe, DC_gen, DC_neg, energy
    for (int i = 0; i < 3; ++i) s.add(NL * e);         // c, P_y, P_s
    s.add(N * 4);                                      // s
    s.add(N * 4);                                      // previous s
    // tiles of the per-pixel kernels: at least 64 pixels up to 32 labels,
    // (256 / L) * 8 above (one lane per label)
    const size_t tp = L <= 32 ? 64 : std::max<size_t>(8, size_t(256 / L) * 8);
    const size_t tiles = N / tp + size_t(B) + 64;
    s.add(tiles * 10 * 8);                             // partial sums
    s.add(2 * 8 * size_t(B) * 10 * 8);                 // step accumulators
    s.add(kMaxSteps * size_t(B) * 4 * 8);              // trace
    s.add(size_t(L) * e);                              // sum_j |mu_ij|
    s.add((kMaxSteps + 1) * tiles * 8);                // S history partial sums
    if (B == 1) {
        // LP: sort keys and values, digit histograms, subgradient, per-lattice
        // sub-lattice tables of 2 N (d+1) slots
        s.add(N * 8);
        s.add(N * 8);
        s.add(N * 4);
        s.add(N * 4);
        s.add((256 * (N / 2048 + 1) + 1) * 8);
        s.add(NL * e);
        s.add(1024 * 8);
        s.add(N * e);
        s.add(N * 4);                                  // sorted position of every pixel
        s.add(N * e);                                  // a subtree's column y(T)
        s.add(size_t(kMaxTreeNodes) * size_t(L) * 4);  // the subtrees' label lists
        for (int m = 0; m < nk; ++m) {
            const size_t D1 = k[m].use_rgb ? 6 : 3, E = N * D1;
            s.add(2 * E * 8);
            s.add(2 * E * 4);
            s.add(E * 4);
            s.add(E * 4);
            s.add(E * 8);
            const size_t dense = lp_dense_cap(E), ld = std::max(E, dense);
            s.add(ld * D1 * 8);
            s.add(dense * 4);                          // dense levels' marks
            for (int i = 0; i < 3; ++i) s.add(ld * 2 * e);
            s.add(E * 4);
            s.add(E * e);
        }
    }
    // derivative: adjoints and reverse-sweep sums (the checkpoint buffer
    // itself is the caller's)
    for (int i = 0; i < 5; ++i) s.add(NL * e);
    for (int m = 0; m < nk; ++m) s.add(N * e);
    s.add(tiles * (1 + 3 * DCRF_MAXK) * 8);
    s.add(size_t(L) * e);
    s.add(N * e);
    s.add(2 * 8 * size_t(B) * (1 + 3 * DCRF_MAXK) * 8);
    s.add(size_t(B) * size_t(nk) * 8);
    s.add(kMaxSteps * size_t(B) * 2 * 8);
    s.add(size_t(B) * (kMaxSteps + 1) * 8);
    // room for the holes that freed blocks leave between kept ones
    return s.total + s.total / 8;
}

}  // namespace dcrf
