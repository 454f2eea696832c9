// Internal declarations of the dcrf library: the context, device buffers and
// the host-side launchers of the kernels in lattice.hip, filter.hip and
// solvers.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "dcrf.h"

#define DCRF_MAXK 4

namespace dcrf {

// ---------------------------------------------------------------- errors

struct Error {
    int code;
    std::string msg;
};

#define DCRF_TRY_HIP(expr)                                                   \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            throw ::dcrf::Error{e_ == hipErrorOutOfMemory ? DCRF_ENOMEM      \
                                                          : DCRF_EHIP,       \
                                std::string(#expr) + ": " +                  \
                                    hipGetErrorString(e_)};                  \
    } while (0)

#define DCRF_CHECK_LAUNCH() DCRF_TRY_HIP(hipGetLastError())

inline void fail(int code, const std::string &msg) { throw Error{code, msg}; }

// ------------------------------------------------------- device buffers

// Device memory handed to a context by its caller (the workspace argument of
// dcrf_set_image): a first-fit allocator over that one range in 256-byte
// granules, with neighbouring free blocks merged. While a context holds
// one, every buffer of the context lives in it and the library calls
// neither hipMalloc nor hipFree for the context.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    size_t in_use = 0, peak = 0;
    hipStream_t stream = nullptr;   // the owner's stream, drained before reuse
    const char *refuse = nullptr;   // set: every allocation fails with this message
    struct Block { size_t off, bytes; bool used; };
    std::vector<Block> blocks;      // in offset order, covering [0, size)
    bool active() const { return base != nullptr; }
    void reset(void *mem, size_t bytes) {
        base = static_cast<char *>(mem);
        size = bytes & ~size_t(255);
        in_use = peak = 0;
        blocks.clear();
        if (base && size) blocks.push_back({0, size, false});
    }
    void *alloc(size_t need) {
        if (refuse) throw Error{DCRF_ENOMEM, refuse};
        const size_t n = (need + 255) & ~size_t(255);
        for (size_t i = 0; i < blocks.size(); ++i) {
            Block &b = blocks[i];
            if (b.used || b.bytes < n) continue;
            if (b.bytes > n)
                blocks.insert(blocks.begin() + i + 1, Block{b.off + n, b.bytes - n, false});
            blocks[i].bytes = n;
            blocks[i].used = true;
            in_use += n;
            if (in_use > peak) peak = in_use;
            return base + blocks[i].off;
        }
        throw Error{DCRF_ENOMEM, "workspace exhausted: " + std::to_string(n) +
                                     " more bytes needed (" + std::to_string(in_use) +
                                     " of " + std::to_string(size) + " in use)"};
    }
    void free(void *p) {
        const size_t off = size_t(static_cast<char *>(p) - base);
        for (size_t i = 0; i < blocks.size(); ++i) {
            if (blocks[i].off != off || !blocks[i].used) continue;
            // kernels still queued on the owner's stream may read the block
            (void)hipStreamSynchronize(stream);
            blocks[i].used = false;
            in_use -= blocks[i].bytes;
            if (i + 1 < blocks.size() && !blocks[i + 1].used) {
                blocks[i].bytes += blocks[i + 1].bytes;
                blocks.erase(blocks.begin() + i + 1);
            }
            if (i > 0 && !blocks[i - 1].used) {
                blocks[i - 1].bytes += blocks[i].bytes;
                blocks.erase(blocks.begin() + i);
            }
            return;
        }
    }
};

// The arena of the context whose call is running on this thread (set by
// the C ABI for the duration of each call), or null: buffers then come
// from hipMalloc.
extern thread_local Arena *tl_arena;

// A grow-only device allocation; new memory is zero-filled. A borrowed
// buffer points into memory the library does not own for this buffer (a
// fixed scratch array): it is never freed, and growing it is an error.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    Arena *arena = nullptr;   // the arena p was taken from, or null (hipMalloc)
    bool borrowed = false;
    void ensure(size_t need, hipStream_t s) {
        if (need <= bytes) return;
        if (borrowed)
            throw Error{DCRF_ENOMEM, "a borrowed buffer is too small (" +
                                         std::to_string(need) + " bytes needed)"};
        release_with(s);
        size_t n = need < 256 ? 256 : need;
        if (tl_arena) {
            p = tl_arena->alloc(n);
            arena = tl_arena;
        } else {
            DCRF_TRY_HIP(hipMalloc(&p, n));
        }
        DCRF_TRY_HIP(hipMemsetAsync(p, 0, n, s));
        bytes = n;
    }
    void release_with(hipStream_t s) {
        if (!p) return;
        if (!borrowed) {
            if (arena) {
                arena->free(p);
            } else {
                DCRF_TRY_HIP(hipStreamSynchronize(s));
                DCRF_TRY_HIP(hipFree(p));
            }
        }
        p = nullptr;
        arena = nullptr;
        bytes = 0;
        borrowed = false;
    }
    void release() {
        if (p && !borrowed) {
            if (arena)
                arena->free(p);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        arena = nullptr;
        bytes = 0;
        borrowed = false;
    }
    template <typename X> X *as() const { return static_cast<X *>(p); }
};

// One permutohedral lattice on the device.
struct Lattice {
    int d = 0;           // feature dimension
    int M = 0;           // number of vertices
    size_t cap = 0;      // hash slots (power of two)
    double gamma = 0;    // slice calibration (4 pi / 3)^{d/2} sqrt(d+1)
    DevBuf hkeys;        // cap x u64 packed vertex keys (~0 = empty)
    DevBuf slot_vid;     // cap x i32 vertex id of each occupied slot
    DevBuf pix_slot;     // N (d+1) x u32 hash slot of each pixel vertex
    DevBuf pix_vid;      // N (d+1) x i32 vertex id, -1 where the weight is 0
    DevBuf pix_w;        // N (d+1) x T barycentric weight
    DevBuf vkeys;        // M x u64
    DevBuf nbr;          // (d+1) x M x 2 i32: id of v + u_j, v - u_j, or -1
    DevBuf V[3];         // M x ld x T: splat target (kept zero), ping, pong
    DevBuf feat;         // N x d x T features (exact mode)
    // inverse index: the (pixel, weight) pairs of vertex v are entries
    // [csr_off[v], csr_off[v+1]); chunks of at most `chunk` entries
    DevBuf csr_off;      // M + 1 i32
    DevBuf csr_tmp;      // M + 1 i32 (counts / cursors while building)
    DevBuf ent_pix;      // N (d+1) i32 pixel of each entry
    DevBuf ent_w;        // N (d+1) x T weight of each entry
    DevBuf ent_v;        // N (d+1) i32 vertex of each entry
    int nent = 0;        // number of entries (pixel vertices with weight > 0)
    DevBuf chunk_off;    // M + 1 i32 chunk counts scanned (build only)
    DevBuf chunks;       // nchunks x int4 (vertex, begin, end, 0), ordered by first pixel
    int nchunks = 0;
    int chunk = 32;
    DevBuf dchunks;      // the same with at most dchunk entries (dense splat)
    int ndchunks = 0;
    int dchunk = 32;
    DevBuf dpix, dw;     // the dense chunks' entries, chunk c at [c dchunk, +dchunk)
                         // (pixel, weight; padded with pixel 0, weight 0)
    // grouped blur: for blur directions taken G at a time, per group and
    // vertex the 3^G vertices reached by the paths of the group (-1 where a
    // path leaves the lattice); [0] forward order, [1] the transpose's order
    DevBuf gtab[2];
    int gtab_G[2] = {0, 0};
    // per-tile vertex slots (tiles.hip)
    DevBuf ts_off;       // ntiles + 1 i32: slots of each pixel tile
    DevBuf ts_vid;       // nslots i32: vertex of each slot
    DevBuf tr_slot;      // N (d+1) u16: slot of each pixel-vertex pair in its tile
    DevBuf sr_off;       // nslots + 1 i32: pairs of each slot
    DevBuf sr_pix;       // nent u8: tile-local pixel of each pair, by slot
    DevBuf sr_w;         // nent x T: weight of each pair, by slot
    DevBuf sr_slot;      // nent u16: slot of each pair (counted from its tile's first)
    DevBuf vs_off;       // M + 1 i32: slots of each vertex
    DevBuf vs_slot;      // nslots i32
    int nslots = 0, max_tile_slots = 0;
    std::vector<int> tile_slots;
    void release() {
        for (DevBuf *b : {&hkeys, &slot_vid, &pix_slot, &pix_vid, &pix_w,
                          &vkeys, &nbr, &V[0], &V[1], &V[2], &feat, &csr_off,
                          &csr_tmp, &ent_pix, &ent_w, &ent_v, &chunk_off, &chunks, &dchunks,
                          &dpix, &dw,
                          &gtab[0], &gtab[1], &ts_off, &ts_vid, &tr_slot, &sr_off,
                          &sr_pix, &sr_w, &sr_slot, &vs_off, &vs_slot})
            b->release();
        nslots = max_tile_slots = 0;
        tile_slots.clear();
        gtab_G[0] = gtab_G[1] = 0;
    }
};

// Row stride of the M x C vertex arrays: C rounded up to 16 bytes so that a
// row can be moved with 16-byte loads; the padding channels stay zero.
inline int row_stride(int C, size_t elt) {
    const int q = int(16 / elt);
    return (C + q - 1) / q * q;
}

// Per-kernel timing with HIP events recorded on the context's stream around
// each launch (enabled only for benchmarks; the events add a small gap).
enum ProfClass {
    PROF_FW_LMO = 0,      // k_fw_lmo_rows: update, gradient, LMO, partial sums
    PROF_BLUR = 1,        // one blur launch over every lattice (k_blur_group,
                          // or k_blur_pass for one direction per launch)
    PROF_FW_SLICE = 2,    // k_fw_slice_rows: slice, mu, diagonal, partial sums
    PROF_SPLAT = 3,       // dense splat (k_splat_gather_lds or k_splat_gather)
    PROF_SLICE = 4,       // raw slice K'Y (k_slice_rows)
    PROF_SLICE_QP = 5,    // slice with mu and the diagonal
    PROF_SPLAT_LABELS = 6,  // one-hot splat (k_splat_labels_chunks)
    PROF_FW_FINAL = 7,    // k_fw_final: the last step size and update of a solve
    PROF_DCNEG = 8,       // k_dcneg_rows: slice and per-pixel step of DC_neg
    PROF_NCLASS = 9
};

struct Profiler {
    bool on = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[PROF_NCLASS] = {};
    long launches[PROF_NCLASS] = {};
    hipEvent_t get() {
        if (pool.empty()) {
            hipEvent_t e;
            DCRF_TRY_HIP(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    void collect() {
        for (auto &p : pending) {
            DCRF_TRY_HIP(hipEventSynchronize(p.second.second));
            float ms = 0;
            DCRF_TRY_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
            total_ms[p.first] += ms;
            launches[p.first] += 1;
            pool.push_back(p.second.first);
            pool.push_back(p.second.second);
        }
        pending.clear();
    }
    void reset() {
        pending.clear();
        for (int i = 0; i < PROF_NCLASS; ++i) total_ms[i] = 0, launches[i] = 0;
    }
    void release() {
        for (auto &p : pending) pool.push_back(p.second.first), pool.push_back(p.second.second);
        pending.clear();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

}  // namespace dcrf

struct dcrf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int H = 0, W = 0, N = 0, nk = 0, dtype = DCRF_F32;
    // Images held by the context: image j owns pixel rows
    // [seg[2j], seg[2j+1]); a single image is the segment [0, N). Rows
    // between segments (alignment padding of a batch) belong to no image.
    int nimg = 1;
    std::vector<int> seg_h;
    std::vector<int> img_H, img_W;
    dcrf::DevBuf seg;
    // launch-shape parameters chosen by dcrf_autotune
    int blur_vpt = 1;        // 16-byte vectors per thread in the blur
    int blur_block = 256;    // threads per block in the blur
    int blur_group = 2;      // blur directions applied per launch (1..3)
    int tile_mode = 0;       // splats and slices through the per-tile slots
    int fw_splat = 0;        // Frank-Wolfe: one-hot splat inside the LMO kernel
    int fw_persistent = 0;   // Frank-Wolfe: every iteration in one cooperative launch
    dcrf::DevBuf fw_bar;     // its grid barrier (count, generation) and timeout flag
    // 2-D pixel tiles of every image (tiles.hip)
    int ntiles = 0;          // 0 until the tile map is built (only when tiles are asked for)
    dcrf::DevBuf tiles;              // ntiles x int4: first row, row stride, rows, cols
    dcrf::DevBuf tile_img_off;       // nimg + 1 i32: first tile of each image
    std::vector<int> tile_img_off_h;
    int mode = DCRF_FILTER_LATTICE;
    bool has_image = false;
    dcrf_kernel kern[DCRF_MAXK];
    dcrf::Lattice lat[DCRF_MAXK];
    double wsum = 0;
    int splat_chunk = 64;    // entries per chunk of the one-hot splat (one wave)
    int dense_chunk = 32;    // entries per chunk of the dense splat
    int splat_lds = 1;       // dense splat: stage each block's pairs in LDS
    dcrf::DevBuf r;          // N x T: K'1
    dcrf::DevBuf scratch;    // small device scratch (flags, counters)
    dcrf::DevBuf tmpA, tmpB; // N x C scratch arrays
    dcrf::DevBuf sep_taps, sep_tmp, sep_acc, sep_part;   // the separable filter mode
    dcrf::DevBuf pack_a, pack_b, pack_c;   // packed copies for the per-image batch calls
    // Frank-Wolfe state
    dcrf::DevBuf fw_c, fw_Py, fw_Ps, fw_s, fw_sprev, fw_part, fw_scal,
        fw_trace, fw_mu;
    // the Potts compatibility [i != j] (L x L, context dtype) that stands in
    // for a null mu argument; the solvers recognise it by its address and
    // never read it back to the host
    dcrf::DevBuf potts;
    int potts_L = 0, potts_dtype = -1;
    dcrf::DevBuf hist;       // per-step partial sums of a solver's history
    dcrf::DevBuf small;      // 4 KB of per-call flags, counters and index tables
    dcrf::DevBuf sub_phi, sub_y, sub_best;   // the LP on a label subset
    dcrf::DevBuf errflag;    // device-detected input errors (non-finite values)
    dcrf::Arena arena;       // the caller's workspace, when one is given
    size_t hash_cap = 0;     // forced hash-table slots per lattice (0: sized by N)
    int lp_leaf = 0;         // LP divide and conquer: exact pairs in nodes of <= this many
    void *lp = nullptr;      // LP divide-and-conquer workspace (lp.hip)
    void *diff = nullptr;    // reverse-sweep workspace (diff.hip)
    dcrf::Profiler prof;
    std::string err;
    size_t elt() const { return dtype == DCRF_F64 ? 8 : 4; }
};

namespace dcrf {

// name of the kernel that profiling class c launches under ctx's launch shapes
const char *prof_name(const dcrf_ctx *ctx, int c);

// ------------------------------------------------------------ launchers

// lattice.hip
void build_lattices(dcrf_ctx *ctx, const float *rgb);
void lattice_export(dcrf_ctx *ctx, int m, int32_t *keys, int32_t *vid,
                    double *w);
// cut every lattice's inverse index into chunks of at most `chunk` entries
// (one-hot splat) and of `dense_chunk` entries (dense splat)
void rechunk(dcrf_ctx *ctx, int chunk, int dense_chunk);

// filter.hip
// out = K' in (N x C), lattice or exact, optionally the transpose
// separable.hip: K'Y with the position-only kernels exact (two 1-D passes)
// and the others by the lattice
void filter_separable(dcrf_ctx *ctx, const void *in, void *out, int C, bool adjoint);
// kind: DCRF_FILTER_LATTICE, DCRF_FILTER_EXACT or DCRF_FILTER_SEPARABLE
void filter_apply(dcrf_ctx *ctx, const void *in, void *out, int C,
                  bool adjoint, int kind);
// r = K'1
void compute_row_sums(dcrf_ctx *ctx);
// make sure every lattice has vertex buffers for C channels
void ensure_vertex_buffers(dcrf_ctx *ctx, int C);
// the grouped blur's path tables for G directions per launch (forward order)
void blur_group_tables(dcrf_ctx *ctx, int G);
// splat of one-hot labels (C = L channels), blur; leaves results in the final
// buffers of each lattice
void splat_labels(dcrf_ctx *ctx, const int32_t *labels, int L);
void splat_dense(dcrf_ctx *ctx, const void *in, int C);
void blur_all(dcrf_ctx *ctx, int C, bool adjoint);
// slice of the blurred lattices: K'Y (qp = false) or (K'Y) mu^T + d * Y
// (qp = true); `pre` replaces the lattice by a given K'Y (exact mode)
void slice_into(dcrf_ctx *ctx, const void *Y, const void *pre, int C,
                const void *mu, const void *mabs, void *out, bool qp);
// index of the buffer that holds the blurred values of a lattice whose blur
// took n launches (the first reads V[0] and writes V[1], then V[1] and V[2]
// alternate)
inline int final_buffer_after(int n) { return (n % 2 == 1) ? 1 : 2; }
// launches of the blur of a d-dimensional lattice, G directions per launch
inline int blur_launches(int d, int G) { return (d + 1 + G - 1) / G; }
// one pass per launch
inline int final_buffer(int d) { return final_buffer_after(d + 1); }

// solvers.hip
// flag (on the device, checked later) any non-finite value among the
// images' rows of x (N x L)
void check_finite(dcrf_ctx *ctx, const void *x, int L);
// wait for the stream; DCRF_EINVAL if a check_finite flag was raised since
// the last call of this (the flag is then cleared)
void raise_device_errors(dcrf_ctx *ctx);
// hash slots of a lattice with n pixel-vertex pairs: a power of two of at
// least 2n (and 1024), or the context's forced capacity
inline size_t hash_slots(const dcrf_ctx *ctx, size_t n) {
    if (ctx->hash_cap) return ctx->hash_cap;
    size_t cap = 1024;
    while (cap < 2 * n) cap <<= 1;
    return cap;
}
// mu itself, or for a null mu the context's device copy of the Potts
// compatibility of L labels (built on first use for each L and dtype)
const void *resolve_mu(dcrf_ctx *ctx, const void *mu, int L);
// whether mu is the context's Potts copy (no host read)
inline bool is_internal_potts(const dcrf_ctx *ctx, const void *mu) {
    return mu != nullptr && mu == ctx->potts.p;
}
void qp_apply(dcrf_ctx *ctx, const void *y, const void *mu, int L, void *out);
void frank_wolfe(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                 void *y, int iters, dcrf_iter_trace *trace, const void *c_in,
                 bool have_Py);
void dc_gen(dcrf_ctx *ctx, const void *unary, const void *mu, int L, void *y,
            int outer, int inner, double *S_hist);
// noalloc.hip: the size of the allocation-free scratch array, and the solve
// on it (its device address taken once per device)
size_t noalloc_scratch_bytes();
void frank_wolfe_noalloc_entry(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                               void *y, int iters, dcrf_iter_trace *trace);
// Frank-Wolfe with the solve's buffers borrowed from base (cap bytes)
void frank_wolfe_noalloc(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                         void *y, int iters, dcrf_iter_trace *trace, void *base,
                         size_t cap);
void round_labels(dcrf_ctx *ctx, const void *y, int L, int32_t *labels);
double energy(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
              const int32_t *labels);

// rounding.hip: Kleinberg-Tardos rounding (returns the pixels left to the
// argmax), the labels present in y, the LP restricted to a label subset
int round_kt(dcrf_ctx *ctx, const void *y, int L, const int32_t *rlab, const void *rth,
             int R, int32_t *labels);
int present_labels(dcrf_ctx *ctx, const void *y, int L, double tau, int32_t *out);
int labels_used(dcrf_ctx *ctx, const int32_t *labels, int L, int32_t *out);
void lp_descent_subset(dcrf_ctx *ctx, const void *unary, int L, void *y,
                       const int32_t *subset, int S, int steps, double beta0,
                       double *best, void *best_y, double *hist);

// workspace.cpp: upper bound of a context's device memory for B images
size_t workspace_bound(int B, const int *H, const int *W, int L,
                       const dcrf_kernel *k, int nk, int dtype);

// dcneg.hip: CCCP on the negative semi-definite decomposition
void dc_neg(dcrf_ctx *ctx, const void *unary, const void *mu, int L, void *y,
            int outer, int inner, double *S_hist);

// Checkpoints of a Frank-Wolfe forward for the reverse sweep: y_t and
// P_t = (Psi + D) y_t (iters x N x L each), s_t (iters x N labels), per
// lattice the blurred vertex values of y_0 and of the one-hot s_t
// ((iters + 1) blocks of sum_m M_m x ld values, block 0 for y_0, block t+1
// for s_t), and per iteration and image kFWStats doubles
// (alpha, a2, b1, interior).
constexpr int kFWStats = 4;
struct FWCheckpoint {
    void *y;
    void *P;
    int32_t *s;
    void *V;
    double *stats;
};
void frank_wolfe_checkpointed(dcrf_ctx *ctx, const void *unary, const void *mu,
                              int L, void *y, int iters, const FWCheckpoint &save);

// diff.hip
void fw_diff_forward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                     void *y_out, int iters, void *saved);
void fw_diff_backward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                      int iters, const void *saved, const void *grad_y,
                      void *grad_unary, double *grad_w);
size_t fw_saved_bytes(dcrf_ctx *ctx, int L, int iters);
void diff_release(dcrf_ctx *ctx);
// K~_m X: the lattice approximation of kernel m alone (weight 1, with its
// own response at a), or its transpose
void filter_kernel(dcrf_ctx *ctx, int m, const void *in, void *out, int C,
                   bool adjoint);
// sum over b != a of k_m(a, b) in_b, exactly, for kernel m alone (weight 1)
void exact_kernel(dcrf_ctx *ctx, int m, const void *in, void *out, int C);
// dcrf_filter's variants: keep_self adds (sum w) in back (K-bar Y);
// per_kernel writes nk blocks of N x C, block m = w_m K_m in without (or,
// with keep_self, with) its self term, for the filter kind given
void filter_parts(dcrf_ctx *ctx, const void *in, void *out, int C, bool adjoint,
                  int kind, bool keep_self, bool per_kernel);

// lp.hip
double lp_subgradient(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                      void *g);
void lp_descent(dcrf_ctx *ctx, const void *unary, int L, void *y, int steps,
                double beta0, double *best, void *best_y, double *hist);
void project_simplex(dcrf_ctx *ctx, const void *v, int L, void *y);
void lp_release(dcrf_ctx *ctx);
// the LP for an r-HST metric: the tree's subtrees with their weights c_T and
// label lists (increasing label order), checked and built from parent[]
constexpr int kMaxTreeNodes = 1024;
struct TreeSpec {
    int n = 0;
    std::vector<double> c;
    std::vector<int> off, lab;   // labels of subtree t: lab[off[t] .. off[t+1])
};
TreeSpec tree_spec(const int32_t *parent, const double *c, int n, int L);
double lp_subgradient_tree(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                           const TreeSpec &tr, void *g);
void lp_descent_tree(dcrf_ctx *ctx, const void *unary, int L, void *y, const TreeSpec &tr,
                     int steps, double beta0, double *best, void *best_y, double *hist);

inline int ceil_div(long long a, long long b) { return int((a + b - 1) / b); }

// 2-D pixel tiles (tiles.hip)
constexpr int kTileH = 16, kTileW = 16, kTilePix = kTileH * kTileW;
// largest d + 1 of a lattice served by the tile kernels (pairs of one tile
// and lattice: at most kTilePix * (d + 1))
constexpr int kMaxD1 = 6;
void build_tiles(dcrf_ctx *ctx);
// the tile map of the current image(s), built on first use
void ensure_tiles(dcrf_ctx *ctx);

// Segments of the pixel range (see dcrf_ctx): set on the host and uploaded.
void set_segments(dcrf_ctx *ctx, const std::vector<int> &seg);
// Number of tiles of TP pixels over all images (no tile straddles two).
// (node, vertex) numbers available to the LP's densely numbered levels, for
// a lattice with E = N (d + 1) entries: four times the entries (at 500x375
// with L = 21 a plain LP step takes 93.5, 91.3 and 89.3 ms with one, two and
// four times; the tables of a 5-D lattice then hold 24 E ints of links)
constexpr size_t kLpDenseFactor = 4;
inline size_t lp_dense_cap(size_t E) {
    return std::min<size_t>(kLpDenseFactor * E, size_t(INT32_MAX));
}

inline int seg_tiles(const dcrf_ctx *ctx, int TP) {
    long long n = 0;
    for (int j = 0; j < ctx->nimg; ++j)
        n += ceil_div(ctx->seg_h[2 * j + 1] - ctx->seg_h[2 * j], TP);
    return int(n);
}
// First tile of each image (nimg + 1 entries) for tiles of TP pixels.
inline std::vector<int> seg_tile_offsets(const dcrf_ctx *ctx, int TP) {
    std::vector<int> o(ctx->nimg + 1, 0);
    for (int j = 0; j < ctx->nimg; ++j)
        o[j + 1] = o[j] + ceil_div(ctx->seg_h[2 * j + 1] - ctx->seg_h[2 * j], TP);
    return o;
}

// batch.hip: the lattices of several images, concatenated (vertex ids,
// neighbour ids and inverse-index entries renumbered), so that every filter
// launch covers the whole batch; sets the segments.
void build_batch(dcrf_ctx *ctx, int B, const int *H, const int *W,
                 const float *const *rgb);
void autotune(dcrf_ctx *ctx, int L, int reps, double *best_ms);

// Records events around the launches made during its lifetime when the
// context's profiler is on.
// Timing of one kernel class while profiling is on: the launches of the scope
// go through DCRF_PLAUNCH, which hands the scope's events to the dispatch
// itself (hipExtLaunchKernelGGL), so the interval is that of the kernels and
// no event packets are inserted between launches. The first launch of the
// scope records the start, every launch the stop (the last one counts).
struct ProfScope {
    dcrf_ctx *ctx;
    int cls;
    hipEvent_t start{}, stop{};
    bool started = false;
    ProfScope(dcrf_ctx *c, int k) : ctx(c), cls(k) {
        if (ctx->prof.on) {
            start = ctx->prof.get();
            stop = ctx->prof.get();
        }
    }
    bool on() const { return ctx->prof.on; }
    hipEvent_t first() {
        if (started) return nullptr;
        started = true;
        return start;
    }
    ~ProfScope() {
        if (!ctx->prof.on) return;
        if (started) {
            ctx->prof.pending.push_back({cls, {start, stop}});
        } else {
            ctx->prof.pool.push_back(start);
            ctx->prof.pool.push_back(stop);
        }
    }
};

#define DCRF_PLAUNCH(ps, kernel, grid, block, shmem, stream, ...)                   \
    do {                                                                           \
        if ((ps).on())                                                             \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, (ps).first(), \
                                  (ps).stop, 0, __VA_ARGS__);                      \
        else                                                                       \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);   \
    } while (0)

}  // namespace dcrf
