// C ABI of the library (declared in include/dcrf.h): argument checks, error
// capture and dispatch to the launchers. No call throws or aborts; failures
// return a status and leave a message in the context.

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dcrf_internal.h"

using dcrf::Error;

namespace dcrf {
thread_local Arena *tl_arena = nullptr;

// name of the kernel that class c launches under the context's launch shapes
const char *prof_name(const dcrf_ctx *ctx, int c) {
    const bool tiles = ctx->tile_mode != 0, staged = ctx->splat_lds != 0;
    switch (c) {
    case PROF_FW_LMO: return "k_fw_lmo_rows";
    case PROF_BLUR: return ctx->blur_group > 1 ? "k_blur_group" : "k_blur_pass";
    case PROF_FW_SLICE: return tiles ? "k_tile_slice" : "k_fw_slice_rows";
    case PROF_SPLAT:
        return tiles ? "k_tile_splat" : staged ? "k_splat_gather_lds" : "k_splat_gather";
    case PROF_SLICE: return tiles ? "k_tile_slice" : "k_slice_rows";
    case PROF_SLICE_QP: return tiles ? "k_tile_slice_qp" : "k_slice_rows_qp";
    case PROF_SPLAT_LABELS:
        return tiles ? "k_tile_labels" : staged ? "k_splat_labels_lds" : "k_splat_labels_chunks";
    case PROF_FW_FINAL: return "k_fw_final";
    case PROF_DCNEG: return "k_dcneg_rows";
    default: return "?";
    }
}
}  // namespace dcrf

namespace {

thread_local std::string g_create_error;

int set_err(dcrf_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

// the context's workspace (when it has one) serves every allocation made
// during a call
struct ArenaScope {
    dcrf::Arena *prev;
    explicit ArenaScope(dcrf_ctx *ctx) : prev(dcrf::tl_arena) {
        ctx->arena.stream = ctx->stream;
        dcrf::tl_arena = ctx->arena.active() ? &ctx->arena : nullptr;
    }
    ~ArenaScope() { dcrf::tl_arena = prev; }
};

template <typename F>
int guarded(dcrf_ctx *ctx, F &&f) {
    if (!ctx) return DCRF_EINVAL;
    try {
        DCRF_TRY_HIP(hipSetDevice(ctx->device));
        ArenaScope scope(ctx);
        f();
        ctx->err.clear();
        return DCRF_OK;
    } catch (const Error &e) {
        return set_err(ctx, e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(ctx, DCRF_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, DCRF_EHIP, "unexpected exception");
    }
}

#define REQUIRE(cond, msg)                                        \
    do {                                                          \
        if (!(cond)) dcrf::fail(DCRF_EINVAL, std::string(msg));   \
    } while (0)

void require_image(dcrf_ctx *ctx) {
    if (!ctx->has_image)
        dcrf::fail(DCRF_ESTATE, "no image set: call dcrf_set_image first");
}

void require_single(dcrf_ctx *ctx) {
    if (ctx->nimg > 1)
        dcrf::fail(DCRF_EUNSUPPORTED, "the LP relaxation of a batch is not built");
}

void check_labels(int L) {
    REQUIRE(L >= 1 && L <= 256, "L must be in [1, 256]");
}

// the LP's pair sums are built for the lattice and exact filter modes only
void require_lp_mode(dcrf_ctx *ctx) {
    if (ctx->mode == DCRF_FILTER_SEPARABLE)
        throw Error{DCRF_EUNSUPPORTED,
                    "the LP needs the lattice or the exact filter mode"};
}

}  // namespace

extern "C" {

const char *dcrf_version(void) { return "dcrf 0.1 (gfx950)"; }

int dcrf_create(dcrf_ctx **out, int device, void *hip_stream) {
    if (!out) return DCRF_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        g_create_error = "no such HIP device";
        return DCRF_EINVAL;
    }
    dcrf_ctx *ctx = new (std::nothrow) dcrf_ctx();
    if (!ctx) return DCRF_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    *out = ctx;
    return DCRF_OK;
}

// every device buffer of the context, back to hipFree or to its workspace
static void release_all(dcrf_ctx *ctx) {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &L : ctx->lat) L.release();
    dcrf::lp_release(ctx);
    dcrf::diff_release(ctx);
    for (dcrf::DevBuf *b :
         {&ctx->r, &ctx->scratch, &ctx->tmpA, &ctx->tmpB, &ctx->fw_c,
          &ctx->fw_Py, &ctx->fw_Ps, &ctx->fw_s, &ctx->fw_sprev, &ctx->fw_part,
          &ctx->fw_scal, &ctx->fw_trace, &ctx->fw_mu, &ctx->potts, &ctx->hist,
          &ctx->errflag, &ctx->fw_bar, &ctx->seg, &ctx->tiles, &ctx->tile_img_off, &ctx->small,
          &ctx->sub_phi, &ctx->sub_y, &ctx->sub_best, &ctx->sep_taps, &ctx->sep_tmp,
          &ctx->sep_acc, &ctx->sep_part, &ctx->pack_a, &ctx->pack_b, &ctx->pack_c})
        b->release();
    ctx->potts_L = 0;
    ctx->potts_dtype = -1;
    ctx->ntiles = 0;
    ctx->has_image = false;
}

int dcrf_destroy(dcrf_ctx *ctx) {
    if (!ctx) return DCRF_EINVAL;
    (void)hipSetDevice(ctx->device);
    release_all(ctx);
    ctx->prof.release();
    delete ctx;
    return DCRF_OK;
}

const char *dcrf_last_error(const dcrf_ctx *ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int dcrf_set_stream(dcrf_ctx *ctx, void *hip_stream) {
    return guarded(ctx, [&] { ctx->stream = static_cast<hipStream_t>(hip_stream); });
}

static void set_kernels(dcrf_ctx *ctx, const dcrf_kernel *kernels, int nk,
                        int dtype) {
    REQUIRE(kernels != nullptr && nk >= 1 && nk <= DCRF_MAXK,
            "need 1 to 4 kernels");
    REQUIRE(dtype == DCRF_F32 || dtype == DCRF_F64, "dtype must be F32 or F64");
    for (int m = 0; m < nk; ++m) {
        const dcrf_kernel &k = kernels[m];
        REQUIRE(std::isfinite(k.theta_pos) && k.theta_pos > 0,
                "theta_pos must be > 0");
        REQUIRE(!k.use_rgb || (std::isfinite(k.theta_rgb) && k.theta_rgb > 0),
                "theta_rgb must be > 0 for a colour kernel");
        REQUIRE(std::isfinite(k.weight) && k.weight >= 0,
                "weights must be finite and >= 0");
    }
    ctx->has_image = false;
    ctx->nk = nk;
    ctx->dtype = dtype;
    ctx->wsum = 0;
    for (int m = 0; m < nk; ++m) {
        ctx->kern[m] = kernels[m];
        ctx->kern[m].use_rgb = kernels[m].use_rgb ? 1 : 0;
        ctx->wsum += kernels[m].weight;
    }
}

// Attach the caller's workspace (or none) before an image is built. Buffers
// move only when a workspace is involved on either side; without one the
// context keeps its grow-only allocations from image to image.
static void attach_workspace(dcrf_ctx *ctx, void *ws, size_t bytes) {
    REQUIRE(ws == nullptr || bytes >= 4096, "workspace smaller than 4096 bytes");
    REQUIRE(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
    if (ws || ctx->arena.active()) {
        release_all(ctx);
        ctx->arena.reset(ws, ws ? bytes : 0);
    }
    ctx->arena.stream = ctx->stream;
    dcrf::tl_arena = ctx->arena.active() ? &ctx->arena : nullptr;
}

int dcrf_set_image(dcrf_ctx *ctx, int H, int W, const float *rgb,
                   const dcrf_kernel *kernels, int nk, int dtype, void *workspace,
                   size_t ws_bytes) {
    return guarded(ctx, [&] {
        REQUIRE(H >= 1 && W >= 1 && (long long)H * W <= (1ll << 28),
                "H and W must be >= 1 with H*W <= 2^28");
        REQUIRE(rgb != nullptr, "rgb is null");
        set_kernels(ctx, kernels, nk, dtype);
        attach_workspace(ctx, workspace, ws_bytes);
        ctx->H = H;
        ctx->W = W;
        ctx->N = H * W;
        ctx->img_H.assign(1, H);
        ctx->img_W.assign(1, W);
        dcrf::build_lattices(ctx, rgb);
        dcrf::set_segments(ctx, {0, ctx->N});
        ctx->ntiles = 0;   // the tile map is built when tiles are asked for
        if (ctx->tile_mode) dcrf::build_tiles(ctx);
        ctx->has_image = true;
        dcrf::compute_row_sums(ctx);
    });
}

int dcrf_set_images(dcrf_ctx *ctx, int B, const int *H, const int *W,
                    const float *const *rgb, const dcrf_kernel *kernels, int nk,
                    int dtype, void *workspace, size_t ws_bytes) {
    return guarded(ctx, [&] {
        REQUIRE(B >= 1 && B <= 4096, "B must be in [1, 4096]");
        REQUIRE(H && W && rgb, "null argument");
        for (int j = 0; j < B; ++j) {
            REQUIRE(H[j] >= 1 && W[j] >= 1 && (long long)H[j] * W[j] <= (1ll << 28),
                    "every H and W must be >= 1 with H*W <= 2^28");
            REQUIRE(rgb[j] != nullptr, "rgb pointer is null");
        }
        set_kernels(ctx, kernels, nk, dtype);
        attach_workspace(ctx, workspace, ws_bytes);
        if (ctx->mode != DCRF_FILTER_LATTICE && B > 1)
            throw Error{DCRF_EUNSUPPORTED, "a batch needs the lattice filter mode"};
        if (B == 1) {
            ctx->H = H[0];
            ctx->W = W[0];
            ctx->N = H[0] * W[0];
            ctx->img_H.assign(1, H[0]);
            ctx->img_W.assign(1, W[0]);
            dcrf::build_lattices(ctx, rgb[0]);
            dcrf::set_segments(ctx, {0, ctx->N});
        } else {
            dcrf::build_batch(ctx, B, H, W, rgb);
        }
        ctx->ntiles = 0;   // the tile map is built when tiles are asked for
        if (ctx->tile_mode) dcrf::build_tiles(ctx);
        ctx->has_image = true;
        dcrf::compute_row_sums(ctx);
    });
}

int dcrf_batch_set_images(dcrf_ctx *ctx, int B, const int *H, const int *W,
                          const float *const *rgb, const dcrf_kernel *kernels, int nk,
                          int dtype, void *workspace, size_t ws_bytes) {
    return dcrf_set_images(ctx, B, H, W, rgb, kernels, nk, dtype, workspace, ws_bytes);
}

int dcrf_image_layout(dcrf_ctx *ctx, int *nimg, int *rows, int *seg) {
    return guarded(ctx, [&] {
        require_image(ctx);
        if (nimg) *nimg = ctx->nimg;
        if (rows) *rows = ctx->N;
        if (seg)
            for (size_t i = 0; i < ctx->seg_h.size(); ++i) seg[i] = ctx->seg_h[i];
    });
}

int dcrf_autotune(dcrf_ctx *ctx, int L, int reps, dcrf_tune *out) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
        if (ctx->mode != DCRF_FILTER_LATTICE)
            throw Error{DCRF_EUNSUPPORTED, "autotuning needs the lattice filter mode"};
        double ms = 0;
        dcrf::autotune(ctx, L, reps, &ms);
        if (out) {
            out->splat_chunk = ctx->splat_chunk;
            out->dense_chunk = ctx->dense_chunk;
            out->splat_stage = ctx->splat_lds;
            out->blur_vectors_per_thread = ctx->blur_vpt;
            out->blur_block = ctx->blur_block;
            out->blur_group = ctx->blur_group;
            out->tiles = ctx->tile_mode;
            out->fw_splat = ctx->fw_splat;
            out->fw_persistent = ctx->fw_persistent;
            out->ms = ms;
        }
    });
}

int dcrf_set_tune(dcrf_ctx *ctx, const dcrf_tune *t) {
    return guarded(ctx, [&] {
        require_image(ctx);
        REQUIRE(t != nullptr, "null argument");
        auto chunk_ok = [](int c) { return c == 16 || c == 32 || c == 64 || c == 128 || c == 256; };
        REQUIRE(chunk_ok(t->splat_chunk) && chunk_ok(t->dense_chunk),
                "splat_chunk and dense_chunk must be 16, 32, 64, 128 or 256");
        REQUIRE(!ctx->arena.active() || t->dense_chunk <= 64,
                "with a caller workspace dense_chunk must be at most 64");
        REQUIRE(t->blur_vectors_per_thread >= 1 && t->blur_vectors_per_thread <= 4,
                "blur_vectors_per_thread must be in 1..4");
        REQUIRE(t->blur_block == 64 || t->blur_block == 128 || t->blur_block == 256,
                "blur_block must be 64, 128 or 256");
        REQUIRE(t->blur_group >= 1 && t->blur_group <= 3, "blur_group must be in 1..3");
        REQUIRE(t->tiles == 0 || t->tiles == 1, "tiles must be 0 or 1");
        REQUIRE(t->splat_stage == 0 || t->splat_stage == 1, "splat_stage must be 0 or 1");
        REQUIRE(t->fw_splat == 0 || t->fw_splat == 1, "fw_splat must be 0 or 1");
        REQUIRE(t->fw_persistent == 0 || t->fw_persistent == 1, "fw_persistent must be 0 or 1");
        if (t->splat_chunk != ctx->splat_chunk || t->dense_chunk != ctx->dense_chunk)
            dcrf::rechunk(ctx, t->splat_chunk, t->dense_chunk);
        ctx->splat_lds = t->splat_stage;
        ctx->blur_vpt = t->blur_vectors_per_thread;
        ctx->blur_block = t->blur_block;
        ctx->blur_group = t->blur_group;
        ctx->tile_mode = t->tiles;
        ctx->fw_splat = t->fw_splat;
        ctx->fw_persistent = t->fw_persistent;
        if (t->tiles && ctx->has_image) dcrf::ensure_tiles(ctx);
    });
}

// replace the kernel weights and recompute r = K'1 (one filter call); the
// lattices do not depend on the weights
static void apply_weights(dcrf_ctx *ctx, const double *w) {
    double s = 0;
    for (int m = 0; m < ctx->nk; ++m) {
        REQUIRE(std::isfinite(w[m]) && w[m] >= 0, "weights must be >= 0");
        s += w[m];
    }
    bool same = true;
    for (int m = 0; m < ctx->nk; ++m) same = same && ctx->kern[m].weight == w[m];
    if (same) return;
    for (int m = 0; m < ctx->nk; ++m) ctx->kern[m].weight = w[m];
    ctx->wsum = s;
    dcrf::compute_row_sums(ctx);
}

int dcrf_set_weights(dcrf_ctx *ctx, const double *w, int nk) {
    return guarded(ctx, [&] {
        require_image(ctx);
        REQUIRE(w != nullptr && nk == ctx->nk, "need one weight per kernel");
        apply_weights(ctx, w);
    });
}

int dcrf_set_filter_mode(dcrf_ctx *ctx, int mode) {
    return guarded(ctx, [&] {
        REQUIRE(mode == DCRF_FILTER_LATTICE || mode == DCRF_FILTER_EXACT ||
                    mode == DCRF_FILTER_SEPARABLE,
                "mode must be DCRF_FILTER_LATTICE, DCRF_FILTER_EXACT or "
                "DCRF_FILTER_SEPARABLE");
        if (mode != DCRF_FILTER_LATTICE && ctx->has_image && ctx->nimg > 1)
            throw Error{DCRF_EUNSUPPORTED, "a batch needs the lattice filter mode"};
        const bool changed = ctx->mode != mode;
        ctx->mode = mode;
        if (changed && ctx->has_image) dcrf::compute_row_sums(ctx);
    });
}

int dcrf_lattice_info(dcrf_ctx *ctx, int m, int *d, int *nvert) {
    return guarded(ctx, [&] {
        require_image(ctx);
        REQUIRE(m >= 0 && m < ctx->nk, "kernel index out of range");
        if (d) *d = ctx->lat[m].d;
        if (nvert) *nvert = ctx->lat[m].M;
    });
}

int dcrf_lattice_export(dcrf_ctx *ctx, int m, int32_t *keys, int32_t *vid,
                        double *w) {
    return guarded(ctx, [&] {
        require_image(ctx);
        REQUIRE(m >= 0 && m < ctx->nk, "kernel index out of range");
        dcrf::lattice_export(ctx, m, keys, vid, w);
    });
}

int dcrf_filter(dcrf_ctx *ctx, const void *in, void *out, int C,
                unsigned flags) {
    return guarded(ctx, [&] {
        require_image(ctx);
        REQUIRE(in && out && in != out, "in and out must be distinct, non-null");
        REQUIRE(C >= 1 && C <= 256, "C must be in [1, 256]");
        REQUIRE((flags & ~(DCRF_ADJOINT | DCRF_EXACT | DCRF_SEPARABLE | DCRF_KEEP_SELF |
                           DCRF_PER_KERNEL)) == 0,
                "unknown flags");
        REQUIRE(!((flags & DCRF_EXACT) && (flags & DCRF_SEPARABLE)),
                "DCRF_EXACT and DCRF_SEPARABLE exclude each other");
        if ((flags & (DCRF_EXACT | DCRF_SEPARABLE)) && ctx->nimg > 1)
            throw Error{DCRF_EUNSUPPORTED, "the exact and separable filters of a batch are not built"};
        const int kind = (flags & DCRF_EXACT)       ? DCRF_FILTER_EXACT
                         : (flags & DCRF_SEPARABLE) ? DCRF_FILTER_SEPARABLE
                                                    : DCRF_FILTER_LATTICE;
        if (flags & (DCRF_KEEP_SELF | DCRF_PER_KERNEL))
            dcrf::filter_parts(ctx, in, out, C, (flags & DCRF_ADJOINT) != 0, kind,
                               (flags & DCRF_KEEP_SELF) != 0, (flags & DCRF_PER_KERNEL) != 0);
        else
            dcrf::filter_apply(ctx, in, out, C, (flags & DCRF_ADJOINT) != 0, kind);
    });
}

int dcrf_qp_apply(dcrf_ctx *ctx, const void *y, const void *mu, int L,
                  void *out) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(y && out && y != out, "null or aliased argument");
        dcrf::qp_apply(ctx, y, dcrf::resolve_mu(ctx, mu, L), L, out);
    });
}

int dcrf_qp_frank_wolfe(dcrf_ctx *ctx, const void *unary, const void *mu,
                        int L, void *y_inout, int iters,
                        dcrf_iter_trace *trace) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout, "null argument");
        REQUIRE(iters >= 0, "iters must be >= 0");
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y_inout, L);
        dcrf::frank_wolfe(ctx, unary, dcrf::resolve_mu(ctx, mu, L), L, y_inout,
                          iters, trace, nullptr, false);
        if (trace) dcrf::raise_device_errors(ctx);
    });
}

int dcrf_qp_frank_wolfe_noalloc(dcrf_ctx *ctx, const void *unary, const void *mu,
                                int L, void *y_inout, int iters,
                                dcrf_iter_trace *trace) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout, "null argument");
        REQUIRE(iters >= 0, "iters must be >= 0");
        dcrf::frank_wolfe_noalloc_entry(ctx, unary, mu, L, y_inout, iters, trace);
    });
}

int dcrf_noalloc_scratch_bytes(size_t *bytes) {
    if (!bytes) return DCRF_EINVAL;
    *bytes = dcrf::noalloc_scratch_bytes();
    return DCRF_OK;
}

int dcrf_dc_gen(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                void *y_inout, int outer, int inner, double *S_hist) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout, "null argument");
        REQUIRE(outer >= 0 && inner >= 1, "outer >= 0 and inner >= 1 required");
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y_inout, L);
        dcrf::dc_gen(ctx, unary, dcrf::resolve_mu(ctx, mu, L), L, y_inout, outer,
                     inner, S_hist);
        if (S_hist) dcrf::raise_device_errors(ctx);
    });
}

int dcrf_dc_neg(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                void *y_inout, int outer, int inner, double *S_hist) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout, "null argument");
        REQUIRE(outer >= 0 && inner >= 1, "outer >= 0 and inner >= 1 required");
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y_inout, L);
        dcrf::dc_neg(ctx, unary, dcrf::resolve_mu(ctx, mu, L), L, y_inout, outer,
                     inner, S_hist);
        if (S_hist) dcrf::raise_device_errors(ctx);
    });
}

int dcrf_round(dcrf_ctx *ctx, const void *y, int L, int32_t *labels) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(y && labels, "null argument");
        dcrf::round_labels(ctx, y, L, labels);
    });
}

int dcrf_energy(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                const int32_t *labels, double *energy) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && labels && energy, "null argument");
        dcrf::check_finite(ctx, unary, L);
        *energy = dcrf::energy(ctx, unary, dcrf::resolve_mu(ctx, mu, L), L, labels);
        dcrf::raise_device_errors(ctx);
    });
}

int dcrf_lp_subgradient(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                        void *g, double *S_lp) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y && g && y != g, "null or aliased argument");
        require_single(ctx);
        require_lp_mode(ctx);
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y, L);
        const double S = dcrf::lp_subgradient(ctx, unary, L, y, g);
        dcrf::raise_device_errors(ctx);
        if (S_lp) *S_lp = S;
    });
}

static void require_diff(dcrf_ctx *ctx, int L, int iters) {
    require_image(ctx);
    check_labels(L);
    REQUIRE(iters >= 1, "iters must be >= 1");
    if (ctx->mode != DCRF_FILTER_LATTICE)
        throw dcrf::Error{DCRF_EUNSUPPORTED,
                          "differentiation needs the lattice filter mode"};
}

int dcrf_fw_saved_size(dcrf_ctx *ctx, int L, int iters, size_t *bytes) {
    return guarded(ctx, [&] {
        require_diff(ctx, L, iters);
        REQUIRE(bytes, "null argument");
        *bytes = dcrf::fw_saved_bytes(ctx, L, iters);
    });
}

int dcrf_fw_forward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                    const double *w, int iters, void *y_out, void *saved) {
    return guarded(ctx, [&] {
        require_diff(ctx, L, iters);
        REQUIRE(unary && y_out && saved, "null argument");
        REQUIRE(y_out != unary, "y_out must not alias unary");
        REQUIRE(iters <= 4096 || !ctx->arena.active(),
                "with a caller workspace at most 4096 unrolled iterations");
        if (w) apply_weights(ctx, w);
        dcrf::check_finite(ctx, unary, L);
        dcrf::fw_diff_forward(ctx, unary, dcrf::resolve_mu(ctx, mu, L), L, y_out,
                              iters, saved);
    });
}

int dcrf_fw_backward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                     int iters, const void *saved, const void *grad_y,
                     void *grad_unary, double *grad_w, double *grad_w_total) {
    return guarded(ctx, [&] {
        require_diff(ctx, L, iters);
        REQUIRE(unary && saved && grad_y && grad_unary, "null argument");
        REQUIRE(grad_unary != grad_y, "grad_unary must not alias grad_y");
        dcrf::check_finite(ctx, grad_y, L);
        std::vector<double> per((size_t)ctx->nimg * ctx->nk, 0.0);
        dcrf::fw_diff_backward(ctx, unary, dcrf::resolve_mu(ctx, mu, L), L, iters,
                               saved, grad_y, grad_unary,
                               (grad_w || grad_w_total) ? per.data() : nullptr);
        if (grad_w)
            for (size_t i = 0; i < per.size(); ++i) grad_w[i] = per[i];
        dcrf::raise_device_errors(ctx);
        if (grad_w_total)   // shared weights: the sum over the images, in order
            for (int m = 0; m < ctx->nk; ++m) {
                double t = 0.0;
                for (int j = 0; j < ctx->nimg; ++j) t += per[(size_t)j * ctx->nk + m];
                grad_w_total[m] = t;
            }
    });
}

// copies between each image's own N_j x L array and the packed layout (rows
// [seg[2j], seg[2j+1]) of `packed`); the rows between images are left alone
static void pack_rows(dcrf_ctx *ctx, const void *const *per_image, void *packed, int L,
                      bool to_packed) {
    const size_t e = ctx->elt(), row = (size_t)L * e;
    for (int j = 0; j < ctx->nimg; ++j) {
        const size_t r0 = ctx->seg_h[2 * j], n = ctx->seg_h[2 * j + 1] - r0;
        char *pk = static_cast<char *>(packed) + r0 * row;
        if (to_packed)
            DCRF_TRY_HIP(hipMemcpyAsync(pk, per_image[j], n * row, hipMemcpyDeviceToDevice,
                                        ctx->stream));
        else
            DCRF_TRY_HIP(hipMemcpyAsync(const_cast<void *>(per_image[j]), pk, n * row,
                                        hipMemcpyDeviceToDevice, ctx->stream));
    }
}

static void require_per_image(dcrf_ctx *ctx, const void *const *a, const char *what) {
    REQUIRE(a != nullptr, std::string(what) + " is null");
    for (int j = 0; j < ctx->nimg; ++j)
        REQUIRE(a[j] != nullptr, std::string(what) + "[" + std::to_string(j) + "] is null");
}

int dcrf_batch_fw_forward(dcrf_ctx *ctx, const void *const *unary, const void *mu, int L,
                          const double *w, int iters, void *const *y_out, void *saved) {
    return guarded(ctx, [&] {
        require_diff(ctx, L, iters);
        require_per_image(ctx, unary, "unary");
        require_per_image(ctx, (const void *const *)y_out, "y_out");
        REQUIRE(saved != nullptr, "null argument");
        REQUIRE(iters <= 4096 || !ctx->arena.active(),
                "with a caller workspace at most 4096 unrolled iterations");
        if (w) apply_weights(ctx, w);
        const size_t bytes = (size_t)ctx->N * L * ctx->elt();
        ctx->pack_a.ensure(bytes, ctx->stream);
        ctx->pack_b.ensure(bytes, ctx->stream);
        pack_rows(ctx, unary, ctx->pack_a.p, L, true);
        dcrf::check_finite(ctx, ctx->pack_a.p, L);
        dcrf::fw_diff_forward(ctx, ctx->pack_a.p, dcrf::resolve_mu(ctx, mu, L), L,
                              ctx->pack_b.p, iters, saved);
        pack_rows(ctx, (const void *const *)y_out, ctx->pack_b.p, L, false);
    });
}

int dcrf_batch_fw_backward(dcrf_ctx *ctx, const void *const *unary, const void *mu, int L,
                           int iters, const void *saved, const void *const *grad_y,
                           void *const *grad_unary, double *grad_w, double *grad_w_total) {
    return guarded(ctx, [&] {
        require_diff(ctx, L, iters);
        require_per_image(ctx, unary, "unary");
        require_per_image(ctx, grad_y, "grad_y");
        require_per_image(ctx, (const void *const *)grad_unary, "grad_unary");
        REQUIRE(saved != nullptr, "null argument");
        const size_t bytes = (size_t)ctx->N * L * ctx->elt();
        for (dcrf::DevBuf *b : {&ctx->pack_a, &ctx->pack_b, &ctx->pack_c})
            b->ensure(bytes, ctx->stream);
        pack_rows(ctx, unary, ctx->pack_a.p, L, true);
        pack_rows(ctx, grad_y, ctx->pack_b.p, L, true);
        dcrf::check_finite(ctx, ctx->pack_b.p, L);
        std::vector<double> per((size_t)ctx->nimg * ctx->nk, 0.0);
        dcrf::fw_diff_backward(ctx, ctx->pack_a.p, dcrf::resolve_mu(ctx, mu, L), L, iters,
                               saved, ctx->pack_b.p, ctx->pack_c.p,
                               (grad_w || grad_w_total) ? per.data() : nullptr);
        pack_rows(ctx, (const void *const *)grad_unary, ctx->pack_c.p, L, false);
        if (grad_w)
            for (size_t i = 0; i < per.size(); ++i) grad_w[i] = per[i];
        dcrf::raise_device_errors(ctx);
        if (grad_w_total)
            for (int m = 0; m < ctx->nk; ++m) {
                double t = 0.0;
                for (int j = 0; j < ctx->nimg; ++j) t += per[(size_t)j * ctx->nk + m];
                grad_w_total[m] = t;
            }
    });
}

int dcrf_lp_descent(dcrf_ctx *ctx, const void *unary, int L, void *y_inout,
                    int steps, double beta0, double *best_obj, void *best_y,
                    double *hist) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout, "null argument");
        require_single(ctx);
        require_lp_mode(ctx);
        REQUIRE(steps >= 0, "steps must be >= 0");
        REQUIRE(std::isfinite(beta0) && beta0 > 0, "beta0 must be > 0");
        REQUIRE(best_y != y_inout, "best_y must not alias y");
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y_inout, L);
        dcrf::lp_descent(ctx, unary, L, y_inout, steps, beta0, best_obj, best_y,
                         hist);
        dcrf::raise_device_errors(ctx);
    });
}

int dcrf_lp_subgradient_tree(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                             int n_nodes, const int32_t *parent, const double *c, void *g,
                             double *S_lp) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y && g && y != g && parent && c, "null or aliased argument");
        require_single(ctx);
        require_lp_mode(ctx);
        const dcrf::TreeSpec tr = dcrf::tree_spec(parent, c, n_nodes, L);
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y, L);
        const double S = dcrf::lp_subgradient_tree(ctx, unary, L, y, tr, g);
        dcrf::raise_device_errors(ctx);
        if (S_lp) *S_lp = S;
    });
}

int dcrf_lp_descent_tree(dcrf_ctx *ctx, const void *unary, int L, void *y_inout,
                         int n_nodes, const int32_t *parent, const double *c, int steps,
                         double beta0, double *best_obj, void *best_y, double *hist) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout && parent && c, "null argument");
        require_single(ctx);
        require_lp_mode(ctx);
        REQUIRE(steps >= 0, "steps must be >= 0");
        REQUIRE(std::isfinite(beta0) && beta0 > 0, "beta0 must be > 0");
        REQUIRE(best_y != y_inout, "best_y must not alias y");
        const dcrf::TreeSpec tr = dcrf::tree_spec(parent, c, n_nodes, L);
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y_inout, L);
        dcrf::lp_descent_tree(ctx, unary, L, y_inout, tr, steps, beta0, best_obj, best_y,
                              hist);
        dcrf::raise_device_errors(ctx);
    });
}

int dcrf_round_kt(dcrf_ctx *ctx, const void *y, int L, const int32_t *round_label,
                  const void *round_theta, int R, int32_t *labels, int *left) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(y && labels && (R == 0 || (round_label && round_theta)), "null argument");
        REQUIRE(R >= 0, "R must be >= 0");
        const int n = dcrf::round_kt(ctx, y, L, round_label, round_theta, R, labels);
        if (left) *left = n;
    });
}

int dcrf_present_labels(dcrf_ctx *ctx, const void *y, int L, double tau,
                        int32_t *labels, int *count) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(y && labels && count, "null argument");
        REQUIRE(std::isfinite(tau), "tau must be finite");
        *count = dcrf::present_labels(ctx, y, L, tau, labels);
    });
}

int dcrf_labels_used(dcrf_ctx *ctx, const int32_t *labels, int L, int32_t *used,
                     int *count) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(labels && used && count, "null argument");
        *count = dcrf::labels_used(ctx, labels, L, used);
    });
}

int dcrf_lp_descent_subset(dcrf_ctx *ctx, const void *unary, int L, void *y_inout,
                           const int32_t *subset, int nsub, int steps, double beta0,
                           double *best_obj, void *best_y, double *hist) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(unary && y_inout && subset, "null argument");
        require_single(ctx);
        require_lp_mode(ctx);
        REQUIRE(nsub >= 1 && nsub <= L, "nsub must be in [1, L]");
        bool seen[256] = {};
        for (int k = 0; k < nsub; ++k) {
            REQUIRE(subset[k] >= 0 && subset[k] < L && !seen[subset[k]],
                    "subset entries must be distinct labels in [0, L)");
            seen[subset[k]] = true;
        }
        REQUIRE(steps >= 0, "steps must be >= 0");
        REQUIRE(std::isfinite(beta0) && beta0 > 0, "beta0 must be > 0");
        REQUIRE(best_y != y_inout, "best_y must not alias y");
        dcrf::check_finite(ctx, unary, L);
        dcrf::check_finite(ctx, y_inout, L);
        dcrf::lp_descent_subset(ctx, unary, L, y_inout, subset, nsub, steps, beta0,
                                best_obj, best_y, hist);
        dcrf::raise_device_errors(ctx);
    });
}

int dcrf_project_simplex(dcrf_ctx *ctx, const void *v, int L, void *y) {
    return guarded(ctx, [&] {
        require_image(ctx);
        check_labels(L);
        REQUIRE(v && y, "null argument");
        dcrf::project_simplex(ctx, v, L, y);
    });
}

int dcrf_workspace_size(int H, int W, int L, const dcrf_kernel *kernels, int nk,
                        int dtype, size_t *bytes) {
    return dcrf_workspace_size_images(1, &H, &W, L, kernels, nk, dtype, bytes);
}

int dcrf_workspace_size_images(int B, const int *H, const int *W, int L,
                               const dcrf_kernel *kernels, int nk, int dtype,
                               size_t *bytes) {
    if (!bytes || !H || !W || !kernels || B < 1 || B > 4096 || nk < 1 ||
        nk > DCRF_MAXK || L < 1 || L > 256 || (dtype != DCRF_F32 && dtype != DCRF_F64))
        return DCRF_EINVAL;
    for (int j = 0; j < B; ++j)
        if (H[j] < 1 || W[j] < 1 || (long long)H[j] * W[j] > (1ll << 28))
            return DCRF_EINVAL;
    *bytes = dcrf::workspace_bound(B, H, W, L, kernels, nk, dtype);
    return DCRF_OK;
}

int dcrf_workspace_used(dcrf_ctx *ctx, size_t *in_use, size_t *peak) {
    return guarded(ctx, [&] {
        REQUIRE(ctx->arena.active(), "the context holds no caller workspace");
        if (in_use) *in_use = ctx->arena.in_use;
        if (peak) *peak = ctx->arena.peak;
    });
}

int dcrf_set_hash_capacity(dcrf_ctx *ctx, size_t slots) {
    return guarded(ctx, [&] {
        REQUIRE(slots == 0 || (slots >= 16 && (slots & (slots - 1)) == 0 &&
                               slots <= (size_t(1) << 32)),
                "slots must be 0 or a power of two in [16, 2^32]");
        ctx->hash_cap = slots;
    });
}

int dcrf_set_lp_leaf(dcrf_ctx *ctx, int leaf) {
    return guarded(ctx, [&] {
        REQUIRE(leaf >= 0 && leaf <= 256, "leaf must be in [0, 256]");
        ctx->lp_leaf = leaf;
    });
}

int dcrf_sync(dcrf_ctx *ctx) {
    return guarded(ctx, [&] { dcrf::raise_device_errors(ctx); });
}

int dcrf_set_profiling(dcrf_ctx *ctx, int enable) {
    return guarded(ctx, [&] {
        DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof.collect();
        ctx->prof.reset();
        ctx->prof.on = enable != 0;
    });
}

int dcrf_get_profile(dcrf_ctx *ctx, int k, const char **name, double *total_ms,
                     long long *launches) {
    return guarded(ctx, [&] {
        REQUIRE(k >= 0 && k < dcrf::PROF_NCLASS, "kernel class out of range");
        ctx->prof.collect();
        if (name) *name = dcrf::prof_name(ctx, k);
        if (total_ms) *total_ms = ctx->prof.total_ms[k];
        if (launches) *launches = ctx->prof.launches[k];
    });
}

}  // extern "C"
