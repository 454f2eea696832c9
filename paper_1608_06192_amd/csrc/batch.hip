// Several images in one context.
//
// The filter of a batch is block-diagonal: no pixel of one image interacts
// with a pixel of another. Each image's lattices are built on their own (the
// vertex keys carry no image index) and then concatenated: vertex ids,
// neighbour ids, inverse-index entries and chunk lists are renumbered by
// per-image offsets. The filter kernels then cover the whole batch in one
// launch per stage without knowing about images at all, since every vertex
// and every neighbour link stays inside its image. The pixel rows of image j
// start at a multiple of kAlign rows, so a tile of the per-pixel kernels
// starts 16-byte aligned exactly as for a single image; the rows between two
// images have no vertices and are not solver variables.
//
// The launch shapes that have a choice (inverse-index chunk length of the
// splats; blur directions per launch, 16-byte vectors per thread and threads
// per block of the blur) are picked by a small autotuner that times the
// filter paths of the context's own lattices for each candidate.

#include <algorithm>
#include <vector>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

constexpr int kAlign = 64;   // pixel rows

// dst[i] = src[i] + add, or -1 where src[i] < 0
__global__ void k_copy_shift(size_t n, const int32_t *__restrict__ src,
                             int32_t *__restrict__ dst, int add) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int32_t v = src[i];
        dst[i] = v >= 0 ? v + add : -1;
    }
}

__global__ void k_fill_neg(size_t n, int32_t *__restrict__ p) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = -1;
}

__global__ void k_set_int(int32_t *p, int v) { *p = v; }

void copy_shift(hipStream_t s, const void *src, void *dst, size_t n, int add) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_copy_shift, dim3(ceil_div((long long)n, 256)), dim3(256),
                       0, s, n, static_cast<const int32_t *>(src),
                       static_cast<int32_t *>(dst), add);
    DCRF_CHECK_LAUNCH();
}

void copy_bytes(hipStream_t s, const void *src, void *dst, size_t bytes) {
    if (bytes)
        DCRF_TRY_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
}

// the buffers of a single-image build that the batch keeps
struct Part {
    int M = 0, nent = 0;
    DevBuf pix_vid, pix_w, nbr, vkeys, csr_off, ent_pix, ent_w, ent_v;
    void release() {
        for (DevBuf *b : {&pix_vid, &pix_w, &nbr, &vkeys, &csr_off, &ent_pix,
                          &ent_w, &ent_v})
            b->release();
    }
};

// a scratch context whose device buffers are released however we leave
struct ScratchCtx {
    dcrf_ctx c;
    ~ScratchCtx() {
        for (auto &L : c.lat) L.release();
        for (DevBuf *b : {&c.r, &c.scratch, &c.tmpA, &c.tmpB, &c.seg}) b->release();
    }
};

struct PartList {
    std::vector<Part> p;
    ~PartList() {
        for (auto &x : p) x.release();
    }
};

}  // namespace

void set_segments(dcrf_ctx *ctx, const std::vector<int> &seg) {
    ctx->nimg = int(seg.size() / 2);
    ctx->seg_h = seg;
    ctx->seg.ensure(seg.size() * 4, ctx->stream);
    DCRF_TRY_HIP(hipMemcpyAsync(ctx->seg.p, ctx->seg_h.data(), seg.size() * 4,
                                hipMemcpyHostToDevice, ctx->stream));
    DCRF_TRY_HIP(hipStreamSynchronize(ctx->stream));
}

void build_batch(dcrf_ctx *ctx, int B, const int *H, const int *W,
                 const float *const *rgb) {
    const hipStream_t s = ctx->stream;
    std::vector<int> seg(2 * (size_t)B);
    long long off = 0;
    for (int j = 0; j < B; ++j) {
        seg[2 * j] = int(off);
        seg[2 * j + 1] = int(off + (long long)H[j] * W[j]);
        off = (seg[2 * j + 1] + kAlign - 1) / kAlign * kAlign;
        if (off > (1ll << 28)) fail(DCRF_EINVAL, "batch larger than 2^28 pixels");
    }
    const int N = seg[2 * B - 1];
    const size_t e = ctx->elt();

    // build every image's lattices in a scratch context
    ScratchCtx tmp;
    tmp.c.device = ctx->device;
    tmp.c.stream = s;
    tmp.c.nk = ctx->nk;
    tmp.c.dtype = ctx->dtype;
    tmp.c.splat_chunk = ctx->splat_chunk;
    tmp.c.hash_cap = ctx->hash_cap;
    for (int m = 0; m < ctx->nk; ++m) tmp.c.kern[m] = ctx->kern[m];
    PartList parts;
    parts.p.resize((size_t)B * ctx->nk);
    for (int j = 0; j < B; ++j) {
        tmp.c.H = H[j];
        tmp.c.W = W[j];
        tmp.c.N = H[j] * W[j];
        build_lattices(&tmp.c, rgb[j]);
        for (int m = 0; m < ctx->nk; ++m) {
            Lattice &L = tmp.c.lat[m];
            Part &P = parts.p[(size_t)j * ctx->nk + m];
            const int D1 = L.d + 1;
            P.M = L.M;
            P.nent = L.nent;
            const size_t np = (size_t)tmp.c.N * D1;
            P.pix_vid.ensure(np * 4, s);
            P.pix_w.ensure(np * e, s);
            P.nbr.ensure((size_t)D1 * std::max(L.M, 1) * 2 * 4, s);
            P.vkeys.ensure((size_t)std::max(L.M, 1) * 8, s);
            P.csr_off.ensure((size_t)(L.M + 1) * 4, s);
            P.ent_pix.ensure((size_t)std::max(L.nent, 1) * 4, s);
            P.ent_w.ensure((size_t)std::max(L.nent, 1) * e, s);
            P.ent_v.ensure((size_t)std::max(L.nent, 1) * 4, s);
            copy_bytes(s, L.pix_vid.p, P.pix_vid.p, np * 4);
            copy_bytes(s, L.pix_w.p, P.pix_w.p, np * e);
            copy_bytes(s, L.nbr.p, P.nbr.p, (size_t)D1 * L.M * 2 * 4);
            copy_bytes(s, L.vkeys.p, P.vkeys.p, (size_t)L.M * 8);
            copy_bytes(s, L.csr_off.p, P.csr_off.p, (size_t)(L.M + 1) * 4);
            copy_bytes(s, L.ent_pix.p, P.ent_pix.p, (size_t)L.nent * 4);
            copy_bytes(s, L.ent_w.p, P.ent_w.p, (size_t)L.nent * e);
            copy_bytes(s, L.ent_v.p, P.ent_v.p, (size_t)L.nent * 4);
        }
    }

    // concatenate
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &L = ctx->lat[m];
        L.release();
        L = Lattice();
        L.d = tmp.c.lat[m].d;
        L.gamma = tmp.c.lat[m].gamma;
        L.chunk = ctx->splat_chunk;
        const int D1 = L.d + 1;
        long long Mt = 0, Et = 0;
        for (int j = 0; j < B; ++j) {
            Mt += parts.p[(size_t)j * ctx->nk + m].M;
            Et += parts.p[(size_t)j * ctx->nk + m].nent;
        }
        if (Mt >= (1ll << 31) / (2 * D1) || Et >= (1ll << 31))
            fail(DCRF_ECAPACITY, "batch lattice too large");
        L.M = int(Mt);
        L.nent = int(Et);
        const size_t np = (size_t)N * D1;
        L.pix_vid.ensure(np * 4, s);
        L.pix_w.ensure(np * e, s);   // zero-filled: rows between images
        hipLaunchKernelGGL(k_fill_neg, dim3(ceil_div((long long)np, 256)), dim3(256),
                           0, s, np, L.pix_vid.as<int32_t>());
        L.nbr.ensure((size_t)D1 * std::max(L.M, 1) * 2 * 4, s);
        L.vkeys.ensure((size_t)std::max(L.M, 1) * 8, s);
        L.csr_off.ensure((size_t)(L.M + 1) * 4, s);
        L.csr_tmp.ensure((size_t)(L.M + 1) * 4, s);
        L.ent_pix.ensure((size_t)std::max(L.nent, 1) * 4, s);
        L.ent_w.ensure((size_t)std::max(L.nent, 1) * e, s);
        L.ent_v.ensure((size_t)std::max(L.nent, 1) * 4, s);
        int Moff = 0, Eoff = 0;
        for (int j = 0; j < B; ++j) {
            const Part &P = parts.p[(size_t)j * ctx->nk + m];
            const int Nj = H[j] * W[j];
            const size_t po = (size_t)seg[2 * j] * D1;
            copy_shift(s, P.pix_vid.p, L.pix_vid.as<int32_t>() + po, (size_t)Nj * D1,
                       Moff);
            copy_bytes(s, P.pix_w.p, L.pix_w.as<char>() + po * e, (size_t)Nj * D1 * e);
            for (int dir = 0; dir < D1; ++dir)
                copy_shift(s, P.nbr.as<int32_t>() + (size_t)dir * P.M * 2,
                           L.nbr.as<int32_t>() + ((size_t)dir * L.M + Moff) * 2,
                           (size_t)P.M * 2, Moff);
            copy_bytes(s, P.vkeys.p, L.vkeys.as<char>() + (size_t)Moff * 8,
                       (size_t)P.M * 8);
            copy_shift(s, P.csr_off.p, L.csr_off.as<int32_t>() + Moff, (size_t)P.M,
                       Eoff);
            copy_shift(s, P.ent_pix.p, L.ent_pix.as<int32_t>() + Eoff, (size_t)P.nent,
                       seg[2 * j]);
            copy_bytes(s, P.ent_w.p, L.ent_w.as<char>() + (size_t)Eoff * e,
                       (size_t)P.nent * e);
            copy_shift(s, P.ent_v.p, L.ent_v.as<int32_t>() + Eoff, (size_t)P.nent,
                       Moff);
            Moff += P.M;
            Eoff += P.nent;
        }
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s,
                           L.csr_off.as<int32_t>() + L.M, L.nent);
        DCRF_CHECK_LAUNCH();
    }
    ctx->N = N;
    ctx->H = 0;
    ctx->W = 0;
    ctx->img_H.assign(H, H + B);
    ctx->img_W.assign(W, W + B);
    rechunk(ctx, ctx->splat_chunk, ctx->dense_chunk);
    set_segments(ctx, seg);
}

namespace {

__global__ void k_iota_mod(int N, int L, int32_t *__restrict__ x) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < N) x[a] = int((a * 7u + (a >> 5)) % unsigned(L));
}

}  // namespace

void autotune(dcrf_ctx *ctx, int L, int reps, double *best_ms) {
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    const size_t NL = (size_t)N * L;
    ctx->tmpA.ensure(NL * ctx->elt(), s);
    ctx->tmpB.ensure(NL * ctx->elt(), s);
    ctx->fw_s.ensure((size_t)N * 4, s);
    fill_ones(ctx, ctx->tmpA.p, NL);
    hipLaunchKernelGGL(k_iota_mod, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, L,
                       ctx->fw_s.as<int32_t>());
    DCRF_CHECK_LAUNCH();
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    hipEvent_t e0, e1;
    DCRF_TRY_HIP(hipEventCreate(&e0));
    DCRF_TRY_HIP(hipEventCreate(&e1));
    struct Cand { int chunk, dense, stage, vpt, block, group, tiles; };
    auto apply = [&](const Cand &c) {
        if (c.chunk != ctx->splat_chunk || c.dense != ctx->dense_chunk)
            rechunk(ctx, c.chunk, c.dense);
        ctx->splat_lds = c.stage;
        ctx->blur_vpt = c.vpt;
        ctx->blur_block = c.block;
        ctx->blur_group = c.group;
        ctx->tile_mode = c.tiles;
        if (c.tiles) ensure_tiles(ctx);
    };
    Cand best = {ctx->splat_chunk, ctx->dense_chunk, ctx->splat_lds, ctx->blur_vpt,
                 ctx->blur_block, ctx->blur_group, ctx->tile_mode};
    double best_t = 1e300;
    auto run = [&] {
        // the dense filter and the one-hot path of a Frank-Wolfe iteration
        filter_apply(ctx, ctx->tmpA.p, ctx->tmpB.p, L, false, DCRF_FILTER_LATTICE);
        splat_labels(ctx, ctx->fw_s.as<int32_t>(), L);
        blur_all(ctx, L, false);
        slice_into(ctx, ctx->tmpA.p, nullptr, L, nullptr, nullptr, ctx->tmpB.p,
                   false);
    };
    auto measure = [&](const std::vector<Cand> &cands) {
        for (const Cand &c : cands) {
            apply(c);
            run();
            DCRF_TRY_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) run();
            DCRF_TRY_HIP(hipEventRecord(e1, s));
            DCRF_TRY_HIP(hipEventSynchronize(e1));
            float ms = 0;
            DCRF_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double t = double(ms) / reps;
            if (t < best_t) {
                best_t = t;
                best = c;
            }
        }
    };
    try {
        // first the blur shape, the tiling and the one-hot chunks, then the
        // dense splat's chunks and staging (which only the dense filter uses)
        std::vector<Cand> cands;
        for (int tiles : {0, 1})
            for (int chunk : {32, 64, 128})
                for (int vpt : {1, 2})
                    for (int block : {128, 256})
                        for (int group : {1, 2, 3}) {
                            if (tiles && chunk != 64) continue;   // no chunks used
                            cands.push_back({chunk, best.dense, best.stage, vpt, block,
                                             group, tiles});
                        }
        measure(cands);
        if (!best.tiles) {
            cands.clear();
            for (int dense : {16, 32, 64})
                for (int stage : {0, 1}) {
                    Cand c = best;
                    c.dense = dense;
                    c.stage = stage;
                    cands.push_back(c);
                }
            best_t = 1e300;
            measure(cands);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->prof.on = prof;
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prof.on = prof;
    apply(best);
    if (best_ms) *best_ms = best_t;
}

}  // namespace dcrf
