// Two-dimensional pixel tiles and the per-tile vertex slots of each lattice.
//
// The pixels of every image are cut into tiles of kTileH x kTileW. Within one
// tile the pixels share most of their lattice vertices: on the 500x375
// Voronoi images a 16x16 tile touches on average 147 distinct vertices of
// the 5-D bilateral lattice for its 1536 pixel-vertex pairs, and 50 of the
// spatial lattice for 768 pairs. The static map built here lists, per tile
// and lattice, those distinct vertices ("slots"), and per pixel-vertex pair
// the slot it falls in:
//   ts_off[t] .. ts_off[t+1]   the slots of tile t; ts_vid[s] their vertex
//   tr_slot[a (d+1) + k]       slot of pair (a, k) counted from ts_off[t]
//   sr_off[s] .. sr_off[s+1]   the pairs of slot s: tile-local pixel sr_pix
//                              (row * kTileW + col) and weight sr_w
//   vs_off[v] .. vs_off[v+1]   the slots of vertex v (vs_slot)
// With it,
//  - the splat becomes a gather inside each tile: the tile's values and its
//    pairs are staged once in LDS, each (slot, channel) sum is formed there
//    and added to the vertex row with one atomic, so the pixel values are
//    read once and coalesced;
//  - the one-hot (label) splat does the same with the tile's labels;
//  - the slices stage each tile's slot rows in LDS once instead of gathering
//    d+1 rows per pixel from L2.

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "dcrf_internal.h"
#include "hash_scan.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

// ------------------------------------------------------------ the build

// tile and tile-local index of every pixel of image j (rows a0 .. a0+H W)
__global__ void k_pixel_tiles(int H, int W, int a0, int t0, int ntx,
                              int32_t *__restrict__ pix_tile,
                              uint8_t *__restrict__ pix_li) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= H * W) return;
    const int r = p / W, c = p - (p / W) * W;
    pix_tile[a0 + p] = t0 + (r / kTileH) * ntx + c / kTileW;
    pix_li[a0 + p] = uint8_t((r % kTileH) * kTileW + (c % kTileW));
}

// sort keys of the pixel-vertex pairs: tile * M + vertex (all ones where the
// weight is 0 or the row belongs to no image)
__global__ void k_tile_keys(size_t cnt, int D1, int M, const int32_t *__restrict__ vid,
                            const int32_t *__restrict__ pix_tile,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ refs) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    const int v = vid[e];
    const int t = pix_tile[e / D1];
    keys[e] = (v >= 0 && t >= 0) ? uint64_t(t) * uint64_t(M) + uint64_t(v) : ~0ull;
    refs[e] = uint32_t(e);
}

// first pair of every slot among the sorted pairs
__global__ void k_slot_flags(int n, const uint64_t *__restrict__ keys,
                             int32_t *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_slot_info(int n, int M, const uint64_t *__restrict__ keys,
                            const int32_t *__restrict__ flag,
                            const int32_t *__restrict__ excl,
                            int32_t *__restrict__ ts_vid, int32_t *__restrict__ sr_off,
                            int32_t *__restrict__ tile_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int s = excl[i];
    ts_vid[s] = int(keys[i] % uint64_t(M));
    sr_off[s] = i;
    atomicAdd(&tile_count[int(keys[i] / uint64_t(M))], 1);
}

template <typename T>
__global__ void k_slot_refs(int n, int D1, const uint64_t *__restrict__ keys,
                            const uint32_t *__restrict__ refs, const int32_t *__restrict__ flag,
                            const int32_t *__restrict__ excl, int M,
                            const int32_t *__restrict__ ts_off,
                            const uint8_t *__restrict__ pix_li, const T *__restrict__ pix_w,
                            uint16_t *__restrict__ tr_slot, uint8_t *__restrict__ sr_pix,
                            T *__restrict__ sr_w, uint16_t *__restrict__ sr_slot,
                            int32_t *__restrict__ vs_count,
                            const int32_t *__restrict__ ts_vid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = refs[i];
    const int s = excl[i] + flag[i] - 1;
    const int t = int(keys[i] / uint64_t(M));
    tr_slot[e] = uint16_t(s - ts_off[t]);
    sr_slot[i] = uint16_t(s - ts_off[t]);
    sr_pix[i] = pix_li[e / uint32_t(D1)];
    sr_w[i] = pix_w[e];
    if (flag[i]) atomicAdd(&vs_count[ts_vid[s]], 1);
}

__global__ void k_fill_u16(size_t n, uint16_t *__restrict__ p, uint16_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i32t(size_t n, int32_t *__restrict__ p, int32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_set_last(int32_t *p, int v) { *p = v; }

// slots listed per vertex: fill by a cursor per vertex, then each vertex's
// list is put in slot order (the slots are few per vertex)
__global__ void k_vertex_slots(int nslots, const int32_t *__restrict__ ts_vid,
                               const int32_t *__restrict__ vs_off,
                               int32_t *__restrict__ cursor, int32_t *__restrict__ vs_slot) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    const int v = ts_vid[s];
    vs_slot[vs_off[v] + atomicAdd(&cursor[v], 1)] = s;
}

__global__ void k_sort_vertex_slots(int M, const int32_t *__restrict__ vs_off,
                                    int32_t *__restrict__ vs_slot) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= M) return;
    const int b = vs_off[v], e = vs_off[v + 1];
    for (int i = b + 1; i < e; ++i) {   // insertion sort
        const int x = vs_slot[i];
        int j = i - 1;
        while (j >= b && vs_slot[j] > x) {
            vs_slot[j + 1] = vs_slot[j];
            --j;
        }
        vs_slot[j + 1] = x;
    }
}

template <typename T>
void build_tile_map(dcrf_ctx *ctx, int m, const int32_t *pix_tile,
                    const uint8_t *pix_li) {
    Lattice &L = ctx->lat[m];
    const hipStream_t s = ctx->stream;
    const int D1 = L.d + 1, M = L.M;
    const size_t cnt = (size_t)ctx->N * D1;
    const int nt = ctx->ntiles;
    DevBuf k0, k1, r0, r1, flag, excl, temp, tcount, cur;
    struct Free {
        DevBuf *b[9];
        ~Free() { for (DevBuf *x : b) x->release(); }
    } fr{{&k0, &k1, &r0, &r1, &flag, &excl, &temp, &tcount, &cur}};
    k0.ensure(cnt * 8, s);
    k1.ensure(cnt * 8, s);
    r0.ensure(cnt * 4, s);
    r1.ensure(cnt * 4, s);
    hipLaunchKernelGGL(k_tile_keys, dim3(ceil_div((long long)cnt, 256)), dim3(256), 0, s,
                       cnt, D1, std::max(M, 1), L.pix_vid.as<int32_t>(), pix_tile,
                       k0.as<uint64_t>(), r0.as<uint32_t>());
    size_t bytes = 0;
    int bits = 1;
    while (bits < 64 && (1ull << bits) <= (unsigned long long)nt * (unsigned long long)std::max(M, 1))
        ++bits;
    DCRF_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k0.as<uint64_t>(),
                                                   k1.as<uint64_t>(), r0.as<uint32_t>(),
                                                   r1.as<uint32_t>(), int(cnt), 0, 64, s));
    temp.ensure(bytes, s);
    // all 64 bits: the invalid key ~0 must sort after every valid one
    DCRF_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, bytes, k0.as<uint64_t>(),
                                                   k1.as<uint64_t>(), r0.as<uint32_t>(),
                                                   r1.as<uint32_t>(), int(cnt), 0, 64, s));
    (void)bits;
    const int n = L.nent;   // the valid pairs, first in the sorted order
    flag.ensure((size_t)std::max(n, 1) * 4, s);
    excl.ensure((size_t)(n + 1) * 4, s);
    ctx->scratch.ensure(64 + (size_t)(ceil_div((long long)std::max({n, M, nt}) + 1,
                                               kScanTile) + 2) * 4, s);
    if (n > 0)
        hipLaunchKernelGGL(k_slot_flags, dim3(ceil_div(n, 256)), dim3(256), 0, s, n,
                           k1.as<uint64_t>(), flag.as<int32_t>());
    scan_ints(ctx, flag.as<int32_t>(), n, excl.as<int32_t>());
    int nslots = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&nslots, excl.as<int32_t>() + n, 4, hipMemcpyDeviceToHost, s));
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    L.nslots = nslots;
    L.ts_vid.ensure((size_t)std::max(nslots, 1) * 4, s);
    L.sr_off.ensure((size_t)(nslots + 1) * 4, s);
    L.ts_off.ensure((size_t)(nt + 1) * 4, s);
    tcount.ensure((size_t)(nt + 1) * 4, s);
    DCRF_TRY_HIP(hipMemsetAsync(tcount.p, 0, (size_t)(nt + 1) * 4, s));
    if (n > 0)
        hipLaunchKernelGGL(k_slot_info, dim3(ceil_div(n, 256)), dim3(256), 0, s, n,
                           std::max(M, 1), k1.as<uint64_t>(), flag.as<int32_t>(),
                           excl.as<int32_t>(), L.ts_vid.as<int32_t>(),
                           L.sr_off.as<int32_t>(), tcount.as<int32_t>());
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, s, L.sr_off.as<int32_t>() + nslots,
                       n);
    scan_ints(ctx, tcount.as<int32_t>(), nt, L.ts_off.as<int32_t>());
    L.tr_slot.ensure(cnt * 2, s);
    hipLaunchKernelGGL(k_fill_u16, dim3(ceil_div((long long)cnt, 256)), dim3(256), 0, s,
                       cnt, L.tr_slot.as<uint16_t>(), uint16_t(0xffff));
    L.sr_pix.ensure((size_t)std::max(n, 1), s);
    L.sr_w.ensure((size_t)std::max(n, 1) * sizeof(T), s);
    L.sr_slot.ensure((size_t)std::max(n, 1) * 2, s);
    L.vs_off.ensure((size_t)(M + 1) * 4, s);
    cur.ensure((size_t)(M + 1) * 4, s);
    DCRF_TRY_HIP(hipMemsetAsync(cur.p, 0, (size_t)(M + 1) * 4, s));
    if (n > 0)
        hipLaunchKernelGGL((k_slot_refs<T>), dim3(ceil_div(n, 256)), dim3(256), 0, s, n, D1,
                           k1.as<uint64_t>(), r1.as<uint32_t>(), flag.as<int32_t>(),
                           excl.as<int32_t>(), std::max(M, 1), L.ts_off.as<int32_t>(),
                           pix_li, L.pix_w.as<T>(), L.tr_slot.as<uint16_t>(),
                           L.sr_pix.as<uint8_t>(), L.sr_w.as<T>(), L.sr_slot.as<uint16_t>(),
                           cur.as<int32_t>(), L.ts_vid.as<int32_t>());
    scan_ints(ctx, cur.as<int32_t>(), M, L.vs_off.as<int32_t>());
    L.vs_slot.ensure((size_t)std::max(nslots, 1) * 4, s);
    DCRF_TRY_HIP(hipMemsetAsync(cur.p, 0, (size_t)(M + 1) * 4, s));
    if (nslots > 0)
        hipLaunchKernelGGL(k_vertex_slots, dim3(ceil_div(nslots, 256)), dim3(256), 0, s,
                           nslots, L.ts_vid.as<int32_t>(), L.vs_off.as<int32_t>(),
                           cur.as<int32_t>(), L.vs_slot.as<int32_t>());
    if (M > 0)
        hipLaunchKernelGGL(k_sort_vertex_slots, dim3(ceil_div(M, 256)), dim3(256), 0, s,
                           M, L.vs_off.as<int32_t>(), L.vs_slot.as<int32_t>());
    DCRF_CHECK_LAUNCH();
    // the largest slot count of a tile (sizes the LDS of the slices)
    std::vector<int> off(nt + 1);
    DCRF_TRY_HIP(hipMemcpyAsync(off.data(), L.ts_off.p, (nt + 1) * 4, hipMemcpyDeviceToHost,
                                s));
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    L.tile_slots.assign(nt, 0);
    int mx = 0;
    for (int t = 0; t < nt; ++t) {
        L.tile_slots[t] = off[t + 1] - off[t];
        mx = std::max(mx, L.tile_slots[t]);
    }
    L.max_tile_slots = mx;
}

}  // namespace

void ensure_tiles(dcrf_ctx *ctx) {
    if (ctx->ntiles == 0) build_tiles(ctx);
}

void build_tiles(dcrf_ctx *ctx) {
    const hipStream_t s = ctx->stream;
    std::vector<int4> td;
    std::vector<int> toff(ctx->nimg + 1, 0);
    for (int j = 0; j < ctx->nimg; ++j) {
        const int H = ctx->img_H[j], W = ctx->img_W[j], a0 = ctx->seg_h[2 * j];
        const int nty = ceil_div(H, kTileH), ntx = ceil_div(W, kTileW);
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx)
                td.push_back(make_int4(a0 + ty * kTileH * W + tx * kTileW, W,
                                       std::min(kTileH, H - ty * kTileH),
                                       std::min(kTileW, W - tx * kTileW)));
        toff[j + 1] = int(td.size());
    }
    ctx->ntiles = int(td.size());
    ctx->tile_img_off_h = toff;
    ctx->tiles.ensure(td.size() * sizeof(int4), s);
    ctx->tile_img_off.ensure(toff.size() * 4, s);
    DCRF_TRY_HIP(hipMemcpyAsync(ctx->tiles.p, td.data(), td.size() * sizeof(int4),
                                hipMemcpyHostToDevice, s));
    DCRF_TRY_HIP(hipMemcpyAsync(ctx->tile_img_off.p, ctx->tile_img_off_h.data(),
                                toff.size() * 4, hipMemcpyHostToDevice, s));
    DevBuf pt, pl;
    struct Free {
        DevBuf *b[2];
        ~Free() { for (DevBuf *x : b) x->release(); }
    } fr{{&pt, &pl}};
    pt.ensure((size_t)ctx->N * 4, s);
    pl.ensure((size_t)ctx->N, s);
    hipLaunchKernelGGL(k_fill_i32t, dim3(ceil_div(ctx->N, 256)), dim3(256), 0, s,
                       (size_t)ctx->N, pt.as<int32_t>(), -1);
    for (int j = 0; j < ctx->nimg; ++j) {
        const int H = ctx->img_H[j], W = ctx->img_W[j];
        hipLaunchKernelGGL(k_pixel_tiles, dim3(ceil_div(H * W, 256)), dim3(256), 0, s, H,
                           W, ctx->seg_h[2 * j], toff[j], ceil_div(W, kTileW),
                           pt.as<int32_t>(), pl.as<uint8_t>());
    }
    DCRF_CHECK_LAUNCH();
    for (int m = 0; m < ctx->nk; ++m) {
        if (ctx->dtype == DCRF_F64)
            build_tile_map<double>(ctx, m, pt.as<int32_t>(), pl.as<uint8_t>());
        else
            build_tile_map<float>(ctx, m, pt.as<int32_t>(), pl.as<uint8_t>());
    }
    DCRF_TRY_HIP(hipStreamSynchronize(s));
}

}  // namespace dcrf
