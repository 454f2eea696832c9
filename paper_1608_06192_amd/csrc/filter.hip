// The pairwise filter K' Y = sum_m w_m K_m Y - (sum_m w_m) Y (eq. fb summed
// over the kernels of eq. pairwise, without the b = a term of
// eq. labelling-energy), in two forms:
//
//  - permutohedral: K_m Y ~ gamma_d slice(blur(splat(Y))). Splat scatters
//    b * Y_a into the d+1 vertices of pixel a's simplex with atomics; the blur
//    runs d+1 out-of-place passes V'[v] = V[v]/2 + (V[v+u_j] + V[v-u_j])/4
//    (missing neighbours read as 0) over both lattices in one launch per pass;
//    slice gathers sum_k b_k V[v_k]. gamma_d = (4 pi / 3)^{d/2} sqrt(d+1)
//    makes the response to a uniform density equal to the Gaussian integral.
//    The transpose runs the same splat and slice with the blur directions in
//    reverse order.
//  - exact: the O(N^2) sum on the vector ALU, tiled through LDS (reference
//    mode for small images and for measuring the lattice's error).
//
// Vertex values are stored row-major, M x C. Three buffers per lattice:
// V[0] is the splat target and is kept all-zero between calls (the second
// blur pass clears it while the passes ping-pong between V[1] and V[2]).

#include <algorithm>

#include "dcrf_internal.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

// ------------------------------------------------------------------ splat

template <typename T>
__global__ void __launch_bounds__(256)
k_splat_dense(int N, int C, const T *__restrict__ in, LatSet<T> ls) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * C) return;
    const int a = int(e / C);
    const int c = int(e - (size_t)a * C);
    const T v = in[e];
    if (v == T(0)) return;
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int D1 = L.d + 1;
        for (int k = 0; k < D1; ++k) {
            const int id = L.vid[(size_t)a * D1 + k];
            if (id >= 0)
                atomic_add(&L.V0[(size_t)id * C + c], L.w[(size_t)a * D1 + k] * v);
        }
    }
}

// one-hot input: pixel a contributes b to channel labels[a]
template <typename T>
__global__ void __launch_bounds__(256)
k_splat_labels(int N, int C, const int32_t *__restrict__ labels, LatSet<T> ls) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int c = labels[a];
    if (c < 0 || c >= C) return;   // out-of-range labels are rejected by the caller
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int D1 = L.d + 1;
        for (int k = 0; k < D1; ++k) {
            const int id = L.vid[(size_t)a * D1 + k];
            if (id >= 0)
                atomic_add(&L.V0[(size_t)id * C + c], L.w[(size_t)a * D1 + k]);
        }
    }
}

// ------------------------------------------------------------------- blur

// pass p of every lattice with d >= p, flattened over sum_m M_m x C
template <typename T>
__global__ void __launch_bounds__(256)
k_blur_pass(LatSet<T> ls, int C, int pass, int reverse, long long total) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int m = 0;
    while (m + 1 < ls.nk && e >= ls.off[m + 1]) ++m;
    const LatView<T> &L = ls.l[m];
    if (pass > L.d) return;
    const long long r = e - ls.off[m];
    const int v = int(r / C);
    const int c = int(r - (long long)v * C);
    const int j = reverse ? (L.d - pass) : pass;
    const T *src = (pass == 0) ? L.V0 : ((pass & 1) ? L.V1 : L.V2);
    T *dst = (pass & 1) ? L.V2 : L.V1;
    const int np = L.nbr[((size_t)j * L.M + v) * 2 + 0];
    const int nm = L.nbr[((size_t)j * L.M + v) * 2 + 1];
    const T vp = np >= 0 ? src[(size_t)np * C + c] : T(0);
    const T vm = nm >= 0 ? src[(size_t)nm * C + c] : T(0);
    dst[(size_t)v * C + c] = T(0.5) * src[(size_t)v * C + c] + T(0.25) * (vp + vm);
    if (pass == 1) L.V0[(size_t)v * C + c] = T(0);
}

// ------------------------------------------------------------------ slice

// out = sum_m w_m gamma_m slice_m - wsum * in   (raw K' in, N x C)
template <typename T>
__global__ void __launch_bounds__(256)
k_slice_raw(int N, int C, const T *__restrict__ in, T *__restrict__ out,
            LatSet<T> ls, T wsum) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * C) return;
    const int a = int(e / C);
    const int c = int(e - (size_t)a * C);
    T acc = T(0);
    for (int m = 0; m < ls.nk; ++m) {
        const LatView<T> &L = ls.l[m];
        const int D1 = L.d + 1;
        T s = T(0);
        for (int k = 0; k < D1; ++k) {
            const int id = L.vid[(size_t)a * D1 + k];
            if (id >= 0) s += L.w[(size_t)a * D1 + k] * L.Vf[(size_t)id * C + c];
        }
        acc += L.wg * s;
    }
    out[e] = acc - wsum * in[e];
}

// ------------------------------------------------------------------ exact

constexpr int kExactTile = 128;
constexpr int kExactMaxF = 16;   // sum of feature dimensions over the kernels
constexpr int kExactCB = 8;      // channels per pass

// out_a[c0 .. c0+CB) (+)= sum_{b != a} sum_m w_m exp(-|f_a - f_b|^2/2) in_b
template <typename T>
__global__ void __launch_bounds__(kExactTile)
k_exact(int N, int C, int c0, const T *__restrict__ in, T *__restrict__ out,
        ExactSet<T> ex) {
    __shared__ T sf[kExactTile][kExactMaxF];
    __shared__ T sv[kExactTile][kExactCB];
    const int a = blockIdx.x * kExactTile + threadIdx.x;
    const int nf = ex.off[ex.nk];
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
    (void)nf;
    if (a < N)
        for (int c = 0; c < cn; ++c) out[(size_t)a * C + c0 + c] = acc[c];
}

template <typename T>
void filter_t(dcrf_ctx *ctx, const void *in_, void *out_, int C, bool adjoint,
              bool exact) {
    const hipStream_t s = ctx->stream;
    const T *in = static_cast<const T *>(in_);
    T *out = static_cast<T *>(out_);
    const int N = ctx->N;
    if (exact) {
        ExactSet<T> ex = make_exact_set<T>(ctx);
        if (ex.off[ex.nk] > kExactMaxF)
            fail(DCRF_EUNSUPPORTED, "exact filter supports at most 16 feature "
                                    "dimensions over all kernels");
        for (int c0 = 0; c0 < C; c0 += kExactCB)
            hipLaunchKernelGGL((k_exact<T>), dim3(ceil_div(N, kExactTile)),
                               dim3(kExactTile), 0, s, N, C, c0, in, out, ex);
        DCRF_CHECK_LAUNCH();
        return;
    }
    splat_dense(ctx, in, C);
    blur_all(ctx, C, adjoint);
    LatSet<T> ls = make_lat_set<T>(ctx, C);
    hipLaunchKernelGGL((k_slice_raw<T>), dim3(ceil_div((long long)N * C, 256)),
                       dim3(256), 0, s, N, C, in, out, ls, T(ctx->wsum));
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void splat_dense_t(dcrf_ctx *ctx, const void *in, int C) {
    ensure_vertex_buffers(ctx, C);
    LatSet<T> ls = make_lat_set<T>(ctx, C);
    hipLaunchKernelGGL((k_splat_dense<T>),
                       dim3(ceil_div((long long)ctx->N * C, 256)), dim3(256), 0,
                       ctx->stream, ctx->N, C, static_cast<const T *>(in), ls);
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void splat_labels_t(dcrf_ctx *ctx, const int32_t *labels, int L) {
    ensure_vertex_buffers(ctx, L);
    LatSet<T> ls = make_lat_set<T>(ctx, L);
    hipLaunchKernelGGL((k_splat_labels<T>), dim3(ceil_div(ctx->N, 256)),
                       dim3(256), 0, ctx->stream, ctx->N, L, labels, ls);
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void blur_all_t(dcrf_ctx *ctx, int C, bool adjoint) {
    LatSet<T> ls = make_lat_set<T>(ctx, C);
    int maxd = 0;
    for (int m = 0; m < ctx->nk; ++m) maxd = std::max(maxd, ctx->lat[m].d);
    const long long total = ls.off[ctx->nk];
    if (total == 0) return;
    for (int p = 0; p <= maxd; ++p)
        hipLaunchKernelGGL((k_blur_pass<T>), dim3(ceil_div(total, 256)),
                           dim3(256), 0, ctx->stream, ls, C, p, adjoint ? 1 : 0,
                           total);
    DCRF_CHECK_LAUNCH();
}

}  // namespace

void ensure_vertex_buffers(dcrf_ctx *ctx, int C) {
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &L = ctx->lat[m];
        const size_t bytes = (size_t)(L.M > 0 ? L.M : 1) * C * ctx->elt();
        for (int b = 0; b < 3; ++b) L.V[b].ensure(bytes, ctx->stream);
    }
}

void splat_dense(dcrf_ctx *ctx, const void *in, int C) {
    if (ctx->dtype == DCRF_F64)
        splat_dense_t<double>(ctx, in, C);
    else
        splat_dense_t<float>(ctx, in, C);
}

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

void filter_apply(dcrf_ctx *ctx, const void *in, void *out, int C,
                  bool adjoint, bool exact) {
    if (ctx->dtype == DCRF_F64)
        filter_t<double>(ctx, in, out, C, adjoint, exact);
    else
        filter_t<float>(ctx, in, out, C, adjoint, exact);
}

void compute_row_sums(dcrf_ctx *ctx) {
    const size_t e = ctx->elt();
    ctx->r.ensure((size_t)ctx->N * e, ctx->stream);
    ctx->tmpA.ensure((size_t)ctx->N * e, ctx->stream);
    fill_ones(ctx, ctx->tmpA.p, ctx->N);
    filter_apply(ctx, ctx->tmpA.p, ctx->r.p, 1, false,
                 ctx->mode == DCRF_FILTER_EXACT);
}

}  // namespace dcrf
