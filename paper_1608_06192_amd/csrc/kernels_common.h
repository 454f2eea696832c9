// Device-side views of the lattices and small helpers shared by the kernels.
#pragma once

#include "dcrf_internal.h"

namespace dcrf {

// One lattice as the splat / blur / slice kernels see it (C channels).
template <typename T>
struct LatView {
    const int32_t *vid;  // N x (d+1) vertex ids (-1: weight 0)
    const T *w;          // N x (d+1) barycentric weights
    const int32_t *nbr;  // (d+1) x M x 2
    T *V0, *V1, *V2;     // M x C: splat target, ping, pong
    const T *Vf;         // the buffer that holds the blurred values
    int d, M;
    T wg;                // w_m * gamma_m
};

template <typename T>
struct LatSet {
    LatView<T> l[DCRF_MAXK];
    long long off[DCRF_MAXK + 1];  // prefix sums of M_m * C
    int nk;
};

template <typename T>
struct ExactSet {
    const T *f[DCRF_MAXK];
    int d[DCRF_MAXK];
    int off[DCRF_MAXK + 1];
    T w[DCRF_MAXK];
    int nk;
};

template <typename T>
inline LatSet<T> make_lat_set(dcrf_ctx *ctx, int C) {
    LatSet<T> s{};
    s.nk = ctx->nk;
    s.off[0] = 0;
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &L = ctx->lat[m];
        LatView<T> &v = s.l[m];
        v.vid = L.pix_vid.as<int32_t>();
        v.w = L.pix_w.as<T>();
        v.nbr = L.nbr.as<int32_t>();
        v.V0 = L.V[0].as<T>();
        v.V1 = L.V[1].as<T>();
        v.V2 = L.V[2].as<T>();
        v.Vf = L.V[final_buffer(L.d)].as<T>();
        v.d = L.d;
        v.M = L.M;
        v.wg = T(ctx->kern[m].weight * L.gamma);
        s.off[m + 1] = s.off[m] + (long long)L.M * C;
    }
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

}  // namespace dcrf
