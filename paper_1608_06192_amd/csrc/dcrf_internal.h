// Internal declarations of the dcrf library: the context, device buffers and
// the host-side launchers of the kernels in lattice.hip, filter.hip and
// solvers.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

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

// A grow-only device allocation; new memory is zero-filled.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need, hipStream_t s) {
        if (need <= bytes) return;
        if (p) {
            DCRF_TRY_HIP(hipStreamSynchronize(s));
            DCRF_TRY_HIP(hipFree(p));
            p = nullptr;
            bytes = 0;
        }
        size_t n = need < 256 ? 256 : need;
        DCRF_TRY_HIP(hipMalloc(&p, n));
        DCRF_TRY_HIP(hipMemsetAsync(p, 0, n, s));
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
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
    DevBuf V[3];         // M x C x T: splat target (kept zero), ping, pong
    DevBuf feat;         // N x d x T features (exact mode)
    void release() {
        for (DevBuf *b : {&hkeys, &slot_vid, &pix_slot, &pix_vid, &pix_w,
                          &vkeys, &nbr, &V[0], &V[1], &V[2], &feat})
            b->release();
    }
};

}  // namespace dcrf

struct dcrf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int H = 0, W = 0, N = 0, nk = 0, dtype = DCRF_F32;
    int mode = DCRF_FILTER_LATTICE;
    bool has_image = false;
    dcrf_kernel kern[DCRF_MAXK];
    dcrf::Lattice lat[DCRF_MAXK];
    double wsum = 0;
    dcrf::DevBuf r;          // N x T: K'1
    dcrf::DevBuf scratch;    // small device scratch (flags, counters)
    dcrf::DevBuf tmpA, tmpB; // N x C scratch arrays
    // Frank-Wolfe state
    dcrf::DevBuf fw_c, fw_Py, fw_Ps, fw_s, fw_sprev, fw_part, fw_scal,
        fw_trace, fw_mu;
    std::string err;
    size_t elt() const { return dtype == DCRF_F64 ? 8 : 4; }
};

namespace dcrf {

// ------------------------------------------------------------ launchers

// lattice.hip
void build_lattices(dcrf_ctx *ctx, const float *rgb);
void lattice_export(dcrf_ctx *ctx, int m, int32_t *keys, int32_t *vid,
                    double *w);

// filter.hip
// out = K' in (N x C), lattice or exact, optionally the transpose
void filter_apply(dcrf_ctx *ctx, const void *in, void *out, int C,
                  bool adjoint, bool exact);
// r = K'1
void compute_row_sums(dcrf_ctx *ctx);
// make sure every lattice has vertex buffers for C channels
void ensure_vertex_buffers(dcrf_ctx *ctx, int C);
// splat of one-hot labels (C = L channels), blur; leaves results in the final
// buffers of each lattice
void splat_labels(dcrf_ctx *ctx, const int32_t *labels, int L);
void splat_dense(dcrf_ctx *ctx, const void *in, int C);
void blur_all(dcrf_ctx *ctx, int C, bool adjoint);
// index of the buffer that holds the blurred values of lattice m
inline int final_buffer(int d) { return (d % 2 == 0) ? 1 : 2; }

// solvers.hip
void qp_apply(dcrf_ctx *ctx, const void *y, const void *mu, int L, void *out);
void frank_wolfe(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                 void *y, int iters, dcrf_iter_trace *trace, const void *c_in,
                 bool have_Py);
void dc_gen(dcrf_ctx *ctx, const void *unary, const void *mu, int L, void *y,
            int outer, int inner, double *S_hist);
void round_labels(dcrf_ctx *ctx, const void *y, int L, int32_t *labels);
double energy(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
              const int32_t *labels);

inline int ceil_div(long long a, long long b) { return int((a + b - 1) / b); }

}  // namespace dcrf
