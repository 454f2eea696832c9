"""Readers of the checkpoint buffer of dcrf_fw_forward, shared by the GPU
tests of the derivative and of the batch (layout as stated in dcrf.h)."""

import numpy as np


def _a256(b):
    return (b + 255) // 256 * 256


def saved_offsets(ctx, N, L, iters, elt):
    """The checkpoint layout stated in the header: y_t, P_t, s_t, the blurred
    vertex values of every lattice ((iters + 1) blocks), then four doubles
    (alpha, a2, b1, interior) per iteration and image, each 256-byte
    aligned. Returns the byte offsets of s_t and of the doubles."""
    q = 16 // elt
    ld = (L + q - 1) // q * q
    vblock = sum(ctx.lattice_info(m)[1] * ld for m in range(ctx.nk))
    p_off = _a256(iters * N * L * elt)
    s_off = _a256(p_off + iters * N * L * elt)
    v_off = _a256(s_off + iters * N * 4)
    st_off = _a256(v_off + (iters + 1) * vblock * elt)
    return s_off, st_off


def unpack_saved(ctx, saved, N, L, iters, elt):
    """(s, stats): s[t] the conditional-gradient labels of iteration t (N
    int32), stats[t * nimg + j] = (alpha, a2, b1, interior) of image j."""
    raw = saved.cpu().numpy()
    s_off, st_off = saved_offsets(ctx, N, L, iters, elt)
    s = raw[s_off:s_off + iters * N * 4].view(np.int32).reshape(iters, N)
    nst = iters * ctx.nimg * 4
    stats = raw[st_off:st_off + nst * 8].view(np.float64).reshape(iters * ctx.nimg, 4)
    return s, stats
