"""Python binding of the HIP library ``libdcrf.so`` (C ABI in include/dcrf.h).

Argument marshalling only: every step runs in the library's kernels. Tensors
supply device memory; calls are enqueued on torch's current stream. The
module raises at import when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcrf.so")

DCRF_OK = 0
DCRF_F32, DCRF_F64 = 0, 1
DCRF_FILTER_LATTICE, DCRF_FILTER_EXACT, DCRF_FILTER_SEPARABLE = 0, 1, 2
DCRF_ADJOINT, DCRF_EXACT, DCRF_SEPARABLE = 1, 2, 4
DCRF_KEEP_SELF, DCRF_PER_KERNEL = 8, 16

STATUS = {0: "DCRF_OK", -1: "DCRF_EINVAL", -2: "DCRF_ENOMEM", -3: "DCRF_ERANGE",
          -4: "DCRF_ECAPACITY", -5: "DCRF_EHIP", -6: "DCRF_EUNSUPPORTED",
          -7: "DCRF_ESTATE"}


class DcrfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class dcrf_kernel(ctypes.Structure):
    _fields_ = [("use_rgb", ctypes.c_int), ("theta_pos", ctypes.c_double),
                ("theta_rgb", ctypes.c_double), ("weight", ctypes.c_double)]


class dcrf_iter_trace(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("gap", ctypes.c_double),
                ("alpha", ctypes.c_double), ("changed", ctypes.c_double)]


class dcrf_tune(ctypes.Structure):
    _fields_ = [("splat_chunk", ctypes.c_int), ("dense_chunk", ctypes.c_int),
                ("splat_stage", ctypes.c_int),
                ("blur_vectors_per_thread", ctypes.c_int),
                ("blur_block", ctypes.c_int), ("blur_group", ctypes.c_int),
                ("tiles", ctypes.c_int), ("fw_splat", ctypes.c_int),
                ("fw_persistent", ctypes.c_int), ("ms", ctypes.c_double)]


# name -> (restype, argtypes); mirrors include/dcrf.h
_P, _I, _U, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
PROTOTYPES = {
    "dcrf_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "dcrf_destroy": (_I, [_P]),
    "dcrf_last_error": (ctypes.c_char_p, [_P]),
    "dcrf_set_stream": (_I, [_P, _P]),
    "dcrf_version": (ctypes.c_char_p, []),
    "dcrf_workspace_size": (_I, [_I, _I, _I, ctypes.POINTER(dcrf_kernel), _I, _I,
                                 ctypes.POINTER(ctypes.c_size_t)]),
    "dcrf_workspace_size_images": (_I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I), _I,
                                        ctypes.POINTER(dcrf_kernel), _I, _I,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "dcrf_set_image": (_I, [_P, _I, _I, _P, ctypes.POINTER(dcrf_kernel), _I, _I, _P,
                            ctypes.c_size_t]),
    "dcrf_set_images": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                             ctypes.POINTER(_P), ctypes.POINTER(dcrf_kernel), _I,
                             _I, _P, ctypes.c_size_t]),
    "dcrf_batch_set_images": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                   ctypes.POINTER(_P), ctypes.POINTER(dcrf_kernel), _I,
                                   _I, _P, ctypes.c_size_t]),
    "dcrf_workspace_used": (_I, [_P, ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t)]),
    "dcrf_set_hash_capacity": (_I, [_P, ctypes.c_size_t]),
    "dcrf_sync": (_I, [_P]),
    "dcrf_image_layout": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I),
                               ctypes.POINTER(_I)]),
    "dcrf_autotune": (_I, [_P, _I, _I, ctypes.POINTER(dcrf_tune)]),
    "dcrf_set_tune": (_I, [_P, ctypes.POINTER(dcrf_tune)]),
    "dcrf_set_weights": (_I, [_P, _PD, _I]),
    "dcrf_set_filter_mode": (_I, [_P, _I]),
    "dcrf_lattice_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "dcrf_lattice_export": (_I, [_P, _I, _P, _P, _P]),
    "dcrf_filter": (_I, [_P, _P, _P, _I, _U]),
    "dcrf_qp_apply": (_I, [_P, _P, _P, _I, _P]),
    "dcrf_qp_frank_wolfe": (_I, [_P, _P, _P, _I, _P, _I,
                                 ctypes.POINTER(dcrf_iter_trace)]),
    "dcrf_dc_gen": (_I, [_P, _P, _P, _I, _P, _I, _I, _PD]),
    "dcrf_qp_frank_wolfe_noalloc": (_I, [_P, _P, _P, _I, _P, _I,
                                         ctypes.POINTER(dcrf_iter_trace)]),
    "dcrf_noalloc_scratch_bytes": (_I, [ctypes.POINTER(ctypes.c_size_t)]),
    "dcrf_dc_neg": (_I, [_P, _P, _P, _I, _P, _I, _I, _PD]),
    "dcrf_round": (_I, [_P, _P, _I, _P]),
    "dcrf_energy": (_I, [_P, _P, _P, _I, _P, _PD]),
    "dcrf_lp_subgradient": (_I, [_P, _P, _I, _P, _P, _PD]),
    "dcrf_lp_descent": (_I, [_P, _P, _I, _P, _I, _D, _PD, _P, _PD]),
    "dcrf_project_simplex": (_I, [_P, _P, _I, _P]),
    "dcrf_lp_subgradient_tree": (_I, [_P, _P, _I, _P, _I, _P, _P, _P, _PD]),
    "dcrf_lp_descent_tree": (_I, [_P, _P, _I, _P, _I, _P, _P, _I, _D, _PD, _P, _PD]),
    "dcrf_round_kt": (_I, [_P, _P, _I, _P, _P, _I, _P, ctypes.POINTER(_I)]),
    "dcrf_set_lp_leaf": (_I, [_P, _I]),
    "dcrf_present_labels": (_I, [_P, _P, _I, _D, _P, ctypes.POINTER(_I)]),
    "dcrf_labels_used": (_I, [_P, _P, _I, _P, ctypes.POINTER(_I)]),
    "dcrf_lp_descent_subset": (_I, [_P, _P, _I, _P, _P, _I, _I, _D, _PD, _P, _PD]),
    "dcrf_fw_saved_size": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_size_t)]),
    "dcrf_fw_forward": (_I, [_P, _P, _P, _I, _PD, _I, _P, _P]),
    "dcrf_fw_backward": (_I, [_P, _P, _P, _I, _I, _P, _P, _P, _PD, _PD]),
    "dcrf_batch_fw_forward": (_I, [_P, _P, _P, _I, _PD, _I, _P, _P]),
    "dcrf_batch_fw_backward": (_I, [_P, _P, _P, _I, _I, _P, _P, _P, _PD, _PD]),
    "dcrf_set_profiling": (_I, [_P, _I]),
    "dcrf_get_profile": (_I, [_P, _I, ctypes.POINTER(ctypes.c_char_p), _PD,
                              ctypes.POINTER(ctypes.c_longlong)]),
}

PROF_CLASSES = 9


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python __graft_entry__.py` "
            "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def workspace_size(sizes, L: int, kernels, dtype=torch.float32) -> int:
    """dcrf_workspace_size(_images) for images of sizes [(H, W), ...]"""
    code = {torch.float32: DCRF_F32, torch.float64: DCRF_F64}[dtype]
    ks = _kernels(kernels)
    B = len(sizes)
    Hs = (ctypes.c_int * B)(*[int(h) for h, _ in sizes])
    Ws = (ctypes.c_int * B)(*[int(w) for _, w in sizes])
    n = ctypes.c_size_t()
    st = _lib.dcrf_workspace_size_images(B, Hs, Ws, L, ks, len(ks), code, ctypes.byref(n))
    if st != DCRF_OK:
        raise DcrfError(st, "invalid workspace size query")
    return n.value


def _kernels(kernels):
    arr = (dcrf_kernel * len(kernels))()
    for i, k in enumerate(kernels):
        if isinstance(k, dict):
            k = (k["use_rgb"], k["theta_pos"], k.get("theta_rgb", 0.0),
                 k["weight"])
        arr[i] = dcrf_kernel(int(k[0]), float(k[1]), float(k[2]), float(k[3]))
    return arr


class Context:
    """One image's lattices and solver workspace on one device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        st = torch.cuda.current_stream(self.device).cuda_stream
        self._check(_lib.dcrf_create(ctypes.byref(self._h), device,
                                     ctypes.c_void_p(st)), create=True)
        self.dtype = None
        self.N = 0
        self.nk = 0
        self.nimg, self.seg = 1, []

    def __del__(self):
        # at interpreter exit the module globals may already be gone; the
        # process end releases the device memory then
        if _lib is not None and getattr(self, "_h", None) and self._h.value:
            _lib.dcrf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def _check(self, status: int, create: bool = False):
        if status != DCRF_OK:
            msg = _lib.dcrf_last_error(None if create else self._h)
            raise DcrfError(status, (msg or b"").decode())

    def _mu(self, mu):
        """mu as a pointer; None stands for the Potts compatibility [i != j]"""
        return None if mu is None else self._arg(mu, name="mu")

    def _stream(self):
        st = torch.cuda.current_stream(self.device).cuda_stream
        self._check(_lib.dcrf_set_stream(self._h, ctypes.c_void_p(st)))

    def _arg(self, t: torch.Tensor, dtype=None, name="argument"):
        dtype = dtype or self.dtype
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor on "
                             f"{self.device}")
        return _ptr(t)

    # -- image -----------------------------------------------------------
    def _workspace(self, ws):
        """(pointer, bytes) of a caller workspace (a uint8 device tensor) or
        (None, 0); the context keeps a reference until the next image."""
        self._ws = ws
        if ws is None:
            return None, 0
        if ws.device != self.device or ws.dtype != torch.uint8 or not ws.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on the device")
        return _ptr(ws), ws.numel()

    def set_image(self, H: int, W: int, rgb: torch.Tensor, kernels,
                  dtype=torch.float32, workspace: torch.Tensor | None = None):
        self._stream()
        code = {torch.float32: DCRF_F32, torch.float64: DCRF_F64}[dtype]
        ks = _kernels(kernels)
        wp, wb = self._workspace(workspace)
        self._check(_lib.dcrf_set_image(
            self._h, H, W, self._arg(rgb, torch.float32, "rgb"), ks, len(ks),
            code, wp, wb))
        self.dtype, self.N, self.nk, self.H, self.W = dtype, H * W, len(ks), H, W
        self.nimg, self.seg = 1, [(0, H * W)]

    def set_images(self, sizes, rgbs, kernels, dtype=torch.float32,
                   workspace: torch.Tensor | None = None):
        """A batch: sizes = [(H, W), ...], rgbs = float32 (H*W, 3) tensors on
        the device. Afterwards every N x C argument is one packed array in
        the layout of `seg` (rows seg[j][0]:seg[j][1] are image j)."""
        B = len(sizes)
        self._stream()
        code = {torch.float32: DCRF_F32, torch.float64: DCRF_F64}[dtype]
        ks = _kernels(kernels)
        Hs = (ctypes.c_int * B)(*[int(h) for h, _ in sizes])
        Ws = (ctypes.c_int * B)(*[int(w) for _, w in sizes])
        ptrs = (ctypes.c_void_p * B)(*[self._arg(r, torch.float32, "rgb").value
                                      for r in rgbs])
        wp, wb = self._workspace(workspace)
        self._check(_lib.dcrf_set_images(self._h, B, Hs, Ws, ptrs, ks, len(ks),
                                         code, wp, wb))
        self.dtype, self.nk = dtype, len(ks)
        self.H = self.W = None
        nimg, rows = ctypes.c_int(), ctypes.c_int()
        seg = (ctypes.c_int * (2 * B))()
        self._check(_lib.dcrf_image_layout(self._h, ctypes.byref(nimg),
                                           ctypes.byref(rows), seg))
        self.nimg, self.N = nimg.value, rows.value
        self.seg = [(seg[2 * j], seg[2 * j + 1]) for j in range(self.nimg)]

    def pack(self, arrays, C: int):
        """Per-image (N_j x C) tensors -> one packed (N x C) tensor; the rows
        between images are zero."""
        out = torch.zeros(self.N, C, dtype=self.dtype, device=self.device)
        for (a, b), x in zip(self.seg, arrays):
            out[a:b].copy_(x.reshape(b - a, C))
        return out

    def unpack(self, packed):
        """One packed (N x C) tensor -> per-image views."""
        return [packed[a:b] for a, b in self.seg]

    def set_tune(self, splat_chunk=64, blur_vectors_per_thread=1,
                 blur_block=256, blur_group=2, tiles=0, dense_chunk=32,
                 splat_stage=1, fw_splat=0, fw_persistent=0, **_):
        t = dcrf_tune(splat_chunk, dense_chunk, splat_stage, blur_vectors_per_thread,
                      blur_block, blur_group, tiles, fw_splat, fw_persistent, 0.0)
        self._stream()
        self._check(_lib.dcrf_set_tune(self._h, ctypes.byref(t)))

    def autotune(self, L: int, reps: int = 5):
        t = dcrf_tune()
        self._stream()
        self._check(_lib.dcrf_autotune(self._h, L, reps, ctypes.byref(t)))
        return dict(splat_chunk=t.splat_chunk, dense_chunk=t.dense_chunk,
                    splat_stage=t.splat_stage,
                    blur_vectors_per_thread=t.blur_vectors_per_thread,
                    blur_block=t.blur_block, blur_group=t.blur_group,
                    tiles=t.tiles, fw_splat=t.fw_splat, fw_persistent=t.fw_persistent,
                    ms=t.ms)

    def workspace_used(self):
        """(bytes in use, peak bytes) of the context's caller workspace"""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(_lib.dcrf_workspace_used(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_hash_capacity(self, slots: int):
        self._check(_lib.dcrf_set_hash_capacity(self._h, int(slots)))

    def sync(self):
        """wait for the stream; raises for device-detected input errors"""
        self._stream()
        self._check(_lib.dcrf_sync(self._h))

    def set_weights(self, w):
        arr = (ctypes.c_double * len(w))(*[float(v) for v in w])
        self._stream()
        self._check(_lib.dcrf_set_weights(self._h, arr, len(w)))

    def set_filter_mode(self, mode: str):
        self._stream()
        m = {"lattice": DCRF_FILTER_LATTICE, "exact": DCRF_FILTER_EXACT,
             "separable": DCRF_FILTER_SEPARABLE}[mode]
        self._check(_lib.dcrf_set_filter_mode(self._h, m))

    def lattice_info(self, m: int):
        d, M = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.dcrf_lattice_info(self._h, m, ctypes.byref(d),
                                           ctypes.byref(M)))
        return d.value, M.value

    def lattice_export(self, m: int):
        import numpy as np
        d, M = self.lattice_info(m)
        keys = np.empty((M, d), np.int32)
        vid = np.empty((self.N, d + 1), np.int32)
        w = np.empty((self.N, d + 1), np.float64)
        self._check(_lib.dcrf_lattice_export(
            self._h, m, keys.ctypes.data_as(_P), vid.ctypes.data_as(_P),
            w.ctypes.data_as(_P)))
        return keys, vid, w

    # -- filter ----------------------------------------------------------
    def filter(self, x: torch.Tensor, adjoint=False, exact=False,
               out: torch.Tensor | None = None, separable=False, keep_self=False,
               per_kernel=False) -> torch.Tensor:
        """K' x (or its variants; per_kernel: a (nk, N, C) tensor of the
        kernels' shares)"""
        C = x.shape[1] if x.dim() == 2 else 1
        if out is None:
            shape = (self.nk,) + tuple(x.shape) if per_kernel else x.shape
            out = torch.empty(shape, dtype=x.dtype, device=x.device)
        flags = ((DCRF_ADJOINT if adjoint else 0) | (DCRF_EXACT if exact else 0)
                 | (DCRF_SEPARABLE if separable else 0) | (DCRF_KEEP_SELF if keep_self else 0)
                 | (DCRF_PER_KERNEL if per_kernel else 0))
        self._stream()
        self._check(_lib.dcrf_filter(self._h, self._arg(x, name="in"),
                                     self._arg(out, name="out"), C, flags))
        return out

    def qp_apply(self, y: torch.Tensor, mu: torch.Tensor,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty_like(y) if out is None else out
        self._stream()
        self._check(_lib.dcrf_qp_apply(self._h, self._arg(y), self._mu(mu),
                                       y.shape[1], self._arg(out)))
        return out

    # -- solvers ---------------------------------------------------------
    def qp_frank_wolfe(self, unary, mu, y, iters: int, trace: bool = True):
        tr = (dcrf_iter_trace * max(iters * self.nimg, 1))() if trace else None
        self._stream()
        self._check(_lib.dcrf_qp_frank_wolfe(
            self._h, self._arg(unary, name="unary"), self._mu(mu),
            unary.shape[1], self._arg(y, name="y"), iters, tr))
        if not trace:
            return None
        rec = [(t.objective, t.gap, t.alpha, t.changed)
               for t in tr[:iters * self.nimg]]
        if self.nimg == 1:
            return rec
        return [rec[j::self.nimg] for j in range(self.nimg)]

    def qp_frank_wolfe_noalloc(self, unary, mu, y, iters: int, trace: bool = True):
        """qp_frank_wolfe through the entry point that allocates nothing"""
        tr = (dcrf_iter_trace * max(iters * self.nimg, 1))() if trace else None
        self._stream()
        self._check(_lib.dcrf_qp_frank_wolfe_noalloc(
            self._h, self._arg(unary, name="unary"), self._mu(mu),
            unary.shape[1], self._arg(y, name="y"), iters, tr))
        if not trace:
            return None
        rec = [(t.objective, t.gap, t.alpha, t.changed)
               for t in tr[:iters * self.nimg]]
        if self.nimg == 1:
            return rec
        return [rec[j::self.nimg] for j in range(self.nimg)]

    def dc_gen(self, unary, mu, y, outer: int, inner: int):
        hist = (ctypes.c_double * (outer + 1))()
        self._stream()
        self._check(_lib.dcrf_dc_gen(
            self._h, self._arg(unary), self._mu(mu), unary.shape[1],
            self._arg(y), outer, inner, hist))
        return list(hist)

    def dc_neg(self, unary, mu, y, outer: int, inner: int = 1, hist: bool = True):
        """CCCP on the negative semi-definite decomposition, in place on y;
        returns S(y) before the first and after every step (None without
        hist)."""
        h = (ctypes.c_double * (outer + 1))() if hist else None
        self._stream()
        self._check(_lib.dcrf_dc_neg(
            self._h, self._arg(unary), self._mu(mu), unary.shape[1],
            self._arg(y), outer, inner, h))
        return list(h) if hist else None

    def round(self, y: torch.Tensor) -> torch.Tensor:
        lab = torch.empty(y.shape[0], dtype=torch.int32, device=self.device)
        self._stream()
        self._check(_lib.dcrf_round(self._h, self._arg(y), y.shape[1],
                                    _ptr(lab)))
        return lab

    # -- LP relaxation (Potts) -------------------------------------------
    def lp_subgradient(self, unary, y, g: torch.Tensor | None = None):
        """(g, S_LP(y)) at y: eq. grad_lp by divide and conquer."""
        g = torch.empty_like(y) if g is None else g
        S = ctypes.c_double()
        self._stream()
        self._check(_lib.dcrf_lp_subgradient(
            self._h, self._arg(unary), unary.shape[1], self._arg(y),
            self._arg(g), ctypes.byref(S)))
        return g, S.value

    def set_lp_leaf(self, leaf: int):
        """exact pair sums inside divide-and-conquer nodes of at most `leaf`
        positions (0: the plain recursion)"""
        self._check(_lib.dcrf_set_lp_leaf(self._h, int(leaf)))

    def lp_descent(self, unary, y, steps: int, beta0: float,
                   best_y: torch.Tensor | None = None):
        """Projected subgradient descent in place on y; returns (best S_LP,
        history of S_LP(y_t))."""
        hist = (ctypes.c_double * max(steps, 1))()
        best = ctypes.c_double()
        self._stream()
        self._check(_lib.dcrf_lp_descent(
            self._h, self._arg(unary), unary.shape[1], self._arg(y), steps,
            float(beta0), ctypes.byref(best),
            None if best_y is None else self._arg(best_y), hist))
        return best.value, list(hist[:steps])

    @staticmethod
    def _tree(parent, c):
        n = len(parent)
        if len(c) != n:
            raise ValueError("parent and c must have one entry per node")
        return (n, (ctypes.c_int32 * n)(*[int(v) for v in parent]),
                (ctypes.c_double * n)(*[float(v) for v in c]))

    def lp_subgradient_tree(self, unary, y, parent, c, g: torch.Tensor | None = None):
        """(g, S) of the LP for the tree metric given by parent[] (node k < L
        is label k) and the subtree weights c"""
        g = torch.empty_like(y) if g is None else g
        n, pa, ca = self._tree(parent, c)
        S = ctypes.c_double()
        self._stream()
        self._check(_lib.dcrf_lp_subgradient_tree(
            self._h, self._arg(unary), unary.shape[1], self._arg(y), n, pa, ca,
            self._arg(g), ctypes.byref(S)))
        return g, S.value

    def lp_descent_tree(self, unary, y, parent, c, steps: int, beta0: float,
                        best_y: torch.Tensor | None = None):
        """projected subgradient descent on the tree LP, in place on y;
        returns (best objective, history)"""
        n, pa, ca = self._tree(parent, c)
        hist = (ctypes.c_double * max(steps, 1))()
        best = ctypes.c_double()
        self._stream()
        self._check(_lib.dcrf_lp_descent_tree(
            self._h, self._arg(unary), unary.shape[1], self._arg(y), n, pa, ca, steps,
            float(beta0), ctypes.byref(best), None if best_y is None else self._arg(best_y),
            hist))
        return best.value, list(hist[:steps])

    def round_kt(self, y, round_label: torch.Tensor, round_theta: torch.Tensor):
        """(labels, pixels left to the argmax): Kleinberg-Tardos rounding with
        the given draws (device tensors: int32 labels, thresholds in the
        context dtype)"""
        lab = torch.empty(y.shape[0], dtype=torch.int32, device=self.device)
        left = ctypes.c_int()
        R = round_label.numel()
        self._stream()
        self._check(_lib.dcrf_round_kt(
            self._h, self._arg(y), y.shape[1],
            self._arg(round_label, torch.int32, "round_label") if R else None,
            self._arg(round_theta, name="round_theta") if R else None, R, _ptr(lab),
            ctypes.byref(left)))
        return lab, left.value

    def present_labels(self, y, tau: float):
        L = y.shape[1]
        out = (ctypes.c_int32 * L)()
        n = ctypes.c_int()
        self._stream()
        self._check(_lib.dcrf_present_labels(self._h, self._arg(y), L, float(tau), out,
                                             ctypes.byref(n)))
        return list(out[:n.value])

    def labels_used(self, labels: torch.Tensor, L: int):
        out = (ctypes.c_int32 * L)()
        n = ctypes.c_int()
        self._stream()
        self._check(_lib.dcrf_labels_used(self._h, self._arg(labels, torch.int32, "labels"),
                                          L, out, ctypes.byref(n)))
        return list(out[:n.value])

    def lp_descent_subset(self, unary, y, subset, steps: int, beta0: float,
                          best_y: torch.Tensor | None = None):
        """the LP descent on the labels of `subset` only, in place on y;
        returns (best S_LP, history)"""
        sub = (ctypes.c_int32 * len(subset))(*[int(i) for i in subset])
        hist = (ctypes.c_double * max(steps, 1))()
        best = ctypes.c_double()
        self._stream()
        self._check(_lib.dcrf_lp_descent_subset(
            self._h, self._arg(unary), unary.shape[1], self._arg(y), sub, len(subset),
            steps, float(beta0), ctypes.byref(best),
            None if best_y is None else self._arg(best_y), hist))
        return best.value, list(hist[:steps])

    def project_simplex(self, v: torch.Tensor, out: torch.Tensor | None = None):
        out = torch.empty_like(v) if out is None else out
        self._stream()
        self._check(_lib.dcrf_project_simplex(self._h, self._arg(v), v.shape[1],
                                              self._arg(out)))
        return out

    # -- differentiation of unrolled Frank-Wolfe --------------------------
    def fw_saved_size(self, L: int, iters: int) -> int:
        n = ctypes.c_size_t()
        self._check(_lib.dcrf_fw_saved_size(self._h, L, iters, ctypes.byref(n)))
        return n.value

    def fw_forward(self, unary, mu, iters: int, w=None):
        """y_T of `iters` Frank-Wolfe iterations from softmax(-unary), with the
        kernel weights w (nk floats; None keeps the context's); returns
        (y_T, saved), saved being the checkpoint buffer (uint8 tensor) that
        fw_backward needs."""
        L = unary.shape[1]
        saved = torch.empty(self.fw_saved_size(L, iters), dtype=torch.uint8,
                            device=self.device)
        y = torch.empty_like(unary)
        wa = None if w is None else (ctypes.c_double * len(w))(*[float(v) for v in w])
        self._stream()
        self._check(_lib.dcrf_fw_forward(
            self._h, self._arg(unary, name="unary"), self._mu(mu), L, wa,
            iters, self._arg(y), _ptr(saved)))
        return y, saved

    def fw_backward(self, unary, mu, iters: int, saved, grad_y, summed=False):
        """(dl/dunary, dl/dw) for dl/dy_T = grad_y; dl/dw is a list of nk
        floats, or for a batch a list of nimg such lists; with ``summed`` the
        batch's sum over its images (the gradient of weights the images
        share), computed in the library."""
        gphi = torch.empty_like(unary)
        gw = (ctypes.c_double * (self.nk * self.nimg))()
        tot = (ctypes.c_double * self.nk)()
        self._stream()
        self._check(_lib.dcrf_fw_backward(
            self._h, self._arg(unary, name="unary"), self._mu(mu),
            unary.shape[1], iters, _ptr(saved), self._arg(grad_y, name="grad_y"),
            self._arg(gphi), gw, tot))
        if summed:
            return gphi, list(tot)
        if self.nimg == 1:
            return gphi, list(gw)
        return gphi, [list(gw[j * self.nk:(j + 1) * self.nk])
                      for j in range(self.nimg)]

    # -- the batch calls with one array per image ------------------------
    def _ptrs(self, ts, name):
        if len(ts) != self.nimg:
            raise ValueError(f"{name} needs one tensor per image ({self.nimg})")
        return (ctypes.c_void_p * len(ts))(*[self._arg(t, name=name) for t in ts])

    def batch_fw_forward(self, unaries, mu, iters: int, w=None):
        """fw_forward with one (N_j, L) tensor per image; returns ([y_j], saved)"""
        L = unaries[0].shape[1]
        saved = torch.empty(self.fw_saved_size(L, iters), dtype=torch.uint8,
                            device=self.device)
        ys = [torch.empty_like(u) for u in unaries]
        wa = None if w is None else (ctypes.c_double * len(w))(*[float(v) for v in w])
        self._stream()
        self._check(_lib.dcrf_batch_fw_forward(
            self._h, self._ptrs(unaries, "unary"), self._mu(mu), L, wa, iters,
            self._ptrs(ys, "y_out"), _ptr(saved)))
        return ys, saved

    def batch_fw_backward(self, unaries, mu, iters: int, saved, grad_ys):
        """fw_backward with one tensor per image: ([dl/dunary_j], per-image
        dl/dw lists, their sum)"""
        L = unaries[0].shape[1]
        gphis = [torch.empty_like(u) for u in unaries]
        gw = (ctypes.c_double * (self.nk * self.nimg))()
        tot = (ctypes.c_double * self.nk)()
        self._stream()
        self._check(_lib.dcrf_batch_fw_backward(
            self._h, self._ptrs(unaries, "unary"), self._mu(mu), L, iters, _ptr(saved),
            self._ptrs(grad_ys, "grad_y"), self._ptrs(gphis, "grad_unary"), gw, tot))
        return gphis, [list(gw[j * self.nk:(j + 1) * self.nk])
                       for j in range(self.nimg)], list(tot)

    # -- profiling -------------------------------------------------------
    def set_profiling(self, on: bool):
        self._check(_lib.dcrf_set_profiling(self._h, int(on)))

    def profile(self):
        """{kernel name: (total ms, launches)} since profiling was enabled."""
        out = {}
        for k in range(PROF_CLASSES):
            name, ms, n = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_longlong()
            self._check(_lib.dcrf_get_profile(self._h, k, ctypes.byref(name),
                                              ctypes.byref(ms), ctypes.byref(n)))
            out[name.value.decode()] = (ms.value, n.value)
        return out

    def energy(self, unary, mu, labels: torch.Tensor) -> float:
        e = ctypes.c_double()
        self._stream()
        self._check(_lib.dcrf_energy(
            self._h, self._arg(unary), self._mu(mu), unary.shape[1],
            self._arg(labels, torch.int32, "labels"), ctypes.byref(e)))
        return e.value
