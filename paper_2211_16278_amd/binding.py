"""Thin ctypes binding of libbblock.so (argument marshalling only).

Every function here has the name and arguments of the C entry point declared
in include/bblock.h; the computation runs entirely in the library's HIP
kernels.  Device buffers are passed as torch tensors (their data pointers);
torch only provides device memory and streams.  There is no fallback: when the
library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbblock.so")

FP64, FP32, BF16X3 = 0, 1, 2
C128, C64 = 0, 1
PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
DTYPE = {"c128": C128, "c64": C64}
STATUS = {0: "BBLOCK_OK", 1: "BBLOCK_EINVAL", 2: "BBLOCK_ENOMEM", 3: "BBLOCK_EHIP", 4: "BBLOCK_ENODEV",
          5: "BBLOCK_EUNSUPPORTED"}

# Every symbol include/bblock.h declares.
EXPORTS = ("bblock_create", "bblock_compute", "bblock_compute_noalloc", "bblock_compute_batch", "bblock_compute_projected",
           "bblock_reconstruct", "bblock_mode_triplets", "bblock_mode_contract", "bblock_mode_contract_batch",
           "bblock_set_graph", "bblock_tune",
           "bblock_set_plan", "bblock_get_plan", "bblock_profile", "bblock_profile_read", "bblock_sync",
           "bblock_destroy", "bblock_last_error", "bblock_version")


class BBlockError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class bblock_desc(ctypes.Structure):
    _fields_ = [("q1", ctypes.c_void_p), ("q2", ctypes.c_void_p), ("q3", ctypes.c_void_p),
                ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("out", ctypes.c_void_p)]


class bblock_plan(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int32), ("splits", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("kernel", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libbblock.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libbblock.so not found at %s: build it with __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    h = ctypes.c_void_p
    i32 = ctypes.c_int32
    vp = ctypes.c_void_p
    ip = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "bblock_create": ([ctypes.POINTER(h), i32, i32, i32, i32, ctypes.c_size_t, vp], ctypes.c_int),
        "bblock_compute": ([h, vp, vp, vp, i32, i32, i32, ip, i32, i32, i32, vp], ctypes.c_int),
        "bblock_compute_noalloc": ([h, vp, vp, vp, i32, i32, i32, ip, i32, i32, i32, vp], ctypes.c_int),
        "bblock_compute_batch": ([h, ctypes.POINTER(bblock_desc), i32, ip, i32], ctypes.c_int),
        "bblock_compute_projected": ([h, ctypes.POINTER(bblock_desc), ctypes.POINTER(ctypes.c_double), i32, ip, i32],
                                     ctypes.c_int),
        "bblock_reconstruct": ([h, vp, i32, vp, i32, i32, vp], ctypes.c_int),
        "bblock_mode_triplets": ([h, vp, i32, ip, i32, vp], ctypes.c_int),
        "bblock_mode_contract": ([h, vp, i32, i32, vp, i32, vp, i32, vp, i32, vp], ctypes.c_int),
        "bblock_mode_contract_batch": ([h, vp, i32, i32, i32, vp, i32, vp, i32, vp, i32, vp], ctypes.c_int),
        "bblock_set_graph": ([h, i32], ctypes.c_int),
        "bblock_tune": ([h, i32, i32, i32, i32], ctypes.c_int),
        "bblock_set_plan": ([h, i32, i32, i32, i32, ctypes.POINTER(bblock_plan)], ctypes.c_int),
        "bblock_get_plan": ([h, i32, i32, i32, i32, ctypes.POINTER(bblock_plan)], ctypes.c_int),
        "bblock_profile": ([h, i32], ctypes.c_int),
        "bblock_profile_read": ([h, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "bblock_sync": ([h], ctypes.c_int),
        "bblock_destroy": ([h], ctypes.c_int),
        "bblock_last_error": ([h], ctypes.c_char_p),
        "bblock_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(handle, status: int):
    if status != 0:
        msg = load().bblock_last_error(handle)
        raise BBlockError(status, msg.decode() if msg else "")


def _momenta(mom):
    m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


# ------------------------------------------------------------- C names ---
def bblock_create(L: int, prec: int, in_dtype: int, max_ndil: int, workspace_cap: int = 0, hip_stream: int = 0):
    h = ctypes.c_void_p()
    _check(None, load().bblock_create(ctypes.byref(h), L, prec, in_dtype, max_ndil, workspace_cap, hip_stream))
    return h


def bblock_compute(h, Q1, Q2, Q3, n1, n2, n3, mom, t_begin, t_end, B):
    m, mp = _momenta(mom)
    _check(h, load().bblock_compute(h, _ptr(Q1), _ptr(Q2), _ptr(Q3), n1, n2, n3, mp, m.shape[0], t_begin, t_end,
                                    _ptr(B)))


def bblock_compute_noalloc(h, Q1, Q2, Q3, n1, n2, n3, mom, t_begin, t_end, B):
    m, mp = _momenta(mom)
    _check(h, load().bblock_compute_noalloc(h, _ptr(Q1), _ptr(Q2), _ptr(Q3), n1, n2, n3, mp, m.shape[0], t_begin,
                                            t_end, _ptr(B)))


def _descs(descs):
    arr = (bblock_desc * len(descs))()
    for i, d in enumerate(descs):
        if isinstance(d, bblock_desc):
            arr[i] = d
        else:
            q1, q2, q3, out = d
            arr[i] = bblock_desc(_ptr(q1), _ptr(q2), _ptr(q3), q1.shape[-1], q2.shape[-1], q3.shape[-1], 0,
                                 _ptr(out))
    return arr


def bblock_compute_batch(h, descs, mom):
    """descs: sequence of (q1, q2, q3, out) torch tensors (or bblock_desc)."""
    m, mp = _momenta(mom)
    _check(h, load().bblock_compute_batch(h, _descs(descs), len(descs), mp, m.shape[0]))


def bblock_compute_projected(h, descs, coef, mom):
    """descs as for bblock_compute_batch; coef: one complex coefficient per
    descriptor.  Descriptors sharing an out tensor are summed into it."""
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128).reshape(-1))
    if c.shape[0] != len(descs):
        raise ValueError("one coefficient per descriptor")
    cr = np.ascontiguousarray(np.stack([c.real, c.imag], axis=1).reshape(-1))
    m, mp = _momenta(mom)
    _check(h, load().bblock_compute_projected(h, _descs(descs), cr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              len(descs), mp, m.shape[0]))


def bblock_reconstruct(h, phi, n_ev, Q, n_dil, n_q, q):
    _check(h, load().bblock_reconstruct(h, _ptr(phi), n_ev, _ptr(Q), n_dil, n_q, _ptr(q)))


def bblock_mode_triplets(h, phi, n_ev, mom, T):
    m, mp = _momenta(mom)
    _check(h, load().bblock_mode_triplets(h, _ptr(phi), n_ev, mp, m.shape[0], _ptr(T)))


def bblock_mode_contract(h, T, n_ev, n_mom, Q1, n1, Q2, n2, Q3, n3, B):
    _check(h, load().bblock_mode_contract(h, _ptr(T), n_ev, n_mom, _ptr(Q1), n1, _ptr(Q2), n2, _ptr(Q3), n3,
                                          _ptr(B)))


def bblock_mode_contract_batch(h, T, n_ev, n_mom, n_c, Q1, n1, Q2, n2, Q3, n3, B):
    _check(h, load().bblock_mode_contract_batch(h, _ptr(T), n_ev, n_mom, n_c, _ptr(Q1), n1, _ptr(Q2), n2, _ptr(Q3),
                                                n3, _ptr(B)))


def bblock_set_graph(h, mode):
    """mode: False/0 eager, True/1 capture and replay, "auto"/2 replay schedules of 4+ launches."""
    m = 2 if mode == "auto" else (1 if mode is True else (0 if mode is False else int(mode)))
    _check(h, load().bblock_set_graph(h, m))


def bblock_tune(h, n1, n2, n3, n_mom):
    _check(h, load().bblock_tune(h, n1, n2, n3, n_mom))


def bblock_set_plan(h, n1, n2, n3, n_mom, plan):
    """plan: dict(kernel=, nb=, splits=, persistent=, grid=) or None to forget a forced plan."""
    p = None if plan is None else ctypes.byref(bblock_plan(plan.get("nb", 0), plan.get("splits", 0),
                                                           plan.get("persistent", 0), plan.get("grid", 0),
                                                           plan.get("kernel", 0)))
    _check(h, load().bblock_set_plan(h, n1, n2, n3, n_mom, p))


def bblock_get_plan(h, n1, n2, n3, n_mom) -> dict:
    p = bblock_plan()
    _check(h, load().bblock_get_plan(h, n1, n2, n3, n_mom, ctypes.byref(p)))
    return dict(kernel=p.kernel, nb=p.nb, splits=p.splits, persistent=p.persistent, grid=p.grid)


def bblock_profile(h, enable: bool):
    _check(h, load().bblock_profile(h, 1 if enable else 0))


def bblock_profile_read(h):
    """(gemm_ms, reduce_ms, prep_ms, gemm_launches) summed since the previous read."""
    g, r, p, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _check(h, load().bblock_profile_read(h, ctypes.byref(g), ctypes.byref(r), ctypes.byref(p), ctypes.byref(n)))
    return g.value, r.value, p.value, n.value


def bblock_sync(h):
    _check(h, load().bblock_sync(h))


def bblock_destroy(h):
    _check(None, load().bblock_destroy(h))


def bblock_last_error(h) -> str:
    return load().bblock_last_error(h).decode()


def bblock_version() -> str:
    return load().bblock_version().decode()


# ------------------------------------------------------- convenience ---
class BaryonBlocks:
    """Handle wrapper.  Quark fields are torch tensors on the GPU with shape
    [T, V, 3, n] or [V, 3, n] (complex128 for "c128", complex64 for "c64");
    outputs are complex128 [T, n_mom, n1, n2, n3]."""

    def __init__(self, L: int, prec: str = "bf16x3", in_dtype: str = "c128", max_ndil: int = 64,
                 workspace_cap: int = 0, stream=None):
        import torch
        self.L, self.prec, self.in_dtype = L, prec, in_dtype
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = bblock_create(L, PREC[prec], DTYPE[in_dtype], max_ndil, workspace_cap, self.stream.cuda_stream)

    def compute(self, q1, q2, q3, mom, t_begin: int = 0, t_end: int | None = None, out=None):
        import torch
        q1, q2, q3 = (q if q.dim() == 4 else q.unsqueeze(0) for q in (q1, q2, q3))
        t_end = q1.shape[0] if t_end is None else t_end
        m = np.asarray(mom, dtype=np.int32).reshape(-1, 3)
        shape = (t_end - t_begin, m.shape[0], q1.shape[-1], q2.shape[-1], q3.shape[-1])
        if out is None:
            out = torch.empty(shape, dtype=torch.complex128, device=q1.device)
        bblock_compute(self.h, q1, q2, q3, q1.shape[-1], q2.shape[-1], q3.shape[-1], m, t_begin, t_end, out)
        return out

    def compute_noalloc(self, q1, q2, q3, mom, out, t_begin: int = 0, t_end: int | None = None):
        """compute() through the allocation-free entry point; out must be given."""
        q1, q2, q3 = (q if q.dim() == 4 else q.unsqueeze(0) for q in (q1, q2, q3))
        t_end = q1.shape[0] if t_end is None else t_end
        m = np.asarray(mom, dtype=np.int32).reshape(-1, 3)
        bblock_compute_noalloc(self.h, q1, q2, q3, q1.shape[-1], q2.shape[-1], q3.shape[-1], m, t_begin, t_end, out)
        return out

    def compute_batch(self, descs, mom):
        bblock_compute_batch(self.h, descs, mom)

    def compute_projected(self, descs, coef, mom):
        bblock_compute_projected(self.h, descs, coef, mom)

    def reconstruct(self, phi, Q, out=None):
        """eq. (2): phi [V, 3, n_ev] complex128, Q [n_q, n_dil, n_ev] (or
        [n_dil, n_ev]) complex128 -> q [n_q, V, 3, n_dil] in the handle's
        input dtype (without the leading axis for a 2-d Q)."""
        import torch
        single = Q.dim() == 2
        Qs = Q.unsqueeze(0) if single else Q
        n_q, n_dil, n_ev = Qs.shape
        if out is None:
            dt = torch.complex64 if self.in_dtype == "c64" else torch.complex128
            out = torch.empty((n_q, phi.shape[0], 3, n_dil), dtype=dt, device=phi.device)
        bblock_reconstruct(self.h, phi, n_ev, Qs, n_dil, n_q, out)
        return out[0] if single else out

    def mode_triplets(self, phi, mom, out=None):
        """eq. (4): phi [V, 3, n_ev] in the input dtype -> T [n_mom, n_ev, n_ev, n_ev] complex128."""
        import torch
        n_ev = phi.shape[-1]
        m = np.asarray(mom, dtype=np.int32).reshape(-1, 3)
        if out is None:
            out = torch.empty((m.shape[0], n_ev, n_ev, n_ev), dtype=torch.complex128, device=phi.device)
        bblock_mode_triplets(self.h, phi, n_ev, m, out)
        return out

    def mode_contract(self, T, Q1, Q2, Q3, out=None):
        """B [n_mom, n1, n2, n3] = sum Q1 Q2 Q3 T (all complex128)."""
        import torch
        n_mom, n_ev = T.shape[0], T.shape[1]
        if out is None:
            out = torch.empty((n_mom, Q1.shape[0], Q2.shape[0], Q3.shape[0]), dtype=torch.complex128,
                              device=T.device)
        bblock_mode_contract(self.h, T, n_ev, n_mom, Q1, Q1.shape[0], Q2, Q2.shape[0], Q3, Q3.shape[0], out)
        return out

    def mode_contract_batch(self, T, Q1, Q2, Q3, out=None):
        """n_c triples: Qi [n_c, n_i, n_ev] complex128 -> B [n_c, n_mom, n1, n2, n3]."""
        import torch
        n_mom, n_ev = T.shape[0], T.shape[1]
        n_c = Q1.shape[0]
        if Q2.shape[0] != n_c or Q3.shape[0] != n_c:
            raise ValueError("one coefficient matrix per triple in each of Q1, Q2, Q3")
        if out is None:
            out = torch.empty((n_c, n_mom, Q1.shape[1], Q2.shape[1], Q3.shape[1]), dtype=torch.complex128,
                              device=T.device)
        bblock_mode_contract_batch(self.h, T, n_ev, n_mom, n_c, Q1, Q1.shape[1], Q2, Q2.shape[1], Q3, Q3.shape[1],
                                   out)
        return out

    def tune(self, n1, n2, n3, n_mom):
        bblock_tune(self.h, n1, n2, n3, n_mom)

    def set_plan(self, n1, n2, n3, n_mom, plan):
        bblock_set_plan(self.h, n1, n2, n3, n_mom, plan)

    def get_plan(self, n1, n2, n3, n_mom):
        return bblock_get_plan(self.h, n1, n2, n3, n_mom)

    def set_graph(self, mode):
        bblock_set_graph(self.h, mode)

    def profile(self, enable: bool):
        bblock_profile(self.h, enable)

    def profile_read(self):
        return bblock_profile_read(self.h)

    def sync(self):
        bblock_sync(self.h)

    def close(self):
        if self.h is not None:
            bblock_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
