"""Thin Python binding of libvlp (include/vlp.h), argument marshalling only.

Every function named vlp_* forwards to the C entry point of the same name and
raises VlpError on a non-zero status.  Device buffers are torch tensors on the
HIP device (int32 or uint32-compatible dtypes); their data_ptr() is passed
through.  The library must be built (build.py); importing this module on a
machine without it raises, and there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvlp.so")

VLP_OK, VLP_EINVAL, VLP_EBUDGET, VLP_EHIP, VLP_EPARAM, VLP_EBUSY = 0, -1, -2, -3, -4, -5
VLP_AND, VLP_OR, VLP_NAND, VLP_XOR, VLP_XNOR, VLP_NOT, VLP_MUX = range(7)
VLP_INTV, VLP_COV, VLP_IDM = range(3)
STATUS_NAMES = {0: "VLP_OK", -1: "VLP_EINVAL", -2: "VLP_EBUDGET", -3: "VLP_EHIP", -4: "VLP_EPARAM", -5: "VLP_EBUSY"}
GATES = {"AND": VLP_AND, "OR": VLP_OR, "NAND": VLP_NAND, "XOR": VLP_XOR, "XNOR": VLP_XNOR, "NOT": VLP_NOT,
         "MUX": VLP_MUX}
MODES = {"intv": VLP_INTV, "cov": VLP_COV, "idm": VLP_IDM}

n, N = 630, 1024
CT_n, CT_N = n + 1, N + 1
MU = 1 << 29

# Every entry point of include/vlp.h.
EXPORTS = [
    "vlp_version", "vlp_default_params", "vlp_ctx_create", "vlp_ctx_destroy", "vlp_last_error", "vlp_mem_info",
    "vlp_keyset_load", "vlp_keyset_destroy", "vlp_bootstrap", "vlp_keyswitch", "vlp_gate", "vlp_gate_noalloc",
    "vlp_evaluate", "vlp_evaluate_ex", "vlp_server_encrypt",
    "vlp_program_create", "vlp_program_create_ex", "vlp_program_reset", "vlp_step", "vlp_program_run",
    "vlp_program_counts", "vlp_plan_counts", "vlp_plan_counts_ex", "vlp_plan_bytes", "vlp_plan_bytes_ex",
    "vlp_program_level_counts", "vlp_program_destroy", "vlp_get_tuning", "vlp_set_tuning", "vlp_sync",
    "vlp_profile_enable", "vlp_profile_read", "vlp_measure_modmul_peak",
]


class VlpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class vlp_params(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in ("n", "N", "k", "bg_bit", "ell", "ks_basebit", "ks_t")]


class vlp_shape(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("M", ctypes.c_uint32), ("l_I", ctypes.c_uint32),
                ("l_S", ctypes.c_uint32), ("d", ctypes.c_uint32)]


class vlp_circuit(ctypes.Structure):
    _fields_ = [("optimized", ctypes.c_uint32), ("agg_k", ctypes.c_uint32)]


class Query(ctypes.Structure):
    """A shape with the circuits that evaluate it (make_shape's result); the
    wrappers below pass it to the _ex entry points."""
    _fields_ = [("shape", vlp_shape), ("circuit", vlp_circuit)]


class vlp_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("items", ctypes.c_uint64), ("ms", ctypes.c_double)]


class vlp_tuning(ctypes.Structure):
    _fields_ = [("br_rotations_per_block", ctypes.c_uint32), ("br_blocks_per_cu", ctypes.c_uint32),
                ("ks_gates_per_block", ctypes.c_uint32), ("br_waves_per_rotation", ctypes.c_uint32)]


_lib = None


def lib():
    """The loaded libvlp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvlp.so is not built (run paper_2506_12761_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, u32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint64
        P = ctypes.POINTER
        sig = {
            "vlp_version": (ctypes.c_char_p, []),
            "vlp_default_params": (None, [P(vlp_params)]),
            "vlp_ctx_create": (ctypes.c_int, [P(vp), P(vlp_params), ctypes.c_int, vp, sz]),
            "vlp_ctx_destroy": (ctypes.c_int, [vp]),
            "vlp_last_error": (ctypes.c_char_p, [vp]),
            "vlp_mem_info": (ctypes.c_int, [vp, P(sz), P(sz)]),
            "vlp_keyset_load": (ctypes.c_int, [vp, vp, vp, P(vp)]),
            "vlp_keyset_destroy": (ctypes.c_int, [vp]),
            "vlp_bootstrap": (ctypes.c_int, [vp, vp, vp, vp, u32, sz]),
            "vlp_keyswitch": (ctypes.c_int, [vp, vp, vp, vp, sz]),
            "vlp_gate": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, vp, vp, vp, sz]),
            "vlp_gate_noalloc": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, vp, vp, vp, sz]),
            "vlp_evaluate": (ctypes.c_int, [vp, vp, P(vlp_shape), vp, vp, vp, vp, vp]),
            "vlp_evaluate_ex": (ctypes.c_int, [vp, vp, P(vlp_shape), P(vlp_circuit), vp, vp, vp, vp, vp]),
            "vlp_server_encrypt": (ctypes.c_int, [vp, P(vlp_shape), vp, vp, vp, vp, vp, vp]),
            "vlp_program_create": (ctypes.c_int, [vp, vp, P(vlp_shape), vp, vp, vp, vp, vp, P(vp)]),
            "vlp_program_create_ex": (ctypes.c_int, [vp, vp, P(vlp_shape), P(vlp_circuit), vp, vp, vp, vp, vp,
                                                     P(vp)]),
            "vlp_program_reset": (ctypes.c_int, [vp]),
            "vlp_step": (ctypes.c_int, [vp, P(vp), sz, P(sz)]),
            "vlp_program_run": (ctypes.c_int, [vp, vp, ctypes.c_int]),
            "vlp_program_counts": (ctypes.c_int, [vp, P(u64), P(u64), P(u64), P(u32)]),
            "vlp_plan_counts": (ctypes.c_int, [P(vlp_shape), P(u64), P(u64), P(u64), P(u32)]),
            "vlp_plan_counts_ex": (ctypes.c_int, [P(vlp_shape), P(vlp_circuit), P(u64), P(u64), P(u64), P(u32)]),
            "vlp_plan_bytes": (ctypes.c_int, [P(vlp_shape), ctypes.c_int, P(sz)]),
            "vlp_plan_bytes_ex": (ctypes.c_int, [P(vlp_shape), P(vlp_circuit), ctypes.c_int, P(sz)]),
            "vlp_program_level_counts": (ctypes.c_int, [vp, u32, P(u64), P(u64)]),
            "vlp_program_destroy": (ctypes.c_int, [vp]),
            "vlp_get_tuning": (ctypes.c_int, [vp, P(vlp_tuning)]),
            "vlp_set_tuning": (ctypes.c_int, [vp, P(vlp_tuning)]),
            "vlp_sync": (ctypes.c_int, [vp]),
            "vlp_profile_enable": (ctypes.c_int, [vp, ctypes.c_int]),
            "vlp_profile_read": (ctypes.c_int, [vp, P(vlp_kernel_stats), P(vlp_kernel_stats)]),
            "vlp_measure_modmul_peak": (ctypes.c_int, [ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double),
                                                       P(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    """Device pointer of a tensor (or None / an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("buffers must live on the HIP device")
    if not t.is_contiguous():
        raise ValueError("buffers must be contiguous")
    return t.data_ptr()


def _check(ctx, st):
    if st != VLP_OK:
        msg = lib().vlp_last_error(ctx)
        raise VlpError(st, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# One wrapper per C entry point (same names, same argument order).
# ---------------------------------------------------------------------------
def vlp_version() -> str:
    return lib().vlp_version().decode()


def vlp_default_params() -> vlp_params:
    p = vlp_params()
    lib().vlp_default_params(ctypes.byref(p))
    return p


def vlp_ctx_create(params: vlp_params | None = None, device: int = 0, hip_stream: int | None = None,
                   hbm_budget: int = 0):
    p = params or vlp_default_params()
    out = ctypes.c_void_p()
    _check(None, lib().vlp_ctx_create(ctypes.byref(out), ctypes.byref(p), device, hip_stream, hbm_budget))
    return out.value


def vlp_ctx_destroy(ctx) -> None:
    _check(ctx, lib().vlp_ctx_destroy(ctx))


def vlp_last_error(ctx) -> str:
    return (lib().vlp_last_error(ctx) or b"").decode()


def vlp_mem_info(ctx) -> tuple[int, int]:
    u, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(ctx, lib().vlp_mem_info(ctx, ctypes.byref(u), ctypes.byref(b)))
    return u.value, b.value


def vlp_keyset_load(ctx, bk_dev, ksk_dev):
    out = ctypes.c_void_p()
    _check(ctx, lib().vlp_keyset_load(ctx, _ptr(bk_dev), _ptr(ksk_dev), ctypes.byref(out)))
    return out.value


def vlp_keyset_destroy(ctx, ks) -> None:
    _check(ctx, lib().vlp_keyset_destroy(ks))


def vlp_bootstrap(ctx, ks, in_dev, out_dev, mu: int, B: int) -> None:
    _check(ctx, lib().vlp_bootstrap(ctx, ks, _ptr(in_dev), _ptr(out_dev), mu, B))


def vlp_keyswitch(ctx, ks, in_dev, out_dev, B: int) -> None:
    _check(ctx, lib().vlp_keyswitch(ctx, ks, _ptr(in_dev), _ptr(out_dev), B))


def vlp_gate(ctx, ks, op, a_dev, b_dev, c_dev, out_dev, B: int) -> None:
    if isinstance(op, str):
        op = GATES[op]
    _check(ctx, lib().vlp_gate(ctx, ks, op, _ptr(a_dev), _ptr(b_dev), _ptr(c_dev), _ptr(out_dev), B))


def vlp_gate_noalloc(ctx, ks, op, a_dev, b_dev, c_dev, out_dev, B: int) -> None:
    if isinstance(op, str):
        op = GATES[op]
    _check(ctx, lib().vlp_gate_noalloc(ctx, ks, op, _ptr(a_dev), _ptr(b_dev), _ptr(c_dev), _ptr(out_dev), B))


def make_shape(mode, M, l_I, l_S=0, d=2, optimized=True, agg_k=0) -> Query:
    if isinstance(mode, str):
        mode = MODES[mode]
    return Query(vlp_shape(mode, M, l_I, l_S, d), vlp_circuit(1 if optimized else 0, agg_k))


def _split(shape):
    """(vlp_shape, vlp_circuit or None) of a vlp_shape or a Query."""
    if isinstance(shape, Query):
        return shape.shape, shape.circuit
    return shape, None


def vlp_evaluate(ctx, ks, shape, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev) -> None:
    s, c = _split(shape)
    if c is not None:
        return vlp_evaluate_ex(ctx, ks, s, c, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev)
    _check(ctx, lib().vlp_evaluate(ctx, ks, ctypes.byref(s), _ptr(query_dev), _ptr(db_loc_dev),
                                   _ptr(db_pay_dev), _ptr(R_dev), _ptr(v_out_dev)))


def vlp_evaluate_ex(ctx, ks, shape: vlp_shape, circuit: vlp_circuit | None, query_dev, db_loc_dev, db_pay_dev,
                    R_dev, v_out_dev) -> None:
    _check(ctx, lib().vlp_evaluate_ex(ctx, ks, ctypes.byref(shape), ctypes.byref(circuit) if circuit else None,
                                      _ptr(query_dev), _ptr(db_loc_dev), _ptr(db_pay_dev), _ptr(R_dev),
                                      _ptr(v_out_dev)))


def vlp_server_encrypt(ctx, shape, pk_loc_dev, pk_pay_dev, loc_dev, pay_dev, out_loc_dev, out_pay_dev) -> None:
    s = _split(shape)[0]
    _check(ctx, lib().vlp_server_encrypt(ctx, ctypes.byref(s), _ptr(pk_loc_dev), _ptr(pk_pay_dev), _ptr(loc_dev),
                                         _ptr(pay_dev), _ptr(out_loc_dev), _ptr(out_pay_dev)))


def vlp_program_create(ctx, ks, shape, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev):
    s, c = _split(shape)
    if c is not None:
        return vlp_program_create_ex(ctx, ks, s, c, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev)
    out = ctypes.c_void_p()
    _check(ctx, lib().vlp_program_create(ctx, ks, ctypes.byref(s), _ptr(query_dev), _ptr(db_loc_dev),
                                         _ptr(db_pay_dev), _ptr(R_dev), _ptr(v_out_dev), ctypes.byref(out)))
    return out.value


def vlp_program_create_ex(ctx, ks, shape: vlp_shape, circuit: vlp_circuit | None, query_dev, db_loc_dev,
                          db_pay_dev, R_dev, v_out_dev):
    out = ctypes.c_void_p()
    _check(ctx, lib().vlp_program_create_ex(ctx, ks, ctypes.byref(shape), ctypes.byref(circuit) if circuit else None,
                                            _ptr(query_dev), _ptr(db_loc_dev), _ptr(db_pay_dev), _ptr(R_dev),
                                            _ptr(v_out_dev), ctypes.byref(out)))
    return out.value


def vlp_program_reset(ctx, prog) -> None:
    _check(ctx, lib().vlp_program_reset(prog))


def vlp_step(ctx, progs) -> int:
    arr = (ctypes.c_void_p * max(1, len(progs)))(*progs)
    rem = ctypes.c_size_t()
    _check(ctx, lib().vlp_step(ctx, arr, len(progs), ctypes.byref(rem)))
    return rem.value


def vlp_program_run(ctx, prog, use_graph: bool = False) -> None:
    _check(ctx, lib().vlp_program_run(ctx, prog, 1 if use_graph else 0))


def vlp_program_counts(ctx, prog) -> dict:
    g, b, k, l = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
    _check(ctx, lib().vlp_program_counts(prog, ctypes.byref(g), ctypes.byref(b), ctypes.byref(k), ctypes.byref(l)))
    return {"gates": g.value, "blind_rotations": b.value, "key_switches": k.value, "levels": l.value}


def vlp_plan_counts(shape) -> dict:
    s, c = _split(shape)
    if c is not None:
        return vlp_plan_counts_ex(s, c)
    g, b, k, l = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
    st = lib().vlp_plan_counts(ctypes.byref(s), ctypes.byref(g), ctypes.byref(b), ctypes.byref(k), ctypes.byref(l))
    if st != VLP_OK:
        raise VlpError(st, "bad shape")
    return {"gates": g.value, "blind_rotations": b.value, "key_switches": k.value, "levels": l.value}


def vlp_plan_counts_ex(shape: vlp_shape, circuit: vlp_circuit | None) -> dict:
    g, b, k, l = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
    st = lib().vlp_plan_counts_ex(ctypes.byref(shape), ctypes.byref(circuit) if circuit else None, ctypes.byref(g),
                                  ctypes.byref(b), ctypes.byref(k), ctypes.byref(l))
    if st != VLP_OK:
        raise VlpError(st, "bad shape or circuit")
    return {"gates": g.value, "blind_rotations": b.value, "key_switches": k.value, "levels": l.value}


def vlp_plan_bytes(shape, with_v_out: bool = True) -> int:
    s, c = _split(shape)
    if c is not None:
        return vlp_plan_bytes_ex(s, c, with_v_out)
    b = ctypes.c_size_t()
    st = lib().vlp_plan_bytes(ctypes.byref(s), 1 if with_v_out else 0, ctypes.byref(b))
    if st != VLP_OK:
        raise VlpError(st, "bad shape")
    return b.value


def vlp_plan_bytes_ex(shape: vlp_shape, circuit: vlp_circuit | None, with_v_out: bool = True) -> int:
    b = ctypes.c_size_t()
    st = lib().vlp_plan_bytes_ex(ctypes.byref(shape), ctypes.byref(circuit) if circuit else None,
                                 1 if with_v_out else 0, ctypes.byref(b))
    if st != VLP_OK:
        raise VlpError(st, "bad shape or circuit")
    return b.value


def vlp_program_level_counts(ctx, prog, level: int) -> dict:
    b, k = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, lib().vlp_program_level_counts(prog, level, ctypes.byref(b), ctypes.byref(k)))
    return {"blind_rotations": b.value, "key_switches": k.value}


def vlp_program_destroy(ctx, prog) -> None:
    _check(ctx, lib().vlp_program_destroy(prog))


def vlp_get_tuning(ctx) -> vlp_tuning:
    t = vlp_tuning()
    _check(ctx, lib().vlp_get_tuning(ctx, ctypes.byref(t)))
    return t


def vlp_set_tuning(ctx, br_rotations_per_block: int, br_blocks_per_cu: int, ks_gates_per_block: int,
                   br_waves_per_rotation: int = 0) -> None:
    t = vlp_tuning(br_rotations_per_block, br_blocks_per_cu, ks_gates_per_block, br_waves_per_rotation)
    _check(ctx, lib().vlp_set_tuning(ctx, ctypes.byref(t)))


def vlp_sync(ctx) -> None:
    _check(ctx, lib().vlp_sync(ctx))


def vlp_profile_enable(ctx, enable: bool = True) -> None:
    _check(ctx, lib().vlp_profile_enable(ctx, 1 if enable else 0))


def vlp_profile_read(ctx) -> dict:
    br, ks = vlp_kernel_stats(), vlp_kernel_stats()
    _check(ctx, lib().vlp_profile_read(ctx, ctypes.byref(br), ctypes.byref(ks)))
    return {"br": {"launches": br.launches, "items": br.items, "ms": br.ms},
            "ks": {"launches": ks.launches, "items": ks.items, "ms": ks.ms}}


def vlp_measure_modmul_peak(device: int = 0) -> dict:
    """Measured butterfly rates of `device` (modular multiplications per second)."""
    f, i, m = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib().vlp_measure_modmul_peak(device, ctypes.byref(f), ctypes.byref(i), ctypes.byref(m))
    if st != VLP_OK:
        raise VlpError(st, "vlp_measure_modmul_peak failed")
    return {"fwd": f.value, "inv": i.value, "mixed": m.value}


# ---------------------------------------------------------------------------
# Convenience: a context object owning its keysets (torch memory and streams).
# ---------------------------------------------------------------------------
class Context:
    """Context on cuda:<device> with its own torch stream (default priority).

    The library runs on that stream; the helpers below allocate, fill and read
    tensors on the same stream, so their work is ordered with the library's."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.ctx = vlp_ctx_create(None, device, self.stream.cuda_stream, hbm_budget)
        self._keysets = []

    def close(self):
        if self.ctx:
            for ks in self._keysets:
                vlp_keyset_destroy(self.ctx, ks)
            self._keysets = []
            vlp_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def tensor(self, arr):
        """Host array of uint32 words -> int32 tensor on the device."""
        import numpy as np
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint32)).view(np.int32)
        with self.torch.cuda.stream(self.stream):
            t = self.torch.from_numpy(a).to(self.device)
        self.stream.synchronize()
        return t

    def array(self, arr):
        """Host array of any fixed-width dtype -> tensor on the device with the
        same bytes (uint64 travels as int64, uint32 as int32)."""
        import numpy as np
        a = np.ascontiguousarray(arr)
        if a.dtype == np.uint64:
            a = a.view(np.int64)
        elif a.dtype == np.uint32:
            a = a.view(np.int32)
        with self.torch.cuda.stream(self.stream):
            t = self.torch.from_numpy(a).to(self.device)
        self.stream.synchronize()
        return t

    def empty(self, *shape):
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(shape, dtype=self.torch.int32, device=self.device)

    def zero(self, t):
        with self.torch.cuda.stream(self.stream):
            t.zero_()

    def to_host(self, t):
        import numpy as np
        self.stream.synchronize()
        return t.cpu().numpy().view(np.uint32)

    def load_keys(self, bk, ksk):
        """Host or device bk [630][6][2][1024] and ksk [1024][8][4][631] -> keyset handle."""
        bk_t = bk if hasattr(bk, "is_cuda") else self.tensor(bk)
        ksk_t = ksk if hasattr(ksk, "is_cuda") else self.tensor(ksk)
        ks = vlp_keyset_load(self.ctx, bk_t, ksk_t)
        vlp_sync(self.ctx)
        self._keysets.append(ks)
        return ks

    def drop_keys(self, ks):
        vlp_keyset_destroy(self.ctx, ks)
        self._keysets.remove(ks)

    def sync(self):
        vlp_sync(self.ctx)
