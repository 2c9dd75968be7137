"""ctypes binding of the C ABI declared in include/tn.h.

Argument marshalling only: every step of the estimate runs in the HIP library
(libtn_gfx950.so).  PyTorch supplies device memory (the workspace) and the
stream.  The library must have been built (paper_2211_17028_amd/build.py);
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtn_gfx950.so")

TN_OK, TN_EINVAL, TN_ENOTCPTP, TN_EUNSUPPORTED, TN_EDEGENERATE = 0, -1, -2, -3, -4
TN_ENOMEM, TN_EHIP, TN_ETOOBIG, TN_ESTATE = -5, -6, -7, -8
TN_GATE, TN_NOISE = 0, 1
TN_STATE_PRODUCT, TN_STATE_CIRCUIT_OUTPUT, TN_STATE_DENSE = 0, 1, 2
TN_STATE_SUM2, TN_STATE_CIRCUIT_OUTPUT_SUM2 = 3, 4
TN_MODE_BATCHED, TN_MODE_PLAIN = 0, 1
TN_MAX_LEVEL = 8

ERROR_NAMES = {0: "TN_OK", -1: "TN_EINVAL", -2: "TN_ENOTCPTP", -3: "TN_EUNSUPPORTED",
               -4: "TN_EDEGENERATE", -5: "TN_ENOMEM", -6: "TN_EHIP", -7: "TN_ETOOBIG",
               -8: "TN_ESTATE"}


class tn_c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class tn_op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nq", C.c_int32), ("q", C.c_int32 * 2),
                ("n_kraus", C.c_int32), ("mat", C.POINTER(tn_c128))]


class tn_circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_ops", C.c_int64), ("ops", C.POINTER(tn_op))]


class tn_state(C.Structure):
    _fields_ = [("kind", C.c_int32), ("data", C.POINTER(tn_c128))]


class tn_plan_opts(C.Structure):
    _fields_ = [("path_trials", C.c_int32), ("seed", C.c_uint64), ("no_light_cone", C.c_int32),
                ("max_log_size", C.c_int32), ("no_diagonal_hyperedges", C.c_int32),
                ("max_work_bytes", C.c_double), ("no_reconfigure", C.c_int32)]


class tn_prune_opts(C.Structure):
    _fields_ = [("min_level", C.c_int32), ("keep", C.POINTER(C.c_uint8)), ("n_keep", C.c_int64)]


class tn_exec_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("use_graph", C.c_int32), ("fp64_level0", C.c_int32),
                ("tune", C.c_int32), ("time_kernels", C.c_int32), ("no_gather", C.c_int32),
                ("no_group", C.c_int32), ("max_ksplit", C.c_int32), ("mixed_shapes", C.c_int32),
                ("all_tiles", C.c_int32)]


class tn_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


class tn_result(C.Structure):
    _fields_ = [("level", C.c_int32), ("clamped", C.c_int32), ("n_terms", C.c_int64),
                ("n_contracted", C.c_int64), ("n_zero_weight", C.c_int64),
                ("level_sum", C.c_double * (TN_MAX_LEVEL + 1)),
                ("level_comp", C.c_double * (TN_MAX_LEVEL + 1)),
                ("A", C.c_double * (TN_MAX_LEVEL + 1)), ("bound", C.c_double),
                ("x0_fp32", C.c_double)]

    def as_dict(self):
        L = self.level
        return {"level": L, "clamped": bool(self.clamped), "n_terms": self.n_terms,
                "n_contracted": self.n_contracted, "n_zero_weight": self.n_zero_weight,
                "T": [self.level_sum[u] for u in range(L + 1)],
                "A": [self.A[u] for u in range(L + 1)], "bound": self.bound,
                "x0_fp32": self.x0_fp32}


class tn_plan_info(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_noise", C.c_int32), ("level", C.c_int32),
                ("clamped", C.c_int32), ("n_clusters", C.c_int32), ("n_leaves", C.c_int32),
                ("max_log_size", C.c_int32), ("flops_per_term", C.c_double),
                ("doubled", C.c_int32), ("n_channels", C.c_int32)]


EXPORTS = [
    "tn_plan_build", "tn_plan_build_doubled", "tn_polarization_combine", "tn_terms_enumerate",
    "tn_terms_enumerate_factored", "tn_terms_groups", "tn_factored_levels",
    "tn_plan_build_trajectories", "tn_terms_trajectories", "tn_exec_submit", "tn_exec_collect", "tn_exec_run_many", "tn_terms_get", "tn_exec_prepare", "tn_exec_run",
    "tn_exec_outputs", "tn_exec_timing", "tn_contract_batch", "tn_estimate", "tn_plan_workspace",
    "tn_release_cached", "tn_estimate_noalloc",
    "tn_plan_get_info", "tn_plan_noise", "tn_plan_describe", "tn_exec_describe",
    "tn_exec_const_bytes", "tn_exec_copy_outputs", "tn_exec_kernel_stats", "tn_plan_destroy", "tn_terms_destroy", "tn_exec_destroy", "tn_last_error",
]

_lib = None


class TNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2211_17028_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.tn_plan_build.argtypes = [C.POINTER(tn_circuit), C.POINTER(tn_state), C.POINTER(tn_state),
                                C.c_int32, C.POINTER(tn_plan_opts), C.POINTER(vp)]
    L.tn_plan_build_doubled.argtypes = [C.POINTER(tn_circuit), C.POINTER(tn_state), C.POINTER(tn_state),
                                        C.POINTER(tn_plan_opts), C.POINTER(vp)]
    L.tn_polarization_combine.argtypes = [C.POINTER(tn_result), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.tn_terms_enumerate_factored.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int32)]
    L.tn_terms_groups.argtypes = [vp, vp, vp, vp]
    L.tn_plan_build_trajectories.argtypes = [C.POINTER(tn_circuit), C.POINTER(tn_state), C.POINTER(tn_state),
                                             C.POINTER(tn_plan_opts), C.POINTER(vp)]
    L.tn_terms_trajectories.argtypes = [vp, C.c_int64, vp, C.POINTER(vp), C.POINTER(C.c_int64)]
    L.tn_factored_levels.argtypes = [vp, vp, vp]
    L.tn_terms_enumerate.argtypes = [vp, C.c_int32, C.POINTER(tn_prune_opts), C.POINTER(vp),
                                     C.POINTER(C.c_int64)]
    L.tn_terms_get.argtypes = [vp, vp, vp]
    L.tn_exec_prepare.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), C.POINTER(tn_exec_opts),
                                  vp, C.c_size_t, vp, C.POINTER(C.c_size_t), C.POINTER(vp)]
    L.tn_exec_run.argtypes = [vp, vp, C.POINTER(tn_result)]
    L.tn_exec_submit.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    L.tn_exec_collect.argtypes = [vp, C.c_int64, C.POINTER(tn_result)]
    L.tn_exec_run_many.argtypes = [vp, vp, C.c_int64, C.POINTER(tn_result)]
    L.tn_exec_outputs.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64)]
    L.tn_exec_timing.argtypes = [vp] + [C.POINTER(C.c_double)] * 4
    L.tn_contract_batch.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), C.c_int64, C.c_int64,
                                    vp, vp, C.c_size_t, vp]
    L.tn_estimate.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), vp, C.c_size_t, vp,
                              C.POINTER(tn_result)]
    L.tn_plan_workspace.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_size_t),
                                    C.POINTER(C.c_size_t)]
    L.tn_release_cached.argtypes = []
    L.tn_release_cached.restype = None
    L.tn_estimate_noalloc.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), vp, C.POINTER(tn_result)]
    L.tn_plan_get_info.argtypes = [vp, C.POINTER(tn_plan_info)]
    L.tn_plan_noise.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(tn_c128),
                                C.POINTER(C.c_double)]
    L.tn_plan_describe.argtypes = [vp, C.c_char_p, C.POINTER(C.c_size_t)]
    L.tn_exec_describe.argtypes = [vp, C.c_char_p, C.POINTER(C.c_size_t)]
    L.tn_exec_const_bytes.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.tn_exec_copy_outputs.argtypes = [vp, C.c_int32, vp, vp]
    L.tn_exec_kernel_stats.argtypes = [vp, C.c_int32, C.POINTER(tn_kernel_stat), C.POINTER(C.c_int32),
                                       C.c_int32]
    L.tn_plan_destroy.argtypes = [vp]
    L.tn_terms_destroy.argtypes = [vp]
    L.tn_exec_destroy.argtypes = [vp]
    L.tn_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("tn_plan_destroy", "tn_terms_destroy", "tn_exec_destroy", "tn_last_error"):
            getattr(L, name).restype = C.c_int
        else:
            if name != "tn_last_error":
                getattr(L, name).restype = None
    _lib = L
    return L


def _check(rc):
    if rc != TN_OK:
        msg = lib().tn_last_error()
        raise TNError(rc, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# circuit marshalling
# ---------------------------------------------------------------------------
class _CircuitBuffers:
    """Keeps the ctypes arrays of one circuit alive while a call uses them."""

    def __init__(self, circ):
        mats = []
        ops = (tn_op * max(1, len(circ.ops)))()
        offsets = []
        off = 0
        for op in circ.ops:
            if op.kind == "gate":
                m = np.ascontiguousarray(op.mat, dtype=np.complex128).reshape(-1)
                nk = 0
            else:
                m = np.concatenate([np.ascontiguousarray(k, dtype=np.complex128).reshape(-1)
                                    for k in op.kraus])
                nk = len(op.kraus)
            mats.append(m)
            offsets.append((off, nk))
            off += m.size
        self.mat = np.ascontiguousarray(np.concatenate(mats) if mats else np.zeros(1, np.complex128))
        base = self.mat.ctypes.data
        for i, op in enumerate(circ.ops):
            o = ops[i]
            o.kind = TN_GATE if op.kind == "gate" else TN_NOISE
            o.nq = len(op.qubits)
            o.q[0] = int(op.qubits[0])
            o.q[1] = int(op.qubits[1]) if len(op.qubits) > 1 else -1
            o.n_kraus = offsets[i][1]
            o.mat = C.cast(base + 16 * offsets[i][0], C.POINTER(tn_c128))
        self.ops = ops
        self.circ = tn_circuit(circ.n_qubits, len(circ.ops), C.cast(ops, C.POINTER(tn_op)))
        self.psi_arr = np.ascontiguousarray(circ.psi, dtype=np.complex128).reshape(-1)
        self.v_arr = np.ascontiguousarray(circ.v, dtype=np.complex128).reshape(-1)
        kind = {"product": TN_STATE_PRODUCT, "circuit_output": TN_STATE_CIRCUIT_OUTPUT,
                "dense": TN_STATE_DENSE, "sum2": TN_STATE_SUM2,
                "circuit_output_sum2": TN_STATE_CIRCUIT_OUTPUT_SUM2}[circ.target]
        self.psi = tn_state(TN_STATE_PRODUCT, C.cast(self.psi_arr.ctypes.data, C.POINTER(tn_c128)))
        self.v = tn_state(kind, C.cast(self.v_arr.ctypes.data, C.POINTER(tn_c128)))


class Plan:
    def __init__(self, handle, circ):
        self.handle = handle
        self.circ = circ

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tn_plan_destroy(self.handle)
            self.handle = None

    def info(self):
        inf = tn_plan_info()
        _check(lib().tn_plan_get_info(self.handle, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in tn_plan_info._fields_}

    def noise(self, s):
        d = (C.c_double * 4)()
        k = (tn_c128 * 16)()
        rate = C.c_double()
        _check(lib().tn_plan_noise(self.handle, s, d, k, C.byref(rate)))
        kk = np.array([complex(x.re, x.im) for x in k]).reshape(4, 2, 2)
        return np.array(list(d)), kk, rate.value

    def describe(self):
        n = C.c_size_t(0)
        _check(lib().tn_plan_describe(self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().tn_plan_describe(self.handle, buf, C.byref(n)))
        return json.loads(buf.value.decode())


class Terms:
    def __init__(self, handle, plan, n):
        self.handle = handle
        self.plan = plan
        self.n = n

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tn_terms_destroy(self.handle)
            self.handle = None

    def get(self):
        N = self.plan.circ.n_noises
        pat = np.zeros((self.n, N), dtype=np.int8)
        w = np.zeros(self.n, dtype=np.float64)
        _check(lib().tn_terms_get(self.handle, pat.ctypes.data if N else None, w.ctypes.data))
        return pat, w


def tn_plan_build(circ, level: Optional[int] = None, path_trials: int = 0, seed: int = 0,
                  light_cone: bool = True, max_log_size: int = 0, diagonal_hyperedges: bool = True,
                  max_work_bytes: float = 0.0, reconfigure: bool = True) -> Plan:
    bufs = _CircuitBuffers(circ)
    opts = tn_plan_opts(path_trials, seed, 0 if light_cone else 1, max_log_size,
                        0 if diagonal_hyperedges else 1, max_work_bytes, 0 if reconfigure else 1)
    h = C.c_void_p()
    lev = circ.level if level is None else level
    _check(lib().tn_plan_build(C.byref(bufs.circ), C.byref(bufs.psi), C.byref(bufs.v), lev,
                               C.byref(opts), C.byref(h)))
    return Plan(h, circ)


def tn_plan_build_doubled(circ, path_trials: int = 0, seed: int = 0, light_cone: bool = True,
                          max_log_size: int = 0, diagonal_hyperedges: bool = True,
                          max_work_bytes: float = 0.0, reconfigure: bool = True) -> Plan:
    """Plan of the doubled network: its one term's estimate is the exact value."""
    bufs = _CircuitBuffers(circ)
    opts = tn_plan_opts(path_trials, seed, 0 if light_cone else 1, max_log_size,
                        0 if diagonal_hyperedges else 1, max_work_bytes, 0 if reconfigure else 1)
    h = C.c_void_p()
    _check(lib().tn_plan_build_doubled(C.byref(bufs.circ), C.byref(bufs.psi), C.byref(bufs.v),
                                       C.byref(opts), C.byref(h)))
    return Plan(h, circ)


def tn_terms_enumerate(plan: Plan, level: int, keep: Optional[np.ndarray] = None,
                       min_level: int = 2) -> Terms:
    h = C.c_void_p()
    n = C.c_int64()
    if keep is None:
        _check(lib().tn_terms_enumerate(plan.handle, level, None, C.byref(h), C.byref(n)))
    else:
        k = np.ascontiguousarray(keep, dtype=np.uint8)
        po = tn_prune_opts(min_level, C.cast(k.ctypes.data, C.POINTER(C.c_uint8)), k.size)
        _check(lib().tn_terms_enumerate(plan.handle, level, C.byref(po), C.byref(h), C.byref(n)))
    return Terms(h, plan, n.value)


def _handles(objs):
    arr = (C.c_void_p * len(objs))()
    for i, o in enumerate(objs):
        arr[i] = o.handle
    return arr


class Exec:
    def __init__(self, handle, plans, terms, ws, need):
        self.handle = handle
        self.plans = plans
        self.terms = terms
        self.ws = ws
        self.need = need

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tn_exec_destroy(self.handle)
            self.handle = None

    def run(self, stream=None) -> List[dict]:
        return [r.as_dict() for r in self.run_raw(stream)]

    def submit(self, stream=None) -> int:
        """Issue one estimate without waiting; returns its ticket."""
        t = C.c_int64()
        _check(lib().tn_exec_submit(self.handle, _stream_ptr(stream), C.byref(t)))
        return t.value

    def collect(self, ticket: int) -> List[dict]:
        """Wait for a submitted estimate (in submission order) and return its results."""
        res = (tn_result * len(self.plans))()
        _check(lib().tn_exec_collect(self.handle, ticket, res))
        return [r.as_dict() for r in res]

    def run_many_raw(self, count: int, stream=None):
        """tn_result array of `count` estimates issued in one call (two in
        flight), estimate-major: entry i * n_plans + p."""
        res = (tn_result * max(1, count * len(self.plans)))()
        _check(lib().tn_exec_run_many(self.handle, _stream_ptr(stream), count, res))
        return res

    def run_many(self, count: int, stream=None) -> List[List[dict]]:
        """Results of `count` estimates issued in one call, one list per estimate."""
        raw = self.run_many_raw(count, stream)
        n = len(self.plans)
        return [[raw[i * n + p].as_dict() for p in range(n)] for i in range(count)]

    def run_raw(self, stream=None):
        """tn_result array of one run (one entry per plan)."""
        res = (tn_result * len(self.plans))()
        _check(lib().tn_exec_run(self.handle, _stream_ptr(stream), res))
        return res

    def kernel_stats(self, reset=False):
        """{kernel name: dict(launches, ms, flops, bytes)} accumulated over runs."""
        n = C.c_int32()
        _check(lib().tn_exec_kernel_stats(self.handle, 0, None, C.byref(n), 0))
        arr = (tn_kernel_stat * max(1, n.value))()
        _check(lib().tn_exec_kernel_stats(self.handle, n.value, arr, C.byref(n), 1 if reset else 0))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms,
                                       "flops": arr[i].flops, "bytes": arr[i].bytes}
                for i in range(n.value)}

    def timing(self):
        v = [C.c_double() for _ in range(4)]
        _check(lib().tn_exec_timing(self.handle, *[C.byref(x) for x in v]))
        return [x.value for x in v]

    def outputs(self):
        dx, da, n = C.c_void_p(), C.c_void_p(), C.c_int64()
        _check(lib().tn_exec_outputs(self.handle, C.byref(dx), C.byref(da), C.byref(n)))
        return dx.value, da.value, n.value

    def describe(self):
        return exec_describe(self.handle)

    def values(self, plan=0):
        """(X_t float64, a_t complex64) of packed plan `plan`, on the host."""
        n = self.terms[plan].n
        x = np.zeros(max(1, n), dtype=np.float64)
        a = np.zeros(max(1, n), dtype=np.complex64)
        _check(lib().tn_exec_copy_outputs(self.handle, plan, x.ctypes.data, a.ctypes.data))
        return x[:n], a[:n]


def exec_describe(handle):
    n = C.c_size_t(0)
    _check(lib().tn_exec_describe(handle, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().tn_exec_describe(handle, buf, C.byref(n)))
    return json.loads(buf.value.decode())


def exec_const_bytes(handle):
    n = C.c_size_t(0)
    _check(lib().tn_exec_const_bytes(handle, None, C.byref(n)))
    buf = np.zeros(n.value, dtype=np.uint8)
    _check(lib().tn_exec_const_bytes(handle, buf.ctypes.data, C.byref(n)))
    return buf


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def exec_opts(mode=TN_MODE_BATCHED, use_graph=False, fp64_level0=True, tune=False, time_kernels=False,
              gather=True, group=True, max_ksplit=0, one_shape_per_level=True, all_tiles=False):
    return tn_exec_opts(mode, 1 if use_graph else 0, 1 if fp64_level0 else 0, 1 if tune else 0,
                        1 if time_kernels else 0, 0 if gather else 1, 0 if group else 1, int(max_ksplit),
                        0 if one_shape_per_level else 1, 1 if all_tiles else 0)


def tn_exec_describe_only(plans: Sequence[Plan], terms: Sequence[Terms], opts=None):
    """Schedule without device memory: (description, staged constants)."""
    o = opts or exec_opts()
    need = C.c_size_t()
    h = C.c_void_p()
    _check(lib().tn_exec_prepare(len(plans), _handles(plans), _handles(terms), C.byref(o), None, 0,
                                 None, C.byref(need), C.byref(h)))
    try:
        return exec_describe(h), exec_const_bytes(h)
    finally:
        lib().tn_exec_destroy(h)


def tn_exec_prepare(plans: Sequence[Plan], terms: Sequence[Terms], opts=None, stream=None) -> Exec:
    """Allocate the workspace with torch on the current device and prepare."""
    import torch
    o = opts or exec_opts()
    need = C.c_size_t()
    _check(lib().tn_exec_prepare(len(plans), _handles(plans), _handles(terms), C.byref(o), None, 0,
                                 None, C.byref(need), None))
    ws = torch.empty(max(256, need.value), dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    _check(lib().tn_exec_prepare(len(plans), _handles(plans), _handles(terms), C.byref(o),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream),
                                 C.byref(need), C.byref(h)))
    return Exec(h, list(plans), list(terms), ws, need.value)


def tn_plan_build_trajectories(circ, path_trials: int = 0, seed: int = 0, light_cone: bool = True,
                               max_log_size: int = 0, diagonal_hyperedges: bool = True,
                               max_work_bytes: float = 0.0, reconfigure: bool = True) -> Plan:
    """Plan whose slots are the Kraus operators E_k / sqrt(q_k) (quantum trajectories)."""
    bufs = _CircuitBuffers(circ)
    opts = tn_plan_opts(path_trials, seed, 0 if light_cone else 1, max_log_size,
                        0 if diagonal_hyperedges else 1, max_work_bytes, 0 if reconfigure else 1)
    h = C.c_void_p()
    _check(lib().tn_plan_build_trajectories(C.byref(bufs.circ), C.byref(bufs.psi), C.byref(bufs.v),
                                            C.byref(opts), C.byref(h)))
    return Plan(h, circ)


def tn_terms_trajectories(plan: Plan, uniforms: np.ndarray) -> Terms:
    """Sampled terms from (n_samples, n_noise) uniforms in [0, 1)."""
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    h = C.c_void_p()
    n = C.c_int64()
    _check(lib().tn_terms_trajectories(plan.handle, u.shape[0], u.ctypes.data, C.byref(h), C.byref(n)))
    return Terms(h, plan, n.value)


def trajectories_estimate(circ, uniforms: np.ndarray, opts=None, plan_kw=None):
    """(sample mean, per-sample X, exec) of the quantum-trajectories estimate."""
    plan = tn_plan_build_trajectories(circ, **(plan_kw or {}))
    terms = tn_terms_trajectories(plan, uniforms)
    ex = tn_exec_prepare([plan], [terms], opts or exec_opts())
    res = ex.run()[0]
    x, _ = ex.values()                 # w X with w = 1 / n_samples
    return res["A"][0], x * terms.n, ex


def tn_terms_enumerate_factored(plan: Plan, level: int) -> Terms:
    """Terms with corrections inside one cluster, grouped by (level, cluster);
    ``.groups`` = (starts, level, cluster) arrays."""
    h = C.c_void_p()
    n = C.c_int64()
    ng = C.c_int32()
    _check(lib().tn_terms_enumerate_factored(plan.handle, level, C.byref(h), C.byref(n), C.byref(ng)))
    t = Terms(h, plan, n.value)
    starts = np.zeros(ng.value + 1, dtype=np.int64)
    lv = np.zeros(ng.value, dtype=np.int32)
    cl = np.zeros(ng.value, dtype=np.int32)
    _check(lib().tn_terms_groups(h, starts.ctypes.data, lv.ctypes.data, cl.ctypes.data))
    t.groups = (starts, lv, cl)
    return t


def kernel_group_sums(d_x, d_starts, n_groups, d_out, stream=None):
    """Deterministic FP64 sums of d_x over [d_starts[g], d_starts[g+1]) into
    d_out[2g] (sum) and d_out[2g+1] (compensation); device pointers."""
    _check(_kernel_lib().tn_kernel_group_sums(C.c_void_p(d_x), C.c_void_p(d_starts), n_groups,
                                              C.c_void_p(d_out), _stream_ptr(stream)))


class FactoredEstimate:
    """A(0..level) by exact cross-term reuse over independent clusters: the
    factored term set through the prepared schedule, per-group sums on the
    device, the per-cluster level polynomials combined on the host."""

    def __init__(self, circ, level: Optional[int] = None, opts=None, plan_kw=None):
        import torch
        lev = circ.level if level is None else level
        self.plan = tn_plan_build(circ, lev, **(plan_kw or {}))
        self.terms = tn_terms_enumerate_factored(self.plan, lev)
        self.ex = tn_exec_prepare([self.plan], [self.terms], opts or exec_opts())
        starts = self.terms.groups[0]
        self.n_groups = len(starts) - 1
        self.d_starts = torch.from_numpy(starts).cuda()
        self.d_sums = torch.zeros(2 * max(1, self.n_groups), dtype=torch.float64, device="cuda")
        self.h_sums = torch.zeros(2 * max(1, self.n_groups), dtype=torch.float64).pin_memory()

    def run(self):
        """(A(0..level), the exec's result dict) of one estimate on the current stream."""
        stream = None
        res = self.ex.run(stream)[0]
        d_x, _, _ = self.ex.outputs()
        kernel_group_sums(d_x, self.d_starts.data_ptr(), self.n_groups, self.d_sums.data_ptr(), stream)
        self.h_sums.copy_(self.d_sums)
        h = np.ascontiguousarray(self.h_sums.numpy()[0::2])
        A = np.zeros(res["level"] + 1, dtype=np.float64)
        _check(lib().tn_factored_levels(self.terms.handle, h.ctypes.data, A.ctypes.data))
        return A, res


def polarization_circuits(circ, x, y, output: bool = True):
    """The four circuits of <x| E |y>: targets v_k = y + i^k x (bond-2 states;
    with ``output`` the circuit's ideal outputs of them), k = 0..3."""
    import dataclasses
    out = []
    for k in range(4):
        flat = np.concatenate([np.asarray(y, dtype=np.complex128).reshape(-1),
                               np.asarray(x, dtype=np.complex128).reshape(-1), [1j ** k]])
        out.append(dataclasses.replace(circ, target="circuit_output_sum2" if output else "sum2", v=flat))
    return out


def offdiagonal(circ, x, y, level: Optional[int] = None, output: bool = True, exact: bool = False,
                opts=None, plan_kw=None):
    """<x| E(|psi><psi|) |y> for product states x, y (n x 2; with ``output`` the
    circuit's ideal outputs of them).  Four estimates with the bond-2 targets of
    the polarization identity run as one packed schedule; tn_polarization_combine
    gives A_xy(u), u = 0..level, as a complex array.  ``exact`` uses the four
    doubled networks instead (one value, the exact element).  Returns
    (A_xy, the four result dicts, the exec)."""
    lev = circ.level if level is None else level
    circs = polarization_circuits(circ, x, y, output)
    kw = plan_kw or {}
    if exact:
        plans = [tn_plan_build_doubled(c, **kw) for c in circs]
        terms = [tn_terms_enumerate(p, 0) for p in plans]
    else:
        plans = [tn_plan_build(c, lev, **kw) for c in circs]
        terms = [tn_terms_enumerate(p, lev) for p in plans]
    ex = tn_exec_prepare(plans, terms, opts or exec_opts())
    raw = ex.run_raw()
    L = raw[0].level
    re = (C.c_double * (L + 1))()
    im = (C.c_double * (L + 1))()
    _check(lib().tn_polarization_combine(raw, re, im))
    return np.array([complex(re[u], im[u]) for u in range(L + 1)]), [r.as_dict() for r in raw], ex


def tn_plan_workspace(plans: Sequence[Plan], terms: Sequence[Terms]):
    """(min_bytes, full_bytes) of tn_estimate's workspace."""
    mn, full = C.c_size_t(), C.c_size_t()
    _check(lib().tn_plan_workspace(len(plans), _handles(plans), _handles(terms), C.byref(mn), C.byref(full)))
    return mn.value, full.value


def tn_estimate(plans: Sequence[Plan], terms: Sequence[Terms], stream=None, ws=None) -> List[dict]:
    """Algorithm 1 end to end through tn_estimate.  ``ws``: a uint8 device
    tensor used as the workspace (default: one of the full size)."""
    import torch
    if ws is None:
        _, full = tn_plan_workspace(plans, terms)
        ws = torch.empty(max(256, full), dtype=torch.uint8, device="cuda")
    res = (tn_result * len(plans))()
    _check(lib().tn_estimate(len(plans), _handles(plans), _handles(terms), C.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream_ptr(stream), res))
    return [r.as_dict() for r in res]


def tn_contract_batch(plans: Sequence[Plan], terms: Sequence[Terms], first: int, count: int,
                      stream=None, ws=None, amp=None):
    """Amplitudes a_t (complex64, slots sqrt(2) K) of terms [first, first+count)
    per plan, as a torch tensor of shape (len(plans), count).  ``ws``: the
    workspace tensor (uint8, device; default: the full estimate's size);
    ``amp``: an output tensor of at least len(plans) * count complex64."""
    import torch
    if ws is None:
        _, full = tn_plan_workspace(plans, terms)
        ws = torch.empty(max(256, full), dtype=torch.uint8, device="cuda")
    if amp is None:
        amp = torch.zeros((len(plans), max(1, count)), dtype=torch.complex64, device="cuda")
    _check(lib().tn_contract_batch(len(plans), _handles(plans), _handles(terms), first, count,
                                   C.c_void_p(amp.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_ptr(stream)))
    return amp.reshape(len(plans), -1)[:, :count]


def tn_estimate_noalloc(plans: Sequence[Plan], terms: Sequence[Terms], stream=None) -> List[dict]:
    """Algorithm 1 end to end in the library's fixed device workspace (no
    allocation)."""
    res = (tn_result * len(plans))()
    _check(lib().tn_estimate_noalloc(len(plans), _handles(plans), _handles(terms), _stream_ptr(stream), res))
    return [r.as_dict() for r in res]


def tn_release_cached():
    """Drop the schedules tn_estimate / tn_contract_batch keep between calls."""
    lib().tn_release_cached()


# ---------------------------------------------------------------------------
# kernel-level entry points (include/tn_kernels.h), for numerical tests
# ---------------------------------------------------------------------------
def _kernel_lib():
    L = lib()
    if not getattr(L, "_kernel_sigs", False):
        vp = C.c_void_p
        L.tn_kernel_gemm.argtypes = [C.c_int32, vp, vp, vp, vp, vp, C.c_int64, C.c_int64, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int32, vp]
        L.tn_kernel_gemm.restype = C.c_int
        L.tn_kernel_permute.argtypes = [C.c_int32, vp, vp, C.c_int64, C.c_int32, vp, C.c_int32, vp]
        L.tn_kernel_permute.restype = C.c_int
        L.tn_kernel_mfma_group.argtypes = [C.c_int32, vp, vp, C.c_int64, vp]
        L.tn_kernel_mfma_group.restype = C.c_int
        L.tn_kernel_mfma_split_reduce.argtypes = [C.c_int32, C.c_int32, vp, vp, C.c_int64, vp]
        L.tn_kernel_mfma_split_reduce.restype = C.c_int
        L.tn_kernel_group_sums.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.tn_kernel_group_sums.restype = C.c_int
        L._kernel_sigs = True
    return L


def kernel_gemm(A, B, C_out, m_log, n_log, k_log, transA=0, transB=0, ia=None, ib=None,
                tile_hint=-1, stream=None):
    """torch complex64/complex128 tensors on the GPU; returns the kernel class."""
    import torch
    fp64 = 1 if A.dtype == torch.complex128 else 0
    n_inst = C_out.shape[0]
    rc = _kernel_lib().tn_kernel_gemm(
        fp64, C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()), C.c_void_p(C_out.data_ptr()),
        C.c_void_p(ia.data_ptr()) if ia is not None else None,
        C.c_void_p(ib.data_ptr()) if ib is not None else None,
        A[0].numel(), B[0].numel(), m_log, n_log, k_log, transA, transB, n_inst, tile_hint,
        _stream_ptr(stream))
    if rc < 0:
        _check(rc)
    return rc


def kernel_permute(src, dst, r, perm, block_elems_log=0, stream=None):
    import torch
    fp64 = 1 if src.dtype == torch.complex128 else 0
    p = np.ascontiguousarray(perm, dtype=np.int32)
    _check(_kernel_lib().tn_kernel_permute(fp64, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                           src.shape[0], r, p.ctypes.data if r else None, block_elems_log,
                                           _stream_ptr(stream)))


class tn_mfma_job(C.Structure):
    _fields_ = [("A", C.c_void_p), ("B", C.c_void_p), ("C", C.c_void_p), ("oa", C.c_void_p),
                ("ob", C.c_void_p), ("oc", C.c_void_p), ("m_log", C.c_int32), ("n_log", C.c_int32),
                ("k_log", C.c_int32), ("merge", C.c_int32), ("a_rowfast", C.c_int32), ("b_colfast", C.c_int32),
                ("a_row", C.c_int8 * 32), ("a_k", C.c_int8 * 32), ("b_k", C.c_int8 * 32),
                ("b_col", C.c_int8 * 32), ("ksplit", C.c_int32), ("pad_", C.c_int32),
                ("partial", C.c_void_p)]


MFMA_TILE = np.dtype([("job", "<i4"), ("cnt", "<i4"), ("s0", "<i8"), ("tm0", "<i8"), ("tn0", "<i8"),
                      ("kpart", "<i4"), ("pair", "<i4")])
MFMA_TILE_SHAPES = [(128, 64), (64, 64), (128, 32), (64, 32), (32, 32), (128, 16), (64, 16), (32, 16)]


def mfma_group_descriptors(jobs, tiles):
    """Device copies of grouped matrix-core job and tile descriptors.  jobs:
    dicts with device tensors A, B, C (complex64) and oa, ob, oc (int64 slice
    offsets), m_log, n_log, k_log, merge, a_rowfast, b_colfast and the
    bit-position lists a_row, a_k, b_k, b_col; tiles: array of MFMA_TILE."""
    import torch
    arr = (tn_mfma_job * len(jobs))()
    for q, j in enumerate(jobs):
        r = arr[q]
        r.A, r.B, r.C = j["A"].data_ptr(), j["B"].data_ptr(), j["C"].data_ptr()
        r.oa, r.ob, r.oc = j["oa"].data_ptr(), j["ob"].data_ptr(), j["oc"].data_ptr()
        for f in ("m_log", "n_log", "k_log", "merge", "a_rowfast", "b_colfast"):
            setattr(r, f, int(j[f]))
        for f in ("a_row", "a_k", "b_k", "b_col"):
            for i, v in enumerate(j[f]):
                getattr(r, f)[i] = int(v)
        r.ksplit = int(j.get("ksplit", 1))
        if r.ksplit > 1:
            r.partial = j["partial"].data_ptr()
    dj = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()
    t = np.ascontiguousarray(tiles, dtype=MFMA_TILE)
    dt = torch.from_numpy(t.view(np.uint8).copy()).cuda()
    return dj, dt, len(t)


def kernel_mfma_group(tile, descriptors, stream=None):
    """One grouped matrix-core launch over descriptors from
    mfma_group_descriptors (asynchronous on the stream).  Jobs with ksplit > 1
    leave partial tiles: follow with kernel_mfma_split_reduce."""
    dj, dt, n = descriptors
    _check(_kernel_lib().tn_kernel_mfma_group(tile, C.c_void_p(dj.data_ptr()), C.c_void_p(dt.data_ptr()),
                                              n, _stream_ptr(stream)))


def kernel_mfma_split_reduce(tile, descriptors, fp64=False, stream=None):
    """Adds the partial tiles of the split jobs of a preceding grouped launch
    on the same descriptors, in part order, and writes their outputs."""
    dj, dt, n = descriptors
    _check(_kernel_lib().tn_kernel_mfma_split_reduce(tile, 1 if fp64 else 0, C.c_void_p(dj.data_ptr()),
                                                     C.c_void_p(dt.data_ptr()), n, _stream_ptr(stream)))


# ---------------------------------------------------------------------------
# learned pruning (include/tn_mlp.h)
# ---------------------------------------------------------------------------
TN_N_FEATURES = 36


class tn_mlp_shape(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32)]


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_sigs", False):
        vp = C.c_void_p
        sp = C.POINTER(tn_mlp_shape)
        L.tn_mlp_sizes.argtypes = [sp, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_size_t),
                                   C.POINTER(C.c_size_t)]
        L.tn_mlp_init.argtypes = [sp, C.c_uint64, vp, vp]
        L.tn_mlp_fit_normalizer.argtypes = [sp, vp, vp, C.c_int64, vp]
        L.tn_mlp_forward.argtypes = [sp, vp, vp, C.c_int64, vp, vp, vp]
        L.tn_mlp_gradients.argtypes = [sp, vp, vp, vp, vp, C.c_int64, vp, vp, vp]
        L.tn_mlp_adam.argtypes = [sp, vp, C.c_float, C.c_int32, vp]
        L.tn_mlp_train_step.argtypes = [sp, vp, vp, vp, vp, C.c_int64, C.c_float, C.c_int32, vp, vp, vp]
        L.tn_terms_features.argtypes = [vp, vp, vp, vp]
        L.tn_prune_threshold.argtypes = [vp, vp, C.c_int64, C.c_double, C.POINTER(C.c_float)]
        L.tn_mlp_log_targets.argtypes = [vp, vp, C.c_int64, C.c_double, vp]
        L.tn_pruner_train_step.argtypes = [sp, vp, vp, vp, vp, C.c_int64, C.c_float, C.c_int32, vp, vp, vp]
        L.tn_pruner_save.argtypes = [sp, vp, vp, C.c_size_t, C.POINTER(C.c_size_t), vp]
        L.tn_pruner_load.argtypes = [sp, vp, vp, C.c_size_t, vp]
        for n in ("tn_mlp_sizes", "tn_mlp_init", "tn_mlp_fit_normalizer", "tn_mlp_forward", "tn_mlp_gradients",
                  "tn_mlp_adam", "tn_mlp_train_step", "tn_terms_features", "tn_prune_threshold",
                  "tn_mlp_log_targets", "tn_pruner_train_step", "tn_pruner_save", "tn_pruner_load"):
            getattr(L, n).restype = C.c_int
        L._mlp_sigs = True
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def tn_terms_features(plan: Plan, terms: Terms, level1_x: Optional[np.ndarray] = None) -> np.ndarray:
    out = np.zeros((max(1, terms.n), TN_N_FEATURES), dtype=np.float32)
    lx = None if level1_x is None else np.ascontiguousarray(level1_x, dtype=np.float64)
    _check(_mlp_lib().tn_terms_features(plan.handle, terms.handle, lx.ctypes.data if lx is not None else None,
                                        out.ctypes.data))
    return out[:terms.n]


def tn_prune_threshold(pred: np.ndarray, x: np.ndarray, budget: float) -> float:
    p = np.ascontiguousarray(pred, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    tau = C.c_float()
    _check(_mlp_lib().tn_prune_threshold(p.ctypes.data, xx.ctypes.data, p.size, budget, C.byref(tau)))
    return tau.value


class MLP:
    """Device state of the pruning network (torch-allocated)."""

    def save(self, stream=None) -> bytes:
        """The model (header, normalizer, parameters) as bytes."""
        need = C.c_size_t()
        _check(_mlp_lib().tn_pruner_save(C.byref(self.shape), _ptr(self.state), None, 0, C.byref(need),
                                         _stream_ptr(stream)))
        buf = (C.c_uint8 * need.value)()
        _check(_mlp_lib().tn_pruner_save(C.byref(self.shape), _ptr(self.state), buf, need.value, C.byref(need),
                                         _stream_ptr(stream)))
        return bytes(buf)

    def load(self, blob: bytes, stream=None):
        """Model bytes from save() into this state (optimizer moments reset)."""
        buf = (C.c_uint8 * len(blob)).from_buffer_copy(blob)
        _check(_mlp_lib().tn_pruner_load(C.byref(self.shape), _ptr(self.state), buf, len(blob),
                                         _stream_ptr(stream)))
        self.step = 0

    def __init__(self, n_in=TN_N_FEATURES, width=128, depth=3, seed=2211170280, max_batch=1 << 16, stream=None):
        import torch
        self.shape = tn_mlp_shape(n_in, width, depth)
        npar, sb, wb = C.c_int64(), C.c_size_t(), C.c_size_t()
        _check(_mlp_lib().tn_mlp_sizes(C.byref(self.shape), max_batch, C.byref(npar), C.byref(sb), C.byref(wb)))
        self.n_params = npar.value
        self.max_batch = max_batch
        self.state = torch.zeros(sb.value // 4, dtype=torch.float32, device="cuda")
        self.ws = torch.zeros(wb.value // 4, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.step = 0
        _check(_mlp_lib().tn_mlp_init(C.byref(self.shape), seed, _ptr(self.state), _stream_ptr(stream)))

    def fit_normalizer(self, x, stream=None):
        _check(_mlp_lib().tn_mlp_fit_normalizer(C.byref(self.shape), _ptr(self.state), _ptr(x), x.shape[0],
                                                _stream_ptr(stream)))

    def forward(self, x, stream=None):
        import torch
        out = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        for s in range(0, x.shape[0], self.max_batch):
            e = min(x.shape[0], s + self.max_batch)
            _check(_mlp_lib().tn_mlp_forward(C.byref(self.shape), _ptr(self.state), _ptr(x[s:e]), e - s,
                                              _ptr(out[s:e]), _ptr(self.ws), _stream_ptr(stream)))
        return out

    def gradients(self, x, t, w=None, stream=None):
        _check(_mlp_lib().tn_mlp_gradients(C.byref(self.shape), _ptr(self.state), _ptr(x), _ptr(t), _ptr(w),
                                           x.shape[0], _ptr(self.ws), _ptr(self.loss), _stream_ptr(stream)))

    def adam(self, lr, stream=None):
        self.step += 1
        _check(_mlp_lib().tn_mlp_adam(C.byref(self.shape), _ptr(self.state), lr, self.step, _stream_ptr(stream)))

    def train_step(self, x, t, w=None, lr=1e-3, stream=None):
        self.step += 1
        _check(_mlp_lib().tn_mlp_train_step(C.byref(self.shape), _ptr(self.state), _ptr(x), _ptr(t), _ptr(w),
                                            x.shape[0], lr, self.step, _ptr(self.ws), _ptr(self.loss),
                                            _stream_ptr(stream)))


def tn_mlp_log_targets(x_dev, floor=1e-30, stream=None):
    """float32 log(max(x, floor)) of a float64 device tensor, computed on the device."""
    import torch
    t = torch.empty(x_dev.shape[0], dtype=torch.float32, device="cuda")
    _check(_mlp_lib().tn_mlp_log_targets(_ptr(x_dev), _ptr(t), x_dev.shape[0], floor, _stream_ptr(stream)))
    return t
