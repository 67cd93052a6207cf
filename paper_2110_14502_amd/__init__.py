"""Python binding of librqc (include/rqc.h): argument marshalling only.

Every computation runs in the native library and its HIP kernels; PyTorch
only provides device memory and the current HIP stream.  Importing this
module fails loudly when the native library has not been built.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librqc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2110_14502_amd/build.py`")

# One HIP runtime per process: torch loads its own copy of the HIP and HSA
# runtimes by path, and a second copy loaded before it (by this library's
# dependencies) cannot see the device once torch has initialised it.  Loading
# torch first makes the library bind to torch's copy.
try:
    import torch  # noqa: F401
except ImportError:  # host-only use (planning, CPU tests) works without it
    pass

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
OK, EINVAL, ENOMEM, EHBM, EDEVICE, EUNSUPPORTED, ENUMERIC = 0, -1, -2, -3, -4, -5, -6
F32, F16, BF16 = 0, 1, 2
PRECISIONS = {"f32": F32, "fp32": F32, "f16": F16, "fp16": F16, "bf16": BF16}
GATE_H, GATE_SQRT_X, GATE_SQRT_Y, GATE_SQRT_W, GATE_FSIM, GATE_U1, GATE_U2 = range(7)
POLICY_SIZE, POLICY_CALIBRATED, POLICY_STORAGE = 0, 1, 2


class RqcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rqc error {code}: {msg}")
        self.code = code


# ---------------------------------------------------------------- structs
class rqc_gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("reserved", C.c_int32), ("theta", C.c_double), ("phi", C.c_double),
                ("u", C.c_double * 32)]


class rqc_plan_opts(C.Structure):
    _fields_ = [("max_log2_elems", C.c_int32), ("n_sliced", C.c_int32),
                ("path_trials", C.c_int32), ("reconf_rounds", C.c_int32),
                ("seed", C.c_uint64), ("n_forced", C.c_int32),
                ("forced_wires", C.POINTER(C.c_int32)), ("lp_min_log2", C.c_int32),
                ("bf16_min_log2", C.c_int32), ("n_local_sliced", C.c_int32),
                ("n_share_bits", C.c_int32), ("share_bits", C.POINTER(C.c_uint8)),
                ("restarts", C.c_int32), ("precision_policy", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64)]


class rqc_plan_info(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_open", C.c_int32), ("n_closed", C.c_int32),
                ("n_sliced", C.c_int32), ("n_slices", C.c_uint64), ("n_leaves", C.c_int32),
                ("n_steps", C.c_int32), ("n_invariant_steps", C.c_int32),
                ("max_log2_elems", C.c_int32), ("flops_per_slice", C.c_double),
                ("flops_invariant", C.c_double), ("bytes_per_slice", C.c_double),
                ("log2_total_flops", C.c_double), ("flops_per_bitstring", C.c_double)]


class rqc_step_info(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("kernel", C.c_int32),
                ("kernel_lp", C.c_int32), ("depends_on_slice", C.c_int32),
                ("depends_on_bits", C.c_int32), ("lp_output", C.c_int32),
                ("lp_output_bf16", C.c_int32), ("reserved", C.c_int32), ("flops", C.c_double),
                ("bytes_c64", C.c_double)]


class rqc_run_report(C.Structure):
    _fields_ = [("n_slices", C.c_uint64), ("fp32_reruns", C.c_uint64),
                ("slices_per_group", C.c_int32), ("bits_per_group", C.c_int32),
                ("graph_reused", C.c_int32), ("reserved", C.c_int32), ("flops", C.c_double)]


class rqc_timing(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("total_ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


class rqc_launch_timing(C.Structure):
    _fields_ = [("step", C.c_int32), ("kernel", C.c_int32), ("m", C.c_int32), ("n", C.c_int32),
                ("k", C.c_int32), ("copies", C.c_int32), ("store_a", C.c_int32),
                ("store_b", C.c_int32), ("store_c", C.c_int32), ("variant", C.c_int32),
                ("ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


class rqc_tune_report(C.Structure):
    _fields_ = [("steps", C.c_int32), ("timed", C.c_int32), ("cached", C.c_int32),
                ("changed", C.c_int32), ("ms_default", C.c_double), ("ms_tuned", C.c_double)]


class rqc_calib_report(C.Structure):
    _fields_ = [("candidates", C.c_int32), ("reduced", C.c_int32),
                ("estimated_err", C.c_double), ("measured_err", C.c_double),
                ("min_step_err", C.c_double), ("max_step_err", C.c_double)]


class rqc_server_opts(C.Structure):
    _fields_ = [("device_pool", C.c_void_p), ("hbm_budget_bytes", C.c_uint64),
                ("max_inflight", C.c_int32), ("n_streams", C.c_int32),
                ("max_batch", C.c_int32), ("device", C.c_int32)]


class rqc_request(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_open", C.c_int32),
                ("gates", C.POINTER(rqc_gate)), ("n_gates", C.c_uint64),
                ("open_qubits", C.POINTER(C.c_int32)), ("closed_bits", C.POINTER(C.c_uint8)),
                ("prec", C.c_int32), ("max_log2_elems", C.c_int32), ("plan_key", C.c_uint64),
                ("seed", C.c_uint64)]


class rqc_result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("n_open", C.c_int32),
                ("amplitudes", C.POINTER(C.c_double)), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("fp32_reruns", C.c_uint64)]


class rqc_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("plans_built", C.c_uint64), ("plans_reused", C.c_uint64),
                ("peak_bytes", C.c_uint64), ("max_inflight_seen", C.c_uint64)]


# ---------------------------------------------------------------- prototypes
_P = C.c_void_p
_S = C.c_int32
_PROTOS = {
    "rqc_circuit_create": (_S, [C.c_int32, C.POINTER(rqc_gate), C.c_size_t, C.POINTER(_P)]),
    "rqc_circuit_destroy": (None, [_P]),
    "rqc_network_create": (_S, [_P, C.POINTER(C.c_int32), C.c_int32, C.POINTER(_P)]),
    "rqc_network_destroy": (None, [_P]),
    "rqc_plan_opts_default": (None, [C.POINTER(rqc_plan_opts)]),
    "rqc_plan_create": (_S, [_P, C.POINTER(rqc_plan_opts), C.POINTER(_P)]),
    "rqc_plan_destroy": (None, [_P]),
    "rqc_plan_info": (_S, [_P, C.POINTER(rqc_plan_info)]),
    "rqc_plan_get_step": (_S, [_P, C.c_int32, C.POINTER(rqc_step_info)]),
    "rqc_plan_export_json": (_S, [_P, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "rqc_plan_resident_bytes": (_S, [_P, C.POINTER(C.c_size_t)]),
    "rqc_plan_bind_memory": (_S, [_P, _P, C.c_size_t, _P]),
    "rqc_contract_workspace": (_S, [_P, C.c_uint64, C.c_uint64, C.c_int32,
                                    C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "rqc_contract": (_S, [_P, C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(C.c_uint8),
                          C.c_uint64, C.c_int32, _P, C.c_size_t, _P, _P, _P]),
    "rqc_contract_status": (_S, [_P, _P, C.POINTER(rqc_run_report)]),
    "rqc_pair_contract": (_S, [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                               C.POINTER(C.c_int32), C.c_int32, _P, _P, _P, C.c_int32,
                               C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _P]),
    "rqc_pair_workspace_bytes": (_S, [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32),
                                      C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                      C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_uint64)]),
    "rqc_pair_contract_ws": (_S, [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                  C.POINTER(C.c_int32), C.c_int32, _P, _P, _P, C.c_int32,
                                  C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _P,
                                  C.c_uint64, _P]),
    "rqc_permute": (_S, [C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32, _P, _P, _P]),
    "rqc_batch_xeb": (_S, [_P, C.c_uint64, C.c_int32, _P, C.c_uint64, _P, _P]),
    "rqc_contract_noalloc": (_S, [_P, C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(C.c_uint8),
                                  C.c_uint64, C.c_int32, _P, _P, _P]),
    "rqc_contract_noalloc_scratch_bytes": (C.c_uint64, []),
    "rqc_cgemm": (_S, [C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P]),
    "rqc_server_create": (_S, [C.POINTER(rqc_server_opts), C.POINTER(_P)]),
    "rqc_server_submit": (_S, [_P, C.POINTER(rqc_request), C.POINTER(C.c_uint64)]),
    "rqc_server_poll": (_S, [_P, C.POINTER(rqc_result), C.c_size_t, C.POINTER(C.c_size_t)]),
    "rqc_server_release": (_S, [_P, C.c_uint64]),
    "rqc_server_drain": (_S, [_P]),
    "rqc_server_get_stats": (_S, [_P, C.POINTER(rqc_server_stats)]),
    "rqc_server_destroy": (None, [_P]),
    "rqc_last_error": (C.c_char_p, []),
    "rqc_version": (C.c_char_p, []),
    "rqc_plan_set_scale_bias": (_S, [_P, C.c_int32, C.c_uint64]),
    "rqc_plan_get_launch_timing": (_S, [_P, C.c_uint64, C.POINTER(rqc_launch_timing)]),
    "rqc_pair_contract_stored": (_S, [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32),
                                      C.c_int32, C.POINTER(C.c_int32), C.c_int32, _P, _P, _P,
                                      C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                      C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                      _P]),
    "rqc_plan_set_timing": (_S, [_P, C.c_int32]),
    "rqc_plan_autotune": (_S, [_P, C.c_int32, C.c_uint64, C.c_uint64, _P, C.c_size_t, C.c_char_p,
                               _P, C.POINTER(rqc_tune_report)]),
    "rqc_plan_calibrate": (_S, [_P, C.c_int32, C.c_uint64, C.POINTER(C.c_uint8), C.c_double,
                                C.c_double, _P, C.c_size_t, _P, C.POINTER(rqc_calib_report)]),
    "rqc_plan_set_group_limit": (_S, [_P, C.c_int32, C.c_int32]),
    "rqc_plan_get_timing": (_S, [_P, C.POINTER(rqc_timing)]),
}
for _name, (_res, _args) in _PROTOS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_PROTOS)


def _check(code):
    if code != OK:
        raise RqcError(code, _lib.rqc_last_error().decode())


def version() -> str:
    return _lib.rqc_version().decode()


def _i32(seq):
    arr = (C.c_int32 * max(1, len(seq)))(*[int(x) for x in seq])
    return arr


def _stream_handle(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def _ptr(t):
    return C.c_void_p(int(t.data_ptr()))


# ---------------------------------------------------------------- gates
def to_gate_array(gates):
    """rqcgen.Gate list (or tuples) -> ctypes array of rqc_gate."""
    arr = (rqc_gate * max(1, len(gates)))()
    for i, g in enumerate(gates):
        a = arr[i]
        a.kind = int(g.kind)
        a.q0 = int(g.q0)
        a.q1 = int(g.q1) if g.q1 is not None else -1
        a.theta = float(g.theta)
        a.phi = float(g.phi)
        if g.u is not None:
            u = np.asarray(g.u, dtype=np.complex128).reshape(-1)
            for j, v in enumerate(u):
                a.u[2 * j] = v.real
                a.u[2 * j + 1] = v.imag
    return arr


class Circuit:
    def __init__(self, n_qubits: int, gates):
        self._gates = to_gate_array(gates)
        h = C.c_void_p()
        _check(_lib.rqc_circuit_create(int(n_qubits), self._gates, len(gates), C.byref(h)))
        self.h = h
        self.n_qubits = int(n_qubits)

    @classmethod
    def from_rqcgen(cls, circ):
        return cls(circ.n_qubits, circ.gates)

    def __del__(self):
        # At interpreter exit the module's globals may already be gone.
        lib = _lib
        if getattr(self, "h", None) and lib is not None:
            lib.rqc_circuit_destroy(self.h)
            self.h = None


class Network:
    def __init__(self, circuit: Circuit, open_qubits):
        self.open = [int(q) for q in open_qubits]
        h = C.c_void_p()
        _check(_lib.rqc_network_create(circuit.h, _i32(self.open), len(self.open), C.byref(h)))
        self.h = h
        self.n_qubits = circuit.n_qubits

    def __del__(self):
        # At interpreter exit the module's globals may already be gone.
        lib = _lib
        if getattr(self, "h", None) and lib is not None:
            lib.rqc_network_destroy(self.h)
            self.h = None


class Plan:
    """Contraction path + slicing plan, optionally bound to device memory."""

    def __init__(self, network: Network, max_log2_elems=0, n_sliced=-1, path_trials=256,
                 reconf_rounds=-1, seed=0, forced_wires=(), lp_min_log2=0, bf16_min_log2=0,
                 n_local_sliced=0, share_bits=(), restarts=1, precision_policy=0,
                 hbm_budget_bytes=0):
        o = rqc_plan_opts()
        _lib.rqc_plan_opts_default(C.byref(o))
        o.max_log2_elems = int(max_log2_elems)
        o.n_sliced = int(n_sliced)
        o.path_trials = int(path_trials)
        o.reconf_rounds = int(reconf_rounds)
        o.seed = int(seed)
        flat = [int(x) for w in forced_wires for x in w]
        self._forced = _i32(flat)
        o.n_forced = len(forced_wires)
        o.forced_wires = C.cast(self._forced, C.POINTER(C.c_int32))
        o.lp_min_log2 = int(lp_min_log2)
        o.bf16_min_log2 = int(bf16_min_log2)
        o.n_local_sliced = int(n_local_sliced)
        self._share = (C.c_uint8 * max(1, len(share_bits)))(*[int(b) for b in share_bits])
        o.n_share_bits = len(share_bits)
        o.restarts = int(restarts)
        o.share_bits = C.cast(self._share, C.POINTER(C.c_uint8))
        o.precision_policy = int(precision_policy)
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        h = C.c_void_p()
        _check(_lib.rqc_plan_create(network.h, C.byref(o), C.byref(h)))
        self.h = h
        self.open = list(network.open)
        self.n_qubits = network.n_qubits
        self._resident = None
        self._ws = None

    def __del__(self):
        # At interpreter exit the module's globals may already be gone.
        lib = _lib
        if getattr(self, "h", None) and lib is not None:
            lib.rqc_plan_destroy(self.h)
            self.h = None

    # ---- host-side description
    def info(self) -> dict:
        i = rqc_plan_info()
        _check(_lib.rqc_plan_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in rqc_plan_info._fields_}

    def steps(self):
        out = []
        for k in range(self.info()["n_steps"]):
            s = rqc_step_info()
            _check(_lib.rqc_plan_get_step(self.h, k, C.byref(s)))
            out.append({f: getattr(s, f) for f, _ in rqc_step_info._fields_})
        return out

    def export(self) -> dict:
        need = C.c_size_t()
        _check(_lib.rqc_plan_export_json(self.h, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check(_lib.rqc_plan_export_json(self.h, buf, need.value, C.byref(need)))
        return json.loads(buf.value.decode())

    def sliced_wires(self):
        """Enumerated sliced wires (q, segment), slice-bit order."""
        return [tuple(w) for w in self.export()["sliced_wires"]]

    def pruned_wires(self):
        """Wires that carry a single value (a zero slab in a leaf), projected
        out before planning: (q, segment, value)."""
        return [tuple(w) for w in self.export()["pruned_wires"]]

    def fixed_wires(self):
        """Sliced wires fixed by the slice share: (q, segment, value), in
        slice-bit order after the enumerated ones."""
        return [tuple(w) for w in self.export()["fixed_wires"]]

    def resident_bytes(self) -> int:
        b = C.c_size_t()
        _check(_lib.rqc_plan_resident_bytes(self.h, C.byref(b)))
        return b.value

    def workspace_bytes(self, n_ids=0, n_batch=1, prec=F32):
        lo, pref = C.c_size_t(), C.c_size_t()
        _check(_lib.rqc_contract_workspace(self.h, int(n_ids), int(n_batch), int(prec),
                                           C.byref(lo), C.byref(pref)))
        return lo.value, pref.value

    # ---- device
    def bind(self, device="cuda", stream=None):
        import torch
        nbytes = max(256, self.resident_bytes())
        self._resident = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _check(_lib.rqc_plan_bind_memory(self.h, _ptr(self._resident), nbytes,
                                         _stream_handle(stream)))
        return self

    def set_scale_bias(self, bias: int, first_bitstring: int = 0):
        """Test hook: bias the 16-bit storage shifts of bitstring groups from
        first_bitstring on (forces the FP32 re-run path)."""
        _check(_lib.rqc_plan_set_scale_bias(self.h, int(bias), int(first_bitstring)))

    def contract(self, closed_bits, slice_ids=None, prec=F32, workspace=None,
                 per_slice=False, stream=None, sync=True, out=None):
        """Amplitudes (complex128, shape (n_batch, 2^n_open)) summed over slices.

        closed_bits: array (n_batch, n_closed) or (n_closed,) of 0/1.
        workspace: torch uint8 device tensor, or None for the preferred size.
        """
        import torch
        bits = np.ascontiguousarray(np.asarray(closed_bits, dtype=np.uint8))
        if bits.ndim == 1:
            bits = bits.reshape(1, -1)
        n_batch = bits.shape[0]
        prec = PRECISIONS.get(prec, prec) if isinstance(prec, str) else int(prec)
        ids = None if slice_ids is None else np.ascontiguousarray(np.asarray(slice_ids, dtype=np.uint64))
        n_ids = 0 if ids is None else ids.size
        n_out = n_batch * (1 << len(self.open))
        dev = self._resident.device
        if out is None:
            out = torch.empty(2 * n_out, dtype=torch.float64, device=dev)
        ps = None
        if per_slice:
            cnt = n_ids if ids is not None else self.info()["n_slices"]
            ps = torch.zeros(2 * n_out * cnt, dtype=torch.float64, device=dev)
        if workspace is None:
            lo, pref = self.workspace_bytes(n_ids, n_batch, prec)
            have = self._ws.numel() if self._ws is not None else 0
            if have < min(pref, max(lo, have)) or have < lo or (have < pref and self._ws is None):
                self._ws = None
                free, _ = torch.cuda.mem_get_info(dev)
                size = int(min(pref, max(lo, 0.8 * free)))
                self._ws = torch.empty(size, dtype=torch.uint8, device=dev)
            workspace = self._ws
        idp = ids.ctypes.data_as(C.POINTER(C.c_uint64)) if ids is not None else None
        _check(_lib.rqc_contract(self.h, idp, n_ids, bits.ctypes.data_as(C.POINTER(C.c_uint8)),
                                 n_batch, prec, _ptr(workspace), workspace.numel(), _ptr(out),
                                 _ptr(ps) if ps is not None else None, _stream_handle(stream)))
        self.last_report = None
        if sync:
            self.last_report = self.report(stream)
        amps = out.view(n_batch, -1, 2)
        if per_slice:
            return amps, ps.view(-1, n_batch, 1 << len(self.open), 2)
        return amps

    def contract_noalloc(self, closed_bits, slice_ids=None, prec=F32, per_slice=False,
                         stream=None, sync=True, out=None):
        """contract() through rqc_contract_noalloc: the workspace is the
        library's static per-device scratch (no workspace argument).  Calls
        on one GPU must not overlap."""
        import torch
        bits = np.ascontiguousarray(np.asarray(closed_bits, dtype=np.uint8))
        if bits.ndim == 1:
            bits = bits.reshape(1, -1)
        n_batch = bits.shape[0]
        prec = PRECISIONS.get(prec, prec) if isinstance(prec, str) else int(prec)
        ids = None if slice_ids is None else np.ascontiguousarray(np.asarray(slice_ids, dtype=np.uint64))
        n_ids = 0 if ids is None else ids.size
        n_out = n_batch * (1 << len(self.open))
        dev = self._resident.device if self._resident is not None else \
            torch.device("cuda", torch.cuda.current_device())
        if out is None:
            out = torch.empty(2 * n_out, dtype=torch.float64, device=dev)
        ps = None
        if per_slice:
            cnt = n_ids if ids is not None else self.info()["n_slices"]
            ps = torch.zeros(2 * n_out * cnt, dtype=torch.float64, device=dev)
        idp = ids.ctypes.data_as(C.POINTER(C.c_uint64)) if ids is not None else None
        _check(_lib.rqc_contract_noalloc(self.h, idp, n_ids,
                                         bits.ctypes.data_as(C.POINTER(C.c_uint8)), n_batch, prec,
                                         _ptr(out), _ptr(ps) if ps is not None else None,
                                         _stream_handle(stream)))
        self.last_report = None
        if sync:
            self.last_report = self.report(stream)
        amps = out.view(n_batch, -1, 2)
        if per_slice:
            return amps, ps.view(-1, n_batch, 1 << len(self.open), 2)
        return amps

    def _scratch(self, n_ids, n_batch, prec, extra=0):
        import torch
        lo, pref = self.workspace_bytes(n_ids, n_batch, prec)
        have = self._ws.numel() if self._ws is not None else 0
        if have < lo + extra:
            self._ws = None
            free, _ = torch.cuda.mem_get_info(self._resident.device)
            size = int(min(pref + extra, max(lo + extra, 0.8 * free)))
            self._ws = torch.empty(size, dtype=torch.uint8, device=self._resident.device)
        return self._ws

    def autotune(self, prec=F32, n_ids=0, n_batch=1, workspace=None, cache_path=None,
                 stream=None) -> dict:
        """Time each step's valid (kernel, variant) pairs for this call shape
        and keep the fastest (rqc_plan_autotune)."""
        prec = PRECISIONS.get(prec, prec) if isinstance(prec, str) else int(prec)
        ws = workspace if workspace is not None else self._scratch(n_ids, n_batch, prec)
        r = rqc_tune_report()
        _check(_lib.rqc_plan_autotune(self.h, prec, int(n_ids), int(n_batch), _ptr(ws), ws.numel(),
                                      cache_path.encode() if cache_path else None,
                                      _stream_handle(stream), C.byref(r)))
        return {f: getattr(r, f) for f, _ in rqc_tune_report._fields_}

    def calibrate(self, closed_bits, prec=F16, slice_id=0, target_err=5e-3, err_floor=0.0,
                  workspace=None, stream=None) -> dict:
        """Per-step precision assignment from the sensitivity of one slice
        (rqc_plan_calibrate)."""
        prec = PRECISIONS.get(prec, prec) if isinstance(prec, str) else int(prec)
        bits = np.ascontiguousarray(np.asarray(closed_bits, dtype=np.uint8).reshape(-1))
        extra = 256 + 16 * (1 << len(self.open))
        ws = workspace if workspace is not None else self._scratch(1, 1, F32, extra)
        r = rqc_calib_report()
        _check(_lib.rqc_plan_calibrate(self.h, prec, int(slice_id),
                                       bits.ctypes.data_as(C.POINTER(C.c_uint8)), float(target_err),
                                       float(err_floor), _ptr(ws), ws.numel(),
                                       _stream_handle(stream), C.byref(r)))
        return {f: getattr(r, f) for f, _ in rqc_calib_report._fields_}

    def set_group_limit(self, max_slices=0, max_bits=0):
        """Bound the slices / bitstrings per batched group (0 = workspace only)."""
        _check(_lib.rqc_plan_set_group_limit(self.h, int(max_slices), int(max_bits)))

    def set_timing(self, kernel: int):
        """Bracket launches of kernel kind (0 SIMT, 1 MFMA, -1 off) with events."""
        _check(_lib.rqc_plan_set_timing(self.h, int(kernel)))

    def timing(self) -> dict:
        t = rqc_timing()
        _check(_lib.rqc_plan_get_timing(self.h, C.byref(t)))
        return {f: getattr(t, f) for f, _ in rqc_timing._fields_}

    def launch_timings(self):
        """Per probed launch of the last reported call: step, kernel, shape,
        storage, event-measured ms, algorithmic flops and bytes."""
        out = []
        for i in range(int(self.timing()["launches"])):
            t = rqc_launch_timing()
            _check(_lib.rqc_plan_get_launch_timing(self.h, i, C.byref(t)))
            out.append({f: getattr(t, f) for f, _ in rqc_launch_timing._fields_})
        return out

    def report(self, stream=None) -> dict:
        r = rqc_run_report()
        _check(_lib.rqc_contract_status(self.h, _stream_handle(stream), C.byref(r)))
        return {f: getattr(r, f) for f, _ in rqc_run_report._fields_}


def to_complex(t):
    """(..., 2) float64 tensor/array -> complex128 numpy array."""
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    return a[..., 0] + 1j * a[..., 1]


# ---------------------------------------------------------------- single steps
def pair_workspace_bytes(labels_a, labels_b, labels_c, kernel=-1, batch=1, stride_a=0,
                         stride_b=0, prec=F32):
    """Device workspace (bytes) that a pair_contract call needs (0: none)."""
    n = C.c_uint64()
    _check(_lib.rqc_pair_workspace_bytes(_i32(labels_a), len(labels_a), _i32(labels_b),
                                         len(labels_b), _i32(labels_c), len(labels_c), int(batch),
                                         int(stride_a), int(stride_b), int(kernel), int(prec),
                                         C.byref(n)))
    return n.value


def pair_contract(A, B, labels_a, labels_b, labels_c, C_out=None, kernel=-1, batch=1,
                  stride_a=0, stride_b=0, stride_c=0, prec=F32, stream=None, workspace=None):
    """C = A * B summed over shared labels (complex64 torch tensors on
    device).  A 16-bit call with a long sum takes the two-phase form and
    needs a device workspace (pair_workspace_bytes); one is allocated with
    torch unless `workspace` (a uint8 device tensor) is given."""
    import torch
    prec = PRECISIONS.get(prec, prec) if isinstance(prec, str) else int(prec)
    if C_out is None:
        C_out = torch.empty(batch << len(labels_c), dtype=torch.complex64, device=A.device)
        stride_c = 1 << len(labels_c) if batch > 1 else stride_c
    need = pair_workspace_bytes(labels_a, labels_b, labels_c, kernel, batch, stride_a, stride_b,
                                prec)
    if need:
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
        _check(_lib.rqc_pair_contract_ws(_i32(labels_a), len(labels_a), _i32(labels_b),
                                         len(labels_b), _i32(labels_c), len(labels_c), _ptr(A),
                                         _ptr(B), _ptr(C_out), int(batch), int(stride_a),
                                         int(stride_b), int(stride_c), int(kernel), int(prec),
                                         _ptr(workspace), int(workspace.numel()),
                                         _stream_handle(stream)))
        return C_out
    _check(_lib.rqc_pair_contract(_i32(labels_a), len(labels_a), _i32(labels_b), len(labels_b),
                                  _i32(labels_c), len(labels_c), _ptr(A), _ptr(B), _ptr(C_out),
                                  int(batch), int(stride_a), int(stride_b), int(stride_c),
                                  int(kernel), int(prec), _stream_handle(stream)))
    return C_out


ST_C64, ST_F16, ST_BF16 = 0, 1, 2
KERN_SIMT, KERN_MFMA, KERN_ROWS, KERN_MFMA16 = 0, 1, 2, 3


VAR_4M, VAR_TILES, VAR_PERSISTENT, VAR_FP32_MATH, VAR_STREAM, VAR_SWAP = 1, 2, 4, 8, 16, 32


def pair_contract_stored(A, B, C_out, labels_a, labels_b, labels_c, store_a, store_b, store_c,
                         kernel, mma_prec=F32, batch=1, stride_a=0, stride_b=0, stride_c=0,
                         variant=0, stream=None):
    """One contraction with explicit operand storage (ST_*) and kernel
    (KERN_*); A, B, C_out are device tensors holding complex64 or packed
    16-bit (re, im) pairs as their storage code says."""
    _check(_lib.rqc_pair_contract_stored(_i32(labels_a), len(labels_a), _i32(labels_b),
                                         len(labels_b), _i32(labels_c), len(labels_c), _ptr(A),
                                         _ptr(B), _ptr(C_out), int(store_a), int(store_b),
                                         int(store_c), int(batch), int(stride_a), int(stride_b),
                                         int(stride_c), int(kernel), int(mma_prec),
                                         int(variant), _stream_handle(stream)))
    return C_out


def batch_xeb(amps, n_qubits, samples=None, stream=None):
    """FP64 statistics of an amplitude batch on the device (rqc_batch_xeb):
    amps is the float64 device tensor of (re, im) pairs that contract()
    returns; samples an int64 device tensor of entry indices or None."""
    import torch
    n = amps.numel() // 2
    out = torch.empty(5, dtype=torch.float64, device=amps.device)
    ns = 0 if samples is None else samples.numel()
    _check(_lib.rqc_batch_xeb(_ptr(amps), n, int(n_qubits),
                              _ptr(samples) if samples is not None else None, ns, _ptr(out),
                              _stream_handle(stream)))
    v = out.cpu().numpy()
    return {"sum_p": float(v[0]), "sum_p2": float(v[1]), "xeb_all": float(v[2]),
            "xeb_ideal_sampling": float(v[3]), "xeb_samples": float(v[4])}


def permute(X, labels_in, labels_out, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty_like(X)
    _check(_lib.rqc_permute(_i32(labels_in), _i32(labels_out), len(labels_in), _ptr(X), _ptr(out),
                            _stream_handle(stream)))
    return out


def cgemm(A, B, M, N, K, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty(M * N, dtype=torch.complex64, device=A.device)
    _check(_lib.rqc_cgemm(int(M), int(N), int(K), _ptr(A), _ptr(B), _ptr(out), _stream_handle(stream)))
    return out


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching server over a device pool allocated with torch."""

    def __init__(self, budget_bytes, max_inflight=8, n_streams=4, max_batch=64, device=0):
        import torch
        self._pool = torch.empty(int(budget_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        o = rqc_server_opts()
        o.device_pool = C.c_void_p(int(self._pool.data_ptr()))
        o.hbm_budget_bytes = int(budget_bytes)
        o.max_inflight = int(max_inflight)
        o.n_streams = int(n_streams)
        o.max_batch = int(max_batch)
        o.device = int(device)
        h = C.c_void_p()
        torch.cuda.synchronize()
        _check(_lib.rqc_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, n_qubits, gates, open_qubits, closed_bits, prec=F32, max_log2_elems=0,
               plan_key=0, seed=0) -> int:
        g = to_gate_array(gates)
        op = _i32(open_qubits)
        bits = (C.c_uint8 * max(1, len(closed_bits)))(*[int(b) for b in closed_bits])
        r = rqc_request()
        r.n_qubits = int(n_qubits)
        r.n_open = len(open_qubits)
        r.gates = C.cast(g, C.POINTER(rqc_gate))
        r.n_gates = len(gates)
        r.open_qubits = C.cast(op, C.POINTER(C.c_int32))
        r.closed_bits = C.cast(bits, C.POINTER(C.c_uint8))
        r.prec = int(prec)
        r.max_log2_elems = int(max_log2_elems)
        r.plan_key = int(plan_key)
        r.seed = int(seed)
        t = C.c_uint64()
        _check(_lib.rqc_server_submit(self.h, C.byref(r), C.byref(t)))
        return t.value

    def poll(self, cap=256):
        arr = (rqc_result * cap)()
        n = C.c_size_t()
        _check(_lib.rqc_server_poll(self.h, arr, cap, C.byref(n)))
        out = []
        for i in range(n.value):
            r = arr[i]
            amps = None
            if r.status == OK:
                ne = 1 << r.n_open
                buf = np.ctypeslib.as_array(r.amplitudes, shape=(2 * ne,)).copy()
                amps = buf[0::2] + 1j * buf[1::2]
            _check(_lib.rqc_server_release(self.h, r.ticket))
            out.append({"ticket": r.ticket, "status": r.status, "amplitudes": amps,
                        "t_submit": r.t_submit, "t_start": r.t_start, "t_done": r.t_done,
                        "fp32_reruns": r.fp32_reruns})
        return out

    def drain(self):
        _check(_lib.rqc_server_drain(self.h))

    def stats(self) -> dict:
        s = rqc_server_stats()
        _check(_lib.rqc_server_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in rqc_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            _lib.rqc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
