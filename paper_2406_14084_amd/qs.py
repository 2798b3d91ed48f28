"""Python binding of libqs (include/qs.h): argument marshalling only.

Every computation runs in the library's HIP kernels; this module converts
Python/numpy/torch arguments to the C ABI and raises on error.  PyTorch
provides device memory (the state vector and outputs) and the stream.
There is no fallback: if libqs.so is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

QS_C128, QS_C64 = 0, 1
_STATUS = {0: "QS_OK", -1: "QS_EINVAL", -2: "QS_ENOMEM", -3: "QS_EHIP", -4: "QS_EUNSUPPORTED", -5: "QS_ESTATE"}


class QSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, code), msg))
        self.code = code


class Circuit_C(C.Structure):
    _fields_ = [("n", C.c_int), ("ngates", C.c_int), ("k", C.POINTER(C.c_int)),
                ("targets", C.POINTER(C.c_int)), ("matrices", C.POINTER(C.c_double))]


class PlanOpts_C(C.Structure):
    _fields_ = [("chunk_qubits", C.c_int), ("low_qubits", C.c_int), ("enable_swaps", C.c_int),
                ("enable_fusion", C.c_int), ("planner", C.c_int), ("cost_model", C.c_void_p),
                ("dtype", C.c_int), ("reg_qubits", C.c_int), ("no_mfma", C.c_int),
                ("no_split", C.c_int)]


class Pauli_C(C.Structure):
    _fields_ = [("xmask", C.c_uint64), ("zmask", C.c_uint64), ("coeff", C.c_double)]


class PlanStats_C(C.Structure):
    _fields_ = [("n", C.c_int), ("dtype", C.c_int), ("gates", C.c_int), ("blocks", C.c_int),
                ("swap_passes", C.c_int), ("ops", C.c_int), ("ops_dense", C.c_int * 6), ("ops_diag", C.c_int),
                ("phases", C.c_int), ("chunk_qubits", C.c_int), ("low_qubits", C.c_int), ("reg_qubits", C.c_int),
                ("flops_per_amp", C.c_double), ("hbm_bytes", C.c_double), ("plan_seconds", C.c_double),
                ("planner", C.c_int), ("candidates", C.c_int), ("predicted_ms", C.c_double),
                ("predicted_heuristic_ms", C.c_double), ("ops_mfma", C.c_int),
                ("ops_rot", C.c_int), ("ops_perm", C.c_int)]


class QaoaInst_C(C.Structure):
    _fields_ = [("n", C.c_int), ("nedges", C.c_int), ("p", C.c_int), ("edges", C.POINTER(C.c_int)),
                ("gammas", C.POINTER(C.c_double)), ("betas", C.POINTER(C.c_double))]


_lib = None

# name -> (restype, argtypes); the full exported surface of qs.h
_P = C.c_void_p
SIGNATURES = {
    "qs_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(_P)]),
    "qs_attach": (C.c_int, [_P, _P, C.c_size_t, _P, _P, C.c_size_t]),
    "qs_workspace_size": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "qs_get_amplitudes": (C.c_int, [_P, C.c_uint64, C.c_uint64, _P]),
    "qs_destroy": (C.c_int, [_P]),
    "qs_init_zero": (C.c_int, [_P]),
    "qs_init_basis": (C.c_int, [_P, C.c_uint64]),
    "qs_apply_gate": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "qs_swap_qubits": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "qs_gate_class": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_int),
                                C.POINTER(C.c_uint64), C.POINTER(C.c_int)]),
    "qs_fuse": (C.c_int, [C.POINTER(Circuit_C), C.c_int, C.POINTER(PlanOpts_C), C.POINTER(_P)]),
    "qs_apply_plan": (C.c_int, [_P, _P]),
    "qs_apply_plan_timed": (C.c_int, [_P, _P, C.POINTER(C.c_float), C.POINTER(C.c_int), C.c_int]),
    "qs_plan_free": (C.c_int, [_P]),
    "qs_plan_dump": (C.c_int, [_P, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "qs_plan_get_stats": (C.c_int, [_P, C.POINTER(PlanStats_C)]),
    "qs_plan_block": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)]),
    "qs_plan_layout": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "qs_plan_program": (C.c_int, [_P, C.POINTER(C.c_int32), C.c_size_t, C.POINTER(C.c_size_t),
                                  C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_size_t, C.POINTER(C.c_size_t)]),
    "qs_probs": (C.c_int, [_P, _P]),
    "qs_expect": (C.c_int, [_P, C.c_int, C.POINTER(Pauli_C), C.POINTER(C.c_double)]),
    "qs_expect_noalloc": (C.c_int, [_P, C.c_int, C.POINTER(Pauli_C), C.POINTER(C.c_double)]),
    "qs_batch_qaoa_create": (C.c_int, [C.c_int, C.POINTER(QaoaInst_C), C.c_int, _P, _P, C.c_size_t, C.POINTER(_P)]),
    "qs_batch_qaoa_workspace_size": (C.c_int, [C.c_int, C.POINTER(QaoaInst_C), C.c_int, C.POINTER(C.c_size_t)]),
    "qs_batch_qaoa_run": (C.c_int, [_P, _P, C.c_int]),
    "qs_batch_qaoa_run_sequential": (C.c_int, [_P, _P]),
    "qs_batch_free": (C.c_int, [_P]),
    "qs_batch_autotune": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "qs_batch_set_choice": (C.c_int, [_P, C.c_int]),
    "qs_batch_error": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "qs_costmodel_create": (C.c_int, [C.c_uint64, _P, C.POINTER(_P)]),
    "qs_costmodel_free": (C.c_int, [_P]),
    "qs_costmodel_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "qs_costmodel_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "qs_costmodel_train_step": (C.c_int, [_P, _P, _P, C.c_int, C.c_float, C.POINTER(C.c_float)]),
    "qs_costmodel_predict": (C.c_int, [_P, _P, _P, C.c_int]),
    "qs_costmodel_get_grads": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "qs_plan_block_features": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int)]),
    "qs_last_error": (C.c_char_p, []),
    "qs_version": (C.c_char_p, []),
}


def lib():
    """Load libqs.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqs.so is not built (run __graft_entry__.build() or "
                               "python paper_2406_14084_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != 0:
        raise QSError(rc, lib().qs_last_error().decode())


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def gate_class(targets, matrix):
    """(kind, control qubits, active targets) of a gate as the gate-by-gate
    path runs it: kind 0 dense, 1 diagonal, 2 permutation with phases."""
    t = np.ascontiguousarray(targets, dtype=np.int32)
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128)).view(np.float64)
    kind, cm, act = C.c_int(), C.c_uint64(), C.c_int()
    check(lib().qs_gate_class(len(t), _ip(t), _dp(m), C.byref(kind), C.byref(cm), C.byref(act)))
    return kind.value, [q for q in range(64) if (cm.value >> q) & 1], act.value


class State:
    """An n-qubit state vector in a torch tensor (complex128 or complex64,
    on a GPU) bound to a libqs handle and a stream."""

    def __init__(self, n, dtype="c128", device="cuda", stream=None, tensor=None, workspace=True):
        """workspace=True: a torch-owned uint8 tensor of qs_workspace_size()
        bytes is handed to the library as its scratch; False: the handle
        allocates its own."""
        torch = _torch()
        self.n = int(n)
        self.dtype = QS_C64 if dtype in ("c64", "complex64", QS_C64) else QS_C128
        tdt = torch.complex64 if self.dtype == QS_C64 else torch.complex128
        if tensor is None:
            tensor = torch.empty(1 << self.n, dtype=tdt, device=device)
        assert tensor.dtype == tdt and tensor.numel() == (1 << self.n) and tensor.is_contiguous()
        self.tensor = tensor
        self.stream = stream
        h = C.c_void_p()
        check(lib().qs_create(self.n, self.dtype, C.byref(h)))
        self.h = h
        self.workspace = None
        ws_ptr, ws_bytes = None, 0
        if workspace:
            nb = C.c_size_t()
            check(lib().qs_workspace_size(self.n, self.dtype, C.byref(nb)))
            self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=tensor.device)
            ws_ptr, ws_bytes = C.c_void_p(self.workspace.data_ptr()), nb.value
        with torch.cuda.device(tensor.device):
            check(lib().qs_attach(h, C.c_void_p(tensor.data_ptr()), tensor.numel() * tensor.element_size(),
                                  _stream_ptr(stream), ws_ptr, ws_bytes))

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            lib().qs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_zero(self):
        check(lib().qs_init_zero(self.h))
        return self

    def init_basis(self, index):
        check(lib().qs_init_basis(self.h, int(index)))
        return self

    def apply_gate(self, targets, matrix):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128)).view(np.float64)
        check(lib().qs_apply_gate(self.h, len(t), _ip(t), _dp(m)))

    def apply_circuit_gbg(self, circuit):
        for g in circuit.gates:
            self.apply_gate(g.targets, g.matrix)

    def swap_qubits(self, a, b):
        a = np.ascontiguousarray(a, dtype=np.int32)
        b = np.ascontiguousarray(b, dtype=np.int32)
        check(lib().qs_swap_qubits(self.h, len(a), _ip(a), _ip(b)))

    def apply_plan(self, plan):
        check(lib().qs_apply_plan(self.h, plan.h))

    def apply_plan_timed(self, plan):
        """Run the plan with an event around every step; returns (ms per step, kind per step: 1 block, 0 swap)."""
        ns = plan.nsteps()
        ms = (C.c_float * max(1, ns))()
        kinds = (C.c_int * max(1, ns))()
        check(lib().qs_apply_plan_timed(self.h, plan.h, ms, kinds, ns))
        return np.array(ms[:ns], dtype=np.float64), np.array(kinds[:ns], dtype=np.int32)

    def probs(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(1 << self.n, dtype=torch.float64, device=self.tensor.device)
        check(lib().qs_probs(self.h, C.c_void_p(out.data_ptr())))
        return out

    def expect(self, terms):
        """terms: iterable of (xmask, zmask, coeff)."""
        terms = list(terms)
        arr = (Pauli_C * max(1, len(terms)))()
        for i, (x, z, c) in enumerate(terms):
            arr[i] = Pauli_C(int(x), int(z), float(c))
        out = C.c_double()
        check(lib().qs_expect(self.h, len(terms), arr, C.byref(out)))
        return out.value

    def numpy(self):
        return self.tensor.cpu().numpy()

    def amplitudes(self, first=0, count=None):
        """Amplitudes [first, first + count) copied to host through the C ABI."""
        count = (1 << self.n) - first if count is None else int(count)
        out = np.empty(count, dtype=np.complex64 if self.dtype == QS_C64 else np.complex128)
        check(lib().qs_get_amplitudes(self.h, int(first), count, C.c_void_p(out.ctypes.data)))
        return out


class Plan:
    """A plan built by qs_fuse from a circuit (inputs.Circuit or anything with
    .n and .arrays())."""

    def __init__(self, circuit, kmax=5, dtype="c128", chunk_qubits=0, low_qubits=0, swaps=True, fusion=True,
                 planner=0, cost_model=None, reg_qubits=0, mfma=True, split=True):
        k, t, m = circuit.arrays()
        self._keep = (k, t, m)
        circ = Circuit_C(circuit.n, len(k), _ip(k), _ip(t), _dp(m))
        opts = PlanOpts_C(chunk_qubits, low_qubits, int(swaps), int(fusion), planner,
                          cost_model.h if cost_model is not None else None,
                          QS_C64 if dtype in ("c64", "complex64", QS_C64) else QS_C128, reg_qubits,
                          0 if mfma else 1, 0 if split else 1)
        h = C.c_void_p()
        check(lib().qs_fuse(C.byref(circ), kmax, C.byref(opts), C.byref(h)))
        self.h = h
        self.n = circuit.n
        self.ngates = len(k)

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            lib().qs_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        s = PlanStats_C()
        check(lib().qs_plan_get_stats(self.h, C.byref(s)))
        d = {f: getattr(s, f) for f, _ in PlanStats_C._fields_}
        d["ops_dense"] = list(s.ops_dense)
        return d

    def dump(self):
        need = C.c_size_t()
        check(lib().qs_plan_dump(self.h, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(lib().qs_plan_dump(self.h, buf, need.value, None))
        return buf.value.decode()

    def blocks(self):
        """[(chunk physical qubits, gate ids)] for every gate block."""
        out = []
        b = 0
        while True:
            phys = (C.c_int * 16)()
            ng = C.c_int()
            rc = lib().qs_plan_block(self.h, b, phys, None, 0, C.byref(ng))
            if rc != 0:
                break
            ids = (C.c_int * max(1, ng.value))()
            check(lib().qs_plan_block(self.h, b, phys, ids, ng.value, C.byref(ng)))
            C_ = self.stats()["chunk_qubits"]
            out.append((list(phys)[:C_], list(ids)[:ng.value]))
            b += 1
        return out

    def program(self):
        """(words int32, step offsets int64, r, C, matrices float64) of the encoded device program."""
        nw, ns, r, Cc, nm = C.c_size_t(), C.c_int(), C.c_int(), C.c_int(), C.c_size_t()
        check(lib().qs_plan_program(self.h, None, 0, C.byref(nw), None, 0, C.byref(ns), C.byref(r), C.byref(Cc),
                                    None, 0, C.byref(nm)))
        w = np.zeros(nw.value, dtype=np.int32)
        o = np.zeros(max(1, ns.value), dtype=np.int64)
        m = np.zeros(nm.value, dtype=np.float64)
        check(lib().qs_plan_program(self.h, w.ctypes.data_as(C.POINTER(C.c_int32)), nw.value, None,
                                    o.ctypes.data_as(C.POINTER(C.c_int64)), ns.value, None, None, None,
                                    _dp(m), nm.value, None))
        return w, o[:ns.value], r.value, Cc.value, m

    def features(self):
        """Cost-model features of every step (gate blocks and swap passes), (steps, 48) float32."""
        nb = C.c_int()
        check(lib().qs_plan_block_features(self.h, None, 0, C.byref(nb)))
        f = np.zeros((nb.value, COST_FEATURES), dtype=np.float32)
        check(lib().qs_plan_block_features(self.h, f.ctypes.data_as(C.POINTER(C.c_float)), nb.value, C.byref(nb)))
        return f

    def nsteps(self):
        ns = C.c_int()
        perm = (C.c_int * self.n)()
        check(lib().qs_plan_layout(self.h, 0, perm, C.byref(ns)))
        return ns.value

    def layouts(self):
        ns = C.c_int()
        perm = (C.c_int * self.n)()
        check(lib().qs_plan_layout(self.h, 0, perm, C.byref(ns)))
        out = []
        for s in range(ns.value + 1):
            check(lib().qs_plan_layout(self.h, s, perm, None))
            out.append(list(perm))
        return out


COST_FEATURES = 48
COST_PARAMS = 128 * 48 + 128 + 128 * 128 + 128 + 128 + 1


class CostModel:
    """The plan cost model (48 -> 128 -> 128 -> 1 FP32 MLP) on the GPU; its
    forward, backward and Adam steps run in the library's own kernels.
    Parameters are a flat float32 vector: W1 (128x48), b1, W2 (128x128), b2,
    W3 (1x128), b3, row-major."""

    def __init__(self, seed=0, stream=None):
        self._torch = _torch()
        self._stream = stream
        h = C.c_void_p()
        check(lib().qs_costmodel_create(int(seed), _stream_ptr(stream), C.byref(h)))
        self.h = h

    def get_params(self):
        p = np.zeros(COST_PARAMS, dtype=np.float32)
        check(lib().qs_costmodel_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float))))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != COST_PARAMS:
            raise ValueError("expected %d parameters" % COST_PARAMS)
        check(lib().qs_costmodel_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float))))

    def get_grads(self):
        g = np.zeros(COST_PARAMS, dtype=np.float32)
        check(lib().qs_costmodel_get_grads(self.h, g.ctypes.data_as(C.POINTER(C.c_float))))
        return g

    def _dev(self, a, dtype):
        torch = self._torch
        t = torch.as_tensor(a, dtype=dtype)
        return t.to("cuda").contiguous()

    def train_step(self, X, y, lr=1e-3, want_loss=True):
        """One Adam step on a minibatch (rows <= 1024); X, y: numpy or cuda tensors."""
        torch = self._torch
        Xd = X if isinstance(X, torch.Tensor) and X.is_cuda else self._dev(X, torch.float32)
        yd = y if isinstance(y, torch.Tensor) and y.is_cuda else self._dev(y, torch.float32)
        loss = C.c_float()
        check(lib().qs_costmodel_train_step(self.h, C.c_void_p(Xd.data_ptr()), C.c_void_p(yd.data_ptr()),
                                            int(Xd.shape[0]), float(lr), C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def predict(self, X):
        """Model outputs for the rows of X (float32 cuda tensor returned)."""
        torch = self._torch
        Xd = X if isinstance(X, torch.Tensor) and X.is_cuda else self._dev(X, torch.float32)
        out = torch.empty(int(Xd.shape[0]), dtype=torch.float32, device="cuda")
        check(lib().qs_costmodel_predict(self.h, C.c_void_p(Xd.data_ptr()), C.c_void_p(out.data_ptr()),
                                         int(Xd.shape[0])))
        (self._stream or torch.cuda.current_stream()).synchronize()
        return out

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            lib().qs_costmodel_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class QaoaBatch:
    """Many MaxCut QAOA instances (inputs.QaoaInstance) run by one persistent
    launch; results are <C> per instance in FP64."""

    def __init__(self, instances, dtype="c64", stream=None):
        torch = _torch()
        self.count = len(instances)
        self._keep = []
        arr = (QaoaInst_C * self.count)()
        for i, q in enumerate(instances):
            e = np.ascontiguousarray(np.array(q.edges, dtype=np.int32).reshape(-1))
            g = np.ascontiguousarray(q.gammas, dtype=np.float64)
            b = np.ascontiguousarray(q.betas, dtype=np.float64)
            self._keep += [e, g, b]
            arr[i] = QaoaInst_C(q.n, len(q.edges), len(g), _ip(e), _dp(g), _dp(b))
        self.dtype = QS_C64 if dtype in ("c64", "complex64", QS_C64) else QS_C128
        nb = C.c_size_t()
        check(lib().qs_batch_qaoa_workspace_size(self.count, arr, self.dtype, C.byref(nb)))
        # the instances' states live in a torch-owned workspace
        self.workspace = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(lib().qs_batch_qaoa_create(self.count, arr, self.dtype, _stream_ptr(stream),
                                         C.c_void_p(self.workspace.data_ptr()) if nb.value else None, nb.value,
                                         C.byref(h)))
        self.h = h
        self.out = torch.zeros(self.count, dtype=torch.float64, device="cuda")

    def run(self, graph=False):
        check(lib().qs_batch_qaoa_run(self.h, C.c_void_p(self.out.data_ptr()), int(graph)))
        return self.out

    def run_sequential(self, out=None):
        out = self.out if out is None else out
        check(lib().qs_batch_qaoa_run_sequential(self.h, C.c_void_p(out.data_ptr())))
        return out

    def autotune(self):
        ch = C.c_int()
        ms = C.c_double()
        check(lib().qs_batch_autotune(self.h, C.byref(ch), C.byref(ms)))
        return ch.value, ms.value

    def set_choice(self, choice):
        check(lib().qs_batch_set_choice(self.h, int(choice)))

    def error(self):
        e = C.c_int()
        check(lib().qs_batch_error(self.h, C.byref(e)))
        return e.value

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            lib().qs_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
