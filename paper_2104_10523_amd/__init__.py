"""Python binding of the MI355X tensor-network simulator (libtn.so).

Functions carry the C ABI's names and only marshal arguments: device
buffers are torch tensors, streams are torch streams, every computation runs
in the native library.  There is no CPU fallback: without the built library
every call raises.
"""

from __future__ import annotations

import ctypes as C
from typing import Iterable, List, Optional, Sequence

import numpy as np

from ._native import (GATE_IDS, PATH_ALGO, PAULI, PREC, TnCircuit, TnExecOpts, TnNetworkInfo, TnOp,
                      TnPathCost, TnPathOpts, TnPlanInfo, TnReport, TnTensor, TnError, check, lib)

__all__ = ["Network", "Path", "Mps", "Pmps", "TnError", "tn_pmps_create", "tn_build_network", "tn_find_path",
           "tn_path_from_pairs", "tn_contract_pair", "tn_amplitudes", "tn_set_workspace",
           "tn_amplitudes_workspace", "tn_build_expectation_network", "tn_build_density_network",
           "tn_pauli_expectation", "tn_sample_amplitudes",
           "tn_mps_create", "tn_mps_apply_gate", "tn_run_trajectories", "PREC", "lib"]


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class _CircuitArgs:
    """Keeps the ctypes op array (and custom matrices) alive for one call."""

    def __init__(self, n_qubits: int, ops: Iterable):
        ops = list(ops)
        self.arr = (TnOp * max(len(ops), 1))()
        self.keep = []
        for i, op in enumerate(ops):
            name, qubits, params = op[0], tuple(op[1]), tuple(op[2]) if len(op) > 2 else ()
            o = self.arr[i]
            o.gate = GATE_IDS[name] if isinstance(name, str) else int(name)
            o.q0 = int(qubits[0])
            o.q1 = int(qubits[1]) if len(qubits) > 1 else -1
            mat = None
            if name in ("custom1", "custom2"):
                mat = np.ascontiguousarray(np.asarray(params[0], dtype=np.complex128)).view(np.float64)
                self.keep.append(mat)
                o.matrix = mat.ctypes.data_as(C.POINTER(C.c_double))
            else:
                for k, v in enumerate(params[:2]):
                    o.param[k] = float(v)
        self.circ = TnCircuit(int(n_qubits), len(ops), self.arr)


class Network:
    def __init__(self, handle: int, n_qubits: int):
        self.h = C.c_void_p(handle)
        self.n_qubits = n_qubits

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            try:
                lib().tn_network_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def info(self) -> TnNetworkInfo:
        info = TnNetworkInfo()
        check(lib().tn_network_get_info(self.h, C.byref(info)))
        return info

    def tensor(self, i: int):
        rank = C.c_int32()
        check(lib().tn_network_get_tensor(self.h, i, C.byref(rank), None, None))
        labels = (C.c_int32 * max(rank.value, 1))()
        data = np.zeros(2 * (1 << rank.value), dtype=np.float64)
        check(lib().tn_network_get_tensor(self.h, i, C.byref(rank), labels,
                                          data.ctypes.data_as(C.POINTER(C.c_double))))
        return data.view(np.complex128).reshape((2,) * rank.value), list(labels)[:rank.value]

    def output_labels(self) -> List[int]:
        out = (C.c_int32 * self.n_qubits)()
        check(lib().tn_network_output_labels(self.h, out))
        return list(out)


class Path:
    def __init__(self, handle: int, cost: TnPathCost):
        self.h = C.c_void_p(handle)
        self.cost = cost

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().tn_path_destroy(self.h)
            except Exception:
                pass
            self.h = None

    @property
    def pairs(self) -> List[tuple]:
        n = self.cost.n_steps
        buf = (C.c_int32 * max(2 * n, 1))()
        check(lib().tn_path_get(self.h, buf, None))
        return [(buf[2 * t], buf[2 * t + 1]) for t in range(n)]

    @property
    def sliced(self) -> List[int]:
        n = self.cost.n_sliced
        buf = (C.c_int32 * max(n, 1))()
        check(lib().tn_path_get(self.h, None, buf))
        return list(buf)[:n]


def tn_build_network(n_qubits: int, ops) -> Network:
    ca = _CircuitArgs(n_qubits, ops)
    h = C.c_void_p()
    check(lib().tn_build_network(C.byref(ca.circ), C.byref(h)))
    return Network(h.value, n_qubits)


def _path_opts(n_qubits, algo, trials, seed, temperature, budget, open_mask):
    o = TnPathOpts()
    o.algo = PATH_ALGO[algo] if isinstance(algo, str) else int(algo)
    o.trials = int(trials)
    o.seed = int(seed)
    o.temperature = float(temperature)
    o.mem_budget_bytes = float(budget)
    keep = None
    if open_mask is not None:
        keep = np.ascontiguousarray(np.asarray(open_mask, dtype=np.int8))
        assert keep.size == n_qubits
        o.open_mask = keep.ctypes.data_as(C.POINTER(C.c_int8))
    return o, keep


def tn_find_path(net: Network, algo: str = "greedy", trials: int = 32, seed: int = 0,
                 temperature: float = 1.0, mem_budget_bytes: float = 0.0,
                 open_mask: Optional[Sequence[int]] = None, rank: str = "flops",
                 rank_precision: str = "auto") -> Path:
    """rank = "time" re-ranks the partition search's best candidates by the
    modelled kernel time of their amplitude plans at rank_precision."""
    o, _keep = _path_opts(net.n_qubits, algo, trials, seed, temperature, mem_budget_bytes, open_mask)
    o.rank = {"flops": 0, "time": 1}[rank]
    o.rank_precision = PREC[rank_precision]
    h = C.c_void_p()
    cost = TnPathCost()
    check(lib().tn_find_path(net.h, C.byref(o), C.byref(h), C.byref(cost)))
    return Path(h.value, cost)


def tn_path_from_pairs(net: Network, pairs, mem_budget_bytes: float = 0.0,
                       open_mask: Optional[Sequence[int]] = None) -> Path:
    o, _keep = _path_opts(net.n_qubits, 0, 0, 0, 1.0, mem_budget_bytes, open_mask)
    flat = (C.c_int32 * max(2 * len(pairs), 1))(*[int(x) for p in pairs for x in p])
    h = C.c_void_p()
    cost = TnPathCost()
    check(lib().tn_path_from_pairs(net.h, C.byref(o), flat, len(pairs), C.byref(h), C.byref(cost)))
    return Path(h.value, cost)


def tn_set_workspace(buf) -> None:
    """Register a device buffer (a torch tensor, kept alive by the caller)."""
    if buf is None:
        check(lib().tn_set_workspace(None, 0))
    else:
        check(lib().tn_set_workspace(C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))


def _tensor(t, extents=None) -> tuple:
    import torch
    assert t.dtype in (torch.complex64, torch.complex128) and t.is_cuda and t.is_contiguous()
    ext = list(t.shape) if extents is None else list(extents)
    arr = (C.c_int64 * max(len(ext), 1))(*ext)
    T = TnTensor(C.c_void_p(t.data_ptr()), len(ext), 0 if t.dtype == torch.complex64 else 1, arr)
    return T, arr


def tn_contract_pair(A, modesA, B, modesB, Cout, modesC, precision: str = "fp32", stream=None,
                     noalloc: bool = False):
    """Cout[modesC] = sum A[modesA] * B[modesB] (einsum semantics), on the GPU.
    noalloc=True calls tn_contract_pair_noalloc (scratch inside the library,
    at most 64 MiB, no workspace needed)."""
    TA, ka = _tensor(A)
    TB, kb = _tensor(B)
    TC, kc = _tensor(Cout)
    ma = (C.c_int32 * max(len(modesA), 1))(*modesA)
    mb = (C.c_int32 * max(len(modesB), 1))(*modesB)
    mc = (C.c_int32 * max(len(modesC), 1))(*modesC)
    fn = lib().tn_contract_pair_noalloc if noalloc else lib().tn_contract_pair
    check(fn(C.byref(TA), ma, C.byref(TB), mb, C.byref(TC), mc,
             PREC[precision] if isinstance(precision, str) else int(precision),
             C.c_void_p(_stream_ptr(stream))))


def tn_amplitudes_workspace(net: Network, path: Path, n_bs: int, precision: str = "fp32") -> int:
    n = C.c_size_t()
    check(lib().tn_amplitudes_workspace(net.h, path.h, int(n_bs), PREC[precision], C.byref(n)))
    return n.value


def tn_amplitudes_autotune(net: Network, path: Path, precision: str = "fp32", reps: int = 2,
                           stream=None) -> None:
    """Time the candidate GEMM tiles of this path's plan and keep the fastest."""
    check(lib().tn_amplitudes_autotune(net.h, path.h, PREC[precision], int(reps),
                                       C.c_void_p(_stream_ptr(stream))))


def tn_amplitudes_plan_info(net: Network, path: Path, precision: str = "fp32"):
    """Summary of one job's kernel sequence (a TnPlanInfo struct)."""
    info = TnPlanInfo()
    check(lib().tn_amplitudes_plan_info(net.h, path.h, PREC[precision], C.byref(info)))
    return info


def tn_amplitudes_plan_ops(net: Network, path: Path, precision: str = "fp32"):
    """Per-op detail of one job: (kind, flops, bytes, shape) numpy arrays,
    shape n_ops x 8 (m, n, k, batch, block-tile id, packed, launches, 0)."""
    n_ops = tn_amplitudes_plan_info(net, path, precision).n_ops
    kind = (C.c_int32 * n_ops)()
    fl = (C.c_double * n_ops)()
    by = (C.c_double * n_ops)()
    shape = (C.c_int64 * (8 * n_ops))()
    check(lib().tn_amplitudes_plan_ops(net.h, path.h, PREC[precision], kind, fl, by, shape))
    return (np.array(kind), np.array(fl), np.array(by), np.array(shape).reshape(n_ops, 8))


def tn_amplitudes(net: Network, path: Path, bits, out=None, precision: str = "fp32",
                  use_graph: bool = False, slice_begin: int = 0, slice_count: int = -1,
                  accumulate: bool = False, sync: bool = True, stream=None):
    """Amplitudes of bit-strings (int array n_bs x n_qubits with 0/1/-1).

    Returns (out, report): out is a complex128 CUDA tensor n_bs x 2^#open.
    """
    import torch
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.int8))
    if b.ndim == 1:
        b = b[None, :]
    n_bs = b.shape[0]
    n_open = int((b[0] < 0).sum())
    if out is None:
        out = torch.zeros((n_bs, 1 << n_open), dtype=torch.complex128, device="cuda")
    o = TnExecOpts(PREC[precision], int(use_graph), int(slice_begin), int(slice_count),
                   int(accumulate), int(sync))
    rep = TnReport()
    check(lib().tn_amplitudes(net.h, path.h, b.ctypes.data_as(C.POINTER(C.c_int8)), n_bs,
                              C.byref(o), C.c_void_p(out.data_ptr()), C.byref(rep),
                              C.c_void_p(_stream_ptr(stream))))
    return out, rep


def _pauli_array(n_qubits: int, pauli) -> np.ndarray:
    """Pauli string as int8 TN_PAULI_* codes: a string like "IZZI", a dict
    {qubit: "X"|"Y"|"Z"}, or a sequence of codes 0..3."""
    if isinstance(pauli, str):
        assert len(pauli) == n_qubits
        arr = [PAULI[c] for c in pauli.upper()]
    elif isinstance(pauli, dict):
        arr = [0] * n_qubits
        for q, c in pauli.items():
            arr[int(q)] = PAULI[c.upper()] if isinstance(c, str) else int(c)
    else:
        arr = list(pauli)
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.int8))
    assert a.size == n_qubits
    return a


def tn_build_expectation_network(n_qubits: int, ops, pauli):
    """Double-depth network of <Psi|P|Psi> after the light-cone collapse.

    Returns (network, number of gates of the circuit that were kept)."""
    ca = _CircuitArgs(n_qubits, ops)
    p = _pauli_array(n_qubits, pauli)
    h = C.c_void_p()
    kept = C.c_int64()
    check(lib().tn_build_expectation_network(C.byref(ca.circ), p.ctypes.data_as(C.POINTER(C.c_int8)),
                                             C.byref(h), C.byref(kept)))
    return Network(h.value, n_qubits), int(kept.value)


def tn_build_density_network(n_qubits: int, ops, pauli):
    """Density-matrix network of Tr(rho P) for a circuit that may hold
    channels; a closed network (no output legs).

    Returns (network, number of ops of the circuit that were kept)."""
    ca = _CircuitArgs(n_qubits, ops)
    p = _pauli_array(n_qubits, pauli)
    h = C.c_void_p()
    kept = C.c_int64()
    check(lib().tn_build_density_network(C.byref(ca.circ), p.ctypes.data_as(C.POINTER(C.c_int8)),
                                         C.byref(h), C.byref(kept)))
    return Network(h.value, 0), int(kept.value)


def tn_sample_amplitudes(psi, uniforms, stream=None):
    """Indices drawn with probability |psi_k|^2 / sum |psi|^2 at the given
    uniforms (psi: a contiguous complex128 CUDA tensor).  Returns
    (indices int64 array, sum |psi|^2)."""
    u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64).reshape(-1))
    out = np.zeros(u.size, dtype=np.int64)
    assert psi.is_contiguous() and psi.dtype.is_complex
    tot = C.c_double()
    check(lib().tn_sample_amplitudes(C.c_void_p(psi.data_ptr()), psi.numel(), u.ctypes.data_as(C.POINTER(C.c_double)),
                                     u.size, out.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(tot),
                                     C.c_void_p(_stream_ptr(stream))))
    return out, float(tot.value)


def tn_pauli_expectation(psi, bits, pauli, stream=None) -> complex:
    """sum_s <psi_s|P|psi_s> over wave-function slices: psi is the complex128
    CUDA tensor tn_amplitudes returned for the bit-strings `bits`."""
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.int8))
    if b.ndim == 1:
        b = b[None, :]
    n_slices, n_qubits = b.shape
    p = _pauli_array(n_qubits, pauli)
    assert psi.is_contiguous() and psi.shape[0] == n_slices
    out = (C.c_double * 2)()
    check(lib().tn_pauli_expectation(C.c_void_p(psi.data_ptr()), b.ctypes.data_as(C.POINTER(C.c_int8)),
                                     n_slices, n_qubits, p.ctypes.data_as(C.POINTER(C.c_int8)), out,
                                     C.c_void_p(_stream_ptr(stream))))
    return complex(out[0], out[1])


class Mps:
    def __init__(self, handle: int, n: int):
        self.h = C.c_void_p(handle)
        self.n = n

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().tn_mps_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def apply_gate1(self, site: int, U, stream=None):
        u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128)).view(np.float64)
        check(lib().tn_mps_apply_gate1(self.h, int(site), u.ctypes.data_as(C.POINTER(C.c_double)),
                                       C.c_void_p(_stream_ptr(stream))))

    def bond_dims(self) -> List[int]:
        out = (C.c_int32 * max(self.n - 1, 1))()
        check(lib().tn_mps_bond_dims(self.h, out))
        return list(out)[:self.n - 1]

    def bond_spectrum(self, bond: int) -> np.ndarray:
        """Kept, renormalised singular values of the last gate on `bond`."""
        cnt = C.c_int32()
        check(lib().tn_mps_bond_spectrum(self.h, int(bond), None, 0, C.byref(cnt)))
        out = np.zeros(max(cnt.value, 1))
        check(lib().tn_mps_bond_spectrum(self.h, int(bond), out.ctypes.data_as(C.POINTER(C.c_double)),
                                         cnt.value, C.byref(cnt)))
        return out[:cnt.value]

    def expect_z(self, stream=None) -> np.ndarray:
        out = np.zeros(self.n)
        check(lib().tn_mps_expect_z(self.h, out.ctypes.data_as(C.POINTER(C.c_double)),
                                    C.c_void_p(_stream_ptr(stream))))
        return out

    def amplitudes(self, bits, stream=None) -> np.ndarray:
        b = np.ascontiguousarray(np.asarray(bits, dtype=np.int8))
        if b.ndim == 1:
            b = b[None, :]
        out = np.zeros(2 * b.shape[0])
        check(lib().tn_mps_amplitudes(self.h, b.ctypes.data_as(C.POINTER(C.c_int8)), b.shape[0],
                                      out.ctypes.data_as(C.POINTER(C.c_double)),
                                      C.c_void_p(_stream_ptr(stream))))
        return out.view(np.complex128)


def tn_mps_create(n_sites: int, chi_max: int, stream=None) -> Mps:
    h = C.c_void_p()
    check(lib().tn_mps_create(int(n_sites), int(chi_max), C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return Mps(h.value, n_sites)


def tn_mps_apply_gate(mps: Mps, site: int, U, chi_max: int, cutoff: float = 1e-12, stream=None) -> float:
    """Two-qubit gate on (site, site+1); returns the discarded weight."""
    u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128)).view(np.float64)
    disc = C.c_double()
    check(lib().tn_mps_apply_gate(mps.h, int(site), u.ctypes.data_as(C.POINTER(C.c_double)),
                                  int(chi_max), float(cutoff), C.byref(disc),
                                  C.c_void_p(_stream_ptr(stream))))
    return disc.value


class Pmps:
    """Locally-purified MPS handle (tn_pmps_*)."""

    def __init__(self, handle: int, n: int):
        self.h = C.c_void_p(handle)
        self.n = n

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().tn_pmps_destroy(self.h)
            except Exception:
                pass
            self.h = None

    @staticmethod
    def _mat(U):
        u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128)).view(np.float64)
        return u, u.ctypes.data_as(C.POINTER(C.c_double))

    def apply_gate1(self, site: int, U, stream=None):
        u, pu = self._mat(U)
        check(lib().tn_pmps_apply_gate1(self.h, int(site), pu, C.c_void_p(_stream_ptr(stream))))

    def apply_gate(self, site: int, U, cutoff: float = 1e-12, stream=None) -> float:
        u, pu = self._mat(U)
        d = C.c_double()
        check(lib().tn_pmps_apply_gate(self.h, int(site), pu, float(cutoff), C.byref(d),
                                       C.c_void_p(_stream_ptr(stream))))
        return d.value

    def apply_channel(self, site: int, kraus, cutoff: float = 1e-12, stream=None):
        """kraus: list of 2x2 or 4x4 matrices; returns (discarded bond, discarded Kraus)."""
        ks = [np.asarray(k, dtype=np.complex128) for k in kraus]
        nq = 1 if ks[0].shape == (2, 2) else 2
        u, pu = self._mat(np.stack(ks))
        db, dk = C.c_double(), C.c_double()
        check(lib().tn_pmps_apply_channel(self.h, int(site), nq, pu, len(ks), float(cutoff), C.byref(db),
                                          C.byref(dk), C.c_void_p(_stream_ptr(stream))))
        return db.value, dk.value

    def dims(self):
        b = (C.c_int32 * max(self.n - 1, 1))()
        k = (C.c_int32 * self.n)()
        check(lib().tn_pmps_dims(self.h, b, k))
        return list(b)[:self.n - 1], list(k)

    def expect_z(self, stream=None) -> np.ndarray:
        out = np.zeros(self.n)
        check(lib().tn_pmps_expect_z(self.h, out.ctypes.data_as(C.POINTER(C.c_double)),
                                     C.c_void_p(_stream_ptr(stream))))
        return out

    def site(self, i: int, stream=None) -> np.ndarray:
        dims = (C.c_int32 * 4)()
        check(lib().tn_pmps_get_site(self.h, int(i), None, dims, C.c_void_p(_stream_ptr(stream))))
        shape = tuple(dims)
        out = np.zeros(2 * int(np.prod(shape)))
        check(lib().tn_pmps_get_site(self.h, int(i), out.ctypes.data_as(C.POINTER(C.c_double)), dims,
                                     C.c_void_p(_stream_ptr(stream))))
        return out.view(np.complex128).reshape(shape)


def tn_pmps_create(n_sites: int, d_max: int, k_max: int, stream=None) -> Pmps:
    h = C.c_void_p()
    check(lib().tn_pmps_create(int(n_sites), int(d_max), int(k_max), C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return Pmps(h.value, n_sites)


def tn_run_trajectories(circuits, traj_per_circ: int, uniforms, stream=None):
    """circuits: list of (n_qubits, ops) with channels; uniforms: (n_traj, n_events) float64.

    Returns (z, report) with z of shape (n_traj, n_qubits).
    """
    args = [_CircuitArgs(n, ops) for n, ops in circuits]
    arr = (C.POINTER(TnCircuit) * len(args))(*[C.pointer(a.circ) for a in args])
    u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
    n_traj = len(args) * traj_per_circ
    nq = circuits[0][0]
    z = np.zeros((n_traj, nq))
    rep = TnReport()
    check(lib().tn_run_trajectories(arr, len(args), int(traj_per_circ),
                                    u.ctypes.data_as(C.POINTER(C.c_double)), u.shape[1],
                                    z.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep),
                                    C.c_void_p(_stream_ptr(stream))))
    return z, rep


class Model:
    """Learned contraction-order scorer (see include/tn.h)."""

    def __init__(self, hidden: int = 128, layers: int = 4):
        h = C.c_void_p()
        check(lib().tn_model_create(int(hidden), int(layers), C.byref(h)))
        self.h = h
        self.hidden, self.layers = hidden, layers

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().tn_model_destroy(self.h)
            except Exception:
                pass
            self.h = None

    @property
    def n_params(self) -> int:
        n = C.c_int64()
        check(lib().tn_model_n_params(self.h, C.byref(n)))
        return n.value

    def set_params(self, theta) -> None:
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        assert t.size == self.n_params
        check(lib().tn_model_set_params(self.h, t.ctypes.data_as(C.POINTER(C.c_double))))

    def get_params(self) -> np.ndarray:
        t = np.zeros(self.n_params)
        check(lib().tn_model_get_params(self.h, t.ctypes.data_as(C.POINTER(C.c_double))))
        return t

    def loss_grad(self, X, nbrs, label, stream=None):
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
        nc = X.shape[0]
        ptr = np.zeros(nc + 1, dtype=np.int32)
        for k, nb in enumerate(nbrs):
            ptr[k + 1] = ptr[k] + len(nb)
        idx = np.array([j for nb in nbrs for j in nb] or [0], dtype=np.int32)
        loss = C.c_double()
        grad = np.zeros(self.n_params)
        scores = np.zeros(nc)
        check(lib().tn_model_loss_grad(self.h, nc, X.ctypes.data_as(C.POINTER(C.c_double)),
                                       ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                                       idx.ctypes.data_as(C.POINTER(C.c_int32)), int(label), C.byref(loss),
                                       grad.ctypes.data_as(C.POINTER(C.c_double)),
                                       scores.ctypes.data_as(C.POINTER(C.c_double)),
                                       C.c_void_p(_stream_ptr(stream))))
        return loss.value, grad, scores

    def add_teacher(self, net: Network, pairs, stride: int = 1, open_mask=None) -> None:
        flat = (C.c_int32 * (2 * len(pairs)))(*[int(x) for p in pairs for x in p])
        om = None if open_mask is None else np.ascontiguousarray(np.asarray(open_mask, dtype=np.int8))
        check(lib().tn_model_add_teacher(self.h, net.h, None if om is None else om.ctypes.data_as(C.POINTER(C.c_int8)),
                                         flat, len(pairs), int(stride)))

    def train(self, epochs: int, batch: int = 16, lr: float = 1e-3, seed: int = 0, stream=None):
        lf, ll = C.c_double(), C.c_double()
        check(lib().tn_model_train(self.h, int(epochs), int(batch), float(lr), int(seed), C.byref(lf),
                                   C.byref(ll), C.c_void_p(_stream_ptr(stream))))
        return lf.value, ll.value


def tn_model_state_features(net: Network, pairs, n_prefix: int, open_mask=None):
    """(candidates, X, neighbour lists) of the state after n_prefix steps."""
    flat = (C.c_int32 * max(2 * len(pairs), 1))(*[int(x) for p in pairs for x in p])
    om = None if open_mask is None else np.ascontiguousarray(np.asarray(open_mask, dtype=np.int8))
    omp = None if om is None else om.ctypes.data_as(C.POINTER(C.c_int8))
    nc, nn = C.c_int32(), C.c_int32()
    check(lib().tn_model_state_features(net.h, omp, flat, int(n_prefix), C.byref(nc), C.byref(nn),
                                        None, None, None, None))
    cand = np.zeros(2 * nc.value, dtype=np.int32)
    X = np.zeros((nc.value, 16))
    ptr = np.zeros(nc.value + 1, dtype=np.int32)
    idx = np.zeros(max(nn.value, 1), dtype=np.int32)
    check(lib().tn_model_state_features(net.h, omp, flat, int(n_prefix), C.byref(nc), C.byref(nn),
                                        cand.ctypes.data_as(C.POINTER(C.c_int32)),
                                        X.ctypes.data_as(C.POINTER(C.c_double)),
                                        ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                                        idx.ctypes.data_as(C.POINTER(C.c_int32))))
    nbrs = [list(idx[ptr[k]:ptr[k + 1]]) for k in range(nc.value)]
    return [tuple(cand[2 * k:2 * k + 2]) for k in range(nc.value)], X, nbrs


def tn_find_path_learned(net: Network, model: Model, mem_budget_bytes: float = 0.0, open_mask=None,
                         rescore_every: int = 1) -> Path:
    """Scores the candidate pairs, takes up to rescore_every of the best
    that share no tensor, and scores again; greedy replaces the result when
    greedy is cheaper."""
    o, _keep = _path_opts(net.n_qubits, "learned", 0, 0, 1.0, mem_budget_bytes, open_mask)
    o.model = model.h
    o.rescore_every = int(rescore_every)
    h = C.c_void_p()
    cost = TnPathCost()
    check(lib().tn_find_path(net.h, C.byref(o), C.byref(h), C.byref(cost)))
    return Path(h.value, cost)
