"""O5: matrix-product-state simulator in complex128 (Sec. 3.2).

A one-qubit gate is absorbed into its site tensor.  A two-qubit gate on
neighbouring sites (i, i+1) follows the paper's steps: merge the two site
tensors with the rank-4 gate, split the result by a singular value
decomposition, truncate the bond between the two new tensors, update.

Readings where the paper is silent (fixed here and in the native library):
    * site tensors have shape (chi_left, 2, chi_right); the state is
      |0...0> initially (all bonds 1);
    * an orthogonality centre is kept, because truncating singular values is
      optimal only when the rest of the chain is orthonormal: before a gate
      the centre is moved onto the gate's pair by QR factorisations (moving
      right: A_c = QR, A_c <- Q, A_{c+1} <- R A_{c+1}; moving left: the
      same on the conjugate transpose);
    * singular values are kept while s / s_max > cutoff, at most chi_max of
      them, in descending order; the kept values are rescaled to unit norm;
      the discarded weight is (sum of dropped s^2) / (sum of all s^2);
    * S is absorbed to the right (centre ends on site i+1) when the centre
      was at or left of site i before the gate, otherwise to the left
      (centre ends on site i).

Parity pins (tests): without truncation the MPS equals the state vector
(O1); for one truncated gate ||theta - theta_kept||^2 equals the dropped
singular-value weight (Eckart-Young); the norm stays 1.
"""

from __future__ import annotations

import math
from typing import List

import numpy as np

from .gates import gate_matrix, is_channel


class MPS:
    def __init__(self, n: int):
        self.n = n
        self.sites: List[np.ndarray] = []
        for _ in range(n):
            A = np.zeros((1, 2, 1), dtype=np.complex128)
            A[0, 0, 0] = 1.0
            self.sites.append(A)
        self.center = 0
        # bond i: kept, renormalised singular values of its last SVD, and
        # per two-qubit gate the relative gap s_keep / s_(keep+1) - 1 at the
        # truncation cut (inf when nothing was cut)
        self.spectra: List[np.ndarray] = [np.ones(1) for _ in range(n - 1)]
        self.cut_gaps: List[float] = []

    # ---------------------------------------------------------------- gauge
    def _move_right(self, c: int):
        A = self.sites[c]
        l, d, r = A.shape
        Q, R = np.linalg.qr(A.reshape(l * d, r))
        k = Q.shape[1]
        self.sites[c] = Q.reshape(l, d, k)
        self.sites[c + 1] = np.tensordot(R, self.sites[c + 1], axes=([1], [0]))
        self.center = c + 1

    def _move_left(self, c: int):
        A = self.sites[c]
        l, d, r = A.shape
        Q, R = np.linalg.qr(A.reshape(l, d * r).conj().T)      # A^dagger = Q R
        k = Q.shape[1]
        self.sites[c] = Q.conj().T.reshape(k, d, r)               # A = R^dagger Q^dagger
        self.sites[c - 1] = np.tensordot(self.sites[c - 1], R.conj().T, axes=([2], [0]))
        self.center = c - 1

    def move_center(self, target: int):
        while self.center < target:
            self._move_right(self.center)
        while self.center > target:
            self._move_left(self.center)

    # ---------------------------------------------------------------- gates
    def apply_gate1(self, site: int, U: np.ndarray):
        self.sites[site] = np.einsum("ts,lsr->ltr", U, self.sites[site])

    def apply_gate2(self, site: int, U: np.ndarray, chi_max: int, cutoff: float = 1e-12) -> float:
        right = self.center <= site
        target = site if self.center <= site else site + 1
        self.move_center(target)
        A, B = self.sites[site], self.sites[site + 1]
        l, r = A.shape[0], B.shape[2]
        theta = np.tensordot(A, B, axes=([2], [0]))                      # l, s1, s2, r
        G = U.reshape(2, 2, 2, 2)                                         # t1, t2, s1, s2
        theta = np.einsum("abst,lstr->labr", G, theta)
        M = theta.reshape(l * 2, 2 * r)
        Um, S, Vh = np.linalg.svd(M, full_matrices=False)
        smax = S[0] if S.size else 0.0
        keep = int(np.sum(S > cutoff * smax)) if smax > 0 else 1
        keep = max(1, min(keep, chi_max))
        total = float(np.sum(S ** 2))
        kept = float(np.sum(S[:keep] ** 2))
        discarded = (total - kept) / total if total > 0 else 0.0
        Sk = S[:keep] / np.sqrt(kept)
        self.spectra[site] = Sk.copy()
        self.cut_gaps.append(float(S[keep - 1] / S[keep] - 1.0) if keep < S.size and S[keep] > 0 else math.inf)
        if right:
            self.sites[site] = Um[:, :keep].reshape(l, 2, keep)
            self.sites[site + 1] = (Sk[:, None] * Vh[:keep]).reshape(keep, 2, r)
            self.center = site + 1
        else:
            self.sites[site] = (Um[:, :keep] * Sk[None, :]).reshape(l, 2, keep)
            self.sites[site + 1] = Vh[:keep].reshape(keep, 2, r)
            self.center = site
        return discarded

    # ----------------------------------------------------------- observables
    def bond_dims(self) -> List[int]:
        return [A.shape[2] for A in self.sites[:-1]]

    def amplitude(self, bits) -> complex:
        v = np.ones((1,), dtype=np.complex128)
        for A, b in zip(self.sites, bits):
            v = v @ A[:, int(b), :]
        return complex(v[0])

    def expect_z(self) -> np.ndarray:
        """<Z_i> from left environments, without changing the gauge."""
        n = self.n
        Ls = [np.ones((1, 1), dtype=np.complex128)]
        for A in self.sites:
            Ls.append(np.einsum("ab,asr,bst->rt", Ls[-1], A.conj(), A, optimize=True))
        Rs = [np.ones((1, 1), dtype=np.complex128)]
        for A in reversed(self.sites):
            Rs.append(np.einsum("asr,bst,rt->ab", A.conj(), A, Rs[-1], optimize=True))
        Rs = Rs[::-1]
        norm = Ls[-1][0, 0].real
        z = np.empty(n)
        zsign = np.array([1.0, -1.0])
        for i, A in enumerate(self.sites):
            z[i] = np.einsum("ab,asr,bst,rt,s->", Ls[i], A.conj(), A, Rs[i + 1], zsign, optimize=True).real / norm
        return z

    def to_statevector(self) -> np.ndarray:
        psi = self.sites[0]
        for A in self.sites[1:]:
            psi = np.tensordot(psi, A, axes=([psi.ndim - 1], [0]))
        return psi.reshape((2,) * self.n)


def run_circuit(n: int, ops, chi_max: int, cutoff: float = 1e-12):
    """Apply a nearest-neighbour circuit; returns (mps, total discarded weight)."""
    m = MPS(n)
    disc = 0.0
    for op in ops:
        if is_channel(op.name):
            raise ValueError("MPS oracle is noiseless")
        U = gate_matrix(op.name, op.params)
        if len(op.qubits) == 1:
            m.apply_gate1(op.qubits[0], U)
        else:
            a, b = op.qubits
            if b != a + 1:
                raise ValueError("MPS needs nearest-neighbour gates (a, a+1)")
            disc += m.apply_gate2(a, U, chi_max, cutoff)
    return m, disc
