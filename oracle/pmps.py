"""O8: locally-purified matrix product state in complex128 (Sec. 3.4, the
locally-purified MPS figure and the Kraus-contraction figure).  Test
infrastructure, like the rest of this package.

The density matrix is rho = Tr_K |X><X|: X is an MPS whose site tensors
T_i[l, s, k, r] carry, beside the physical leg s (2) and the virtual bonds l,
r (dimension D), a Kraus leg k (dimension K_i) that is summed between X and
its conjugate.  Following Sec. 3.4:

    * gates act on the physical legs as in the MPS of Sec. 3.2: a one-qubit
      gate is absorbed into its site; a two-qubit gate on (i, i+1) merges the
      two site tensors over their bond, acts on (s_i, s_i+1), and is split
      again by an SVD of the (l, s_i, k_i) x (s_i+1, k_i+1, r) matrix, which
      changes only the virtual bond D (at most d_max values kept);
    * a channel with Kraus operators {A_a} is contracted with the physical
      leg, T'[l, s, (k, a), r] = sum_s' A_a[s, s'] T[l, s', k, r], which
      multiplies the Kraus dimension by the number of operators; an SVD along
      the Kraus leg (rows (l, s, r), columns (k, a)) then brings it back to
      K' <= k_max values: T <- U S, the right factor dropping out of rho
      because the Kraus leg is traced.  A two-qubit channel acts on the
      merged pair; its Kraus index joins the Kraus leg of the first site of
      the pair before the SVD that splits the pair, and that site's Kraus leg
      is then compressed.

Readings where the paper is silent (the MPS readings of oracle/mps.py carry
over: orthogonality centre moved by QR factorisations over the combined
(s, k) leg, singular values kept while s / s_max > cutoff and at most the
maximum, kept values rescaled to unit norm, discarded weight = dropped
sum s^2 / sum s^2):
    * the Kraus leg is compressed at the orthogonality centre, so its
      singular values are those of the whole purification and Tr rho stays 1;
    * the combined leg index is s * K + k (the physical bit most significant);
    * a channel on one qubit is applied without moving the Kraus index
      elsewhere; every site starts with K = 1 (|0><0|).

Parity pins (tests): without truncation rho equals the density-matrix
oracle (O3) for noisy circuits, and |psi><psi| of the state vector (O1) for
noiseless ones; Tr rho = 1; compressing the Kraus leg with every non-zero
singular value kept leaves rho unchanged while K' never exceeds the rank
bound 2 * D_l * D_r; <Z_i> from the network equals Tr(rho Z_i) of the
contracted density matrix.
"""

from __future__ import annotations

import math
from typing import List

import numpy as np

from .gates import gate_matrix, is_channel, kraus_ops


class PMPS:
    def __init__(self, n: int):
        self.n = n
        self.sites: List[np.ndarray] = []        # (D_l, 2, K, D_r)
        for _ in range(n):
            T = np.zeros((1, 2, 1, 1), dtype=np.complex128)
            T[0, 0, 0, 0] = 1.0
            self.sites.append(T)
        self.center = 0

    # ---------------------------------------------------------------- gauge
    def _move_right(self, c: int):
        T = self.sites[c]
        l, d, k, r = T.shape
        Q, R = np.linalg.qr(T.reshape(l * d * k, r))
        m = Q.shape[1]
        self.sites[c] = Q.reshape(l, d, k, m)
        self.sites[c + 1] = np.tensordot(R, self.sites[c + 1], axes=([1], [0]))
        self.center = c + 1

    def _move_left(self, c: int):
        T = self.sites[c]
        l, d, k, r = T.shape
        Q, R = np.linalg.qr(T.reshape(l, d * k * r).conj().T)      # T^dagger = Q R
        m = Q.shape[1]
        self.sites[c] = Q.conj().T.reshape(m, d, k, r)              # T = R^dagger Q^dagger
        self.sites[c - 1] = np.tensordot(self.sites[c - 1], R.conj().T, axes=([3], [0]))
        self.center = c - 1

    def move_center(self, target: int):
        while self.center < target:
            self._move_right(self.center)
        while self.center > target:
            self._move_left(self.center)

    # ---------------------------------------------------------------- truncation
    @staticmethod
    def _keep(S: np.ndarray, cap: int, cutoff: float):
        smax = S[0] if S.size else 0.0
        keep = int(np.sum(S > cutoff * smax)) if smax > 0 else 1
        keep = max(1, min(keep, cap))
        total = float(np.sum(S ** 2))
        kept = float(np.sum(S[:keep] ** 2))
        discarded = (total - kept) / total if total > 0 else 0.0
        return keep, discarded, math.sqrt(kept) if kept > 0 else 1.0

    def _compress_kraus(self, site: int, k_max: int, cutoff: float) -> float:
        """SVD along the Kraus leg of the centre site: T[(l, s, r), k] = U S V^dagger,
        T <- U S truncated."""
        assert self.center == site
        T = self.sites[site]
        l, d, k, r = T.shape
        M = np.transpose(T, (0, 1, 3, 2)).reshape(l * d * r, k)
        U, S, _ = np.linalg.svd(M, full_matrices=False)
        keep, disc, norm = self._keep(S, k_max, cutoff)
        Mk = U[:, :keep] * (S[:keep] / norm)[None, :]
        self.sites[site] = np.transpose(Mk.reshape(l, d, r, keep), (0, 1, 3, 2))
        return disc

    # ---------------------------------------------------------------- gates
    def apply_gate1(self, site: int, U: np.ndarray):
        self.sites[site] = np.einsum("ts,lskr->ltkr", U, self.sites[site])

    def _split(self, site: int, theta: np.ndarray, right: bool, d_max: int, cutoff: float) -> float:
        """theta[l, s1, k1, s2, k2, r] -> two sites, bond truncated to d_max."""
        l, _, k1, _, k2, r = theta.shape
        Mt = theta.reshape(l * 2 * k1, 2 * k2 * r)
        Um, S, Vh = np.linalg.svd(Mt, full_matrices=False)
        keep, disc, norm = self._keep(S, d_max, cutoff)
        Sk = S[:keep] / norm
        if right:
            self.sites[site] = Um[:, :keep].reshape(l, 2, k1, keep)
            self.sites[site + 1] = (Sk[:, None] * Vh[:keep]).reshape(keep, 2, k2, r)
            self.center = site + 1
        else:
            self.sites[site] = (Um[:, :keep] * Sk[None, :]).reshape(l, 2, k1, keep)
            self.sites[site + 1] = Vh[:keep].reshape(keep, 2, k2, r)
            self.center = site
        return disc

    def _merged(self, site: int):
        right = self.center <= site
        self.move_center(site if right else site + 1)
        A, B = self.sites[site], self.sites[site + 1]
        return np.tensordot(A, B, axes=([3], [0])), right        # l, s1, k1, s2, k2, r

    def apply_gate2(self, site: int, U: np.ndarray, d_max: int, cutoff: float = 1e-12) -> float:
        theta, right = self._merged(site)
        G = U.reshape(2, 2, 2, 2)                                   # t1, t2, s1, s2
        theta = np.einsum("abst,lsjtmr->lajbmr", G, theta)
        return self._split(site, theta, right, d_max, cutoff)

    def apply_channel1(self, site: int, kraus, k_max: int, cutoff: float = 1e-12) -> float:
        self.move_center(site)
        T = self.sites[site]
        l, _, k, r = T.shape
        parts = [np.einsum("ts,lskr->ltkr", A, T) for A in kraus]   # a-th block of the Kraus leg
        self.sites[site] = np.stack(parts, axis=3).reshape(l, 2, k * len(kraus), r)   # (k, a), a fastest
        return self._compress_kraus(site, k_max, cutoff)

    def apply_channel2(self, site: int, kraus, d_max: int, k_max: int, cutoff: float = 1e-12):
        """Returns (discarded weight of the bond split, of the Kraus compression)."""
        theta, _ = self._merged(site)
        l, _, k1, _, k2, r = theta.shape
        parts = [np.einsum("abst,lsjtmr->lajbmr", A.reshape(2, 2, 2, 2), theta) for A in kraus]
        # Kraus index a joins site's Kraus leg: (k1, a), a fastest
        th = np.stack(parts, axis=3).reshape(l, 2, k1 * len(kraus), 2, k2, r)
        disc = self._split(site, th, False, d_max, cutoff)          # centre ends on site
        return disc, self._compress_kraus(site, k_max, cutoff)

    # ----------------------------------------------------------- observables
    def bond_dims(self) -> List[int]:
        return [T.shape[3] for T in self.sites[:-1]]

    def kraus_dims(self) -> List[int]:
        return [T.shape[2] for T in self.sites]

    def _env(self, ops):
        """Tr(rho O_0 x ... x O_{n-1}) with O_i acting on site i's physical leg."""
        E = np.ones((1, 1), dtype=np.complex128)
        for T, O in zip(self.sites, ops):
            OT = np.einsum("ts,lskr->ltkr", O, T)
            E = np.einsum("ab,atkr,btks->rs", E, T.conj(), OT, optimize=True)
        return E[0, 0]

    def trace(self) -> float:
        return float(self._env([np.eye(2)] * self.n).real)

    def expect_z(self) -> np.ndarray:
        Z = np.diag([1.0, -1.0]).astype(np.complex128)
        I = np.eye(2, dtype=np.complex128)
        tr = self._env([I] * self.n).real
        return np.array([self._env([Z if j == i else I for j in range(self.n)]).real / tr
                         for i in range(self.n)])

    def to_density_matrix(self) -> np.ndarray:
        """rho with shape (2,)*2n: ket axes 0..n-1, bra n..2n-1 (small n),
        built site by site with each Kraus leg summed against its conjugate."""
        R = np.ones((1, 1, 1, 1), dtype=np.complex128)               # (ket, bra, l, l')
        for T in self.sites:
            R = np.einsum("ablm,lskr,mtkq->asbtrq", R, T, T.conj(), optimize=True)
            a, s_, b, t, r, q = R.shape
            R = R.reshape(a * s_, b * t, r, q)
        return R[:, :, 0, 0].reshape((2,) * (2 * self.n))


def run_circuit(n: int, ops, d_max: int, k_max: int, cutoff: float = 1e-12):
    """Apply a nearest-neighbour noisy circuit; returns (pmps, total discarded
    weight of bond truncations, total discarded weight of Kraus compressions)."""
    m = PMPS(n)
    disc_bond = disc_kraus = 0.0
    for op in ops:
        q = op.qubits
        if len(q) == 2 and q[1] != q[0] + 1:
            raise ValueError("PMPS needs nearest-neighbour operations (a, a+1)")
        if is_channel(op.name):
            K = kraus_ops(op.name, op.params)
            if len(q) == 1:
                disc_kraus += m.apply_channel1(q[0], K, k_max, cutoff)
            else:
                db, dk = m.apply_channel2(q[0], K, d_max, k_max, cutoff)
                disc_bond += db
                disc_kraus += dk
            continue
        U = gate_matrix(op.name, op.params)
        if len(q) == 1:
            m.apply_gate1(q[0], U)
        else:
            disc_bond += m.apply_gate2(q[0], U, d_max, cutoff)
    return m, disc_bond, disc_kraus
