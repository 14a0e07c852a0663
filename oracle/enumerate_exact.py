"""Exact enumeration of all 2^N states of a tiny thin-film Ising lattice.

TEST INFRASTRUCTURE ONLY (pins the oracle; never used by the product).

Written independently of ``islf_oracle.c``: instead of a bond list it evaluates
the Hamiltonian of Sec. II.A Eq. 1 directly on the coordinate array, with the y
boundary applied as the ghost-row identity the paper states (Eq. 11 for the
generalized antiperiodic condition, S(k_x, k_y + Ly, k_z) = -S(Lx+1-k_x, k_y, k_z);
plain periodic or sign-flipped periodic rows for PBC / APBC), periodic z and
free x surfaces carrying h1 (layer k_x = 1) and hn (layer k_x = Lx).  Each site
contributes the three "forward" products with x+1 (inside the film), y+1 (ghost
row for the last y) and z+1 (mod Lz), so a pair reached twice on a lattice with
Ly = 2 or Lz = 2 counts twice.

Returns exact Boltzmann averages of E, M, M1, Mn (and their field-conjugate
combination M1 - Mn) and ln Z, for N <= 20.
"""
from __future__ import annotations

import numpy as np

PBC, APBC, GAPBC = 0, 1, 2


def all_states(Lx: int, Ly: int, Lz: int) -> np.ndarray:
    """All 2^N spin configurations, shape (2^N, Lx, Ly, Lz), entries +-1 (int8).

    State number k has spin +1 at flat site i iff bit i of k is 0.
    """
    N = Lx * Ly * Lz
    if N > 20:
        raise ValueError("enumeration limited to N <= 20 spins")
    k = np.arange(2 ** N, dtype=np.int64)[:, None]
    bits = (k >> np.arange(N, dtype=np.int64)[None, :]) & 1
    s = (1 - 2 * bits).astype(np.int8)
    return s.reshape(-1, Lx, Ly, Lz)


def ghost_y_row(S: np.ndarray, ybc: int) -> np.ndarray:
    """The row just past y = Ly-1, expressed through row y = 0 (Eq. 11)."""
    row0 = S[:, :, 0, :]
    if ybc == PBC:
        return row0
    if ybc == APBC:
        return -row0
    # generalized antiperiodic: reflect x (k_x -> Lx+1-k_x) and flip the sign
    return -row0[:, ::-1, :]


def bond_sum(S: np.ndarray, ybc: int) -> np.ndarray:
    """B = sum over sites of the products with the x+1, y+1, z+1 partners."""
    S32 = S.astype(np.int32)
    b = np.zeros(S.shape[0], dtype=np.int64)
    # x: only inside the film
    b += (S32[:, :-1, :, :] * S32[:, 1:, :, :]).sum(axis=(1, 2, 3))
    # z: periodic
    b += (S32 * np.roll(S32, -1, axis=3)).sum(axis=(1, 2, 3))
    # y: interior rows, then the last row against the ghost row
    b += (S32[:, :, :-1, :] * S32[:, :, 1:, :]).sum(axis=(1, 2, 3))
    ghost = ghost_y_row(S32, ybc)
    b += (S32[:, :, -1, :] * ghost).sum(axis=(1, 2))
    return b


def observables(S: np.ndarray, ybc: int) -> np.ndarray:
    """(B, M, M1, Mn) for every state; columns as int64."""
    B = bond_sum(S, ybc)
    M = S.astype(np.int64).sum(axis=(1, 2, 3))
    M1 = S[:, 0, :, :].astype(np.int64).sum(axis=(1, 2))
    Mn = S[:, -1, :, :].astype(np.int64).sum(axis=(1, 2))
    return np.stack([B, M, M1, Mn], axis=1)


def energies(obs: np.ndarray, J: float, H: float, h1: float, hn: float) -> np.ndarray:
    """Eq. 1: E = -J B - H M - h1 M1 - hn Mn."""
    return (-J * obs[:, 0] - H * obs[:, 1] - h1 * obs[:, 2] - hn * obs[:, 3]).astype(np.float64)


class Exact:
    """Exact thermodynamics of one small lattice at one parameter point."""

    def __init__(self, Lx, Ly, Lz, ybc=GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=0.0, hn=0.0):
        self.shape = (Lx, Ly, Lz)
        self.S = all_states(Lx, Ly, Lz)
        self.obs = observables(self.S, ybc)
        self.E = energies(self.obs, J, H, h1, hn)
        self.beta = beta
        a = -beta * self.E
        amax = a.max()
        w = np.exp(a - amax)
        self.Z_scaled = w.sum()
        self.lnZ = float(np.log(self.Z_scaled) + amax)
        self.p = w / self.Z_scaled

    def mean(self, q: np.ndarray) -> float:
        return float((self.p * q).sum())

    def var(self, q: np.ndarray) -> float:
        m = self.mean(q)
        return float((self.p * (q - m) ** 2).sum())

    @property
    def means(self) -> dict:
        o = self.obs.astype(np.float64)
        return {
            "E": self.mean(self.E),
            "B": self.mean(o[:, 0]),
            "M": self.mean(o[:, 1]),
            "M1": self.mean(o[:, 2]),
            "Mn": self.mean(o[:, 3]),
        }

    def flat_states(self) -> np.ndarray:
        return self.S.reshape(self.S.shape[0], -1)
