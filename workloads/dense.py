"""Dense synthetic Fock-like matrices with a prescribed spectrum.

The paper builds its dense test matrices (sec. 4.1, the N = 1000 example, and
sec. 5, the N = 200 example) from random orthogonal eigenvectors and
equidistant eigenvalues in two bands separated by the homo-lumo gap. The
workloads here follow the same recipe; by default the eigenvalues are drawn
uniformly inside each band with the four band end points pinned, so that the
gap and the spectral bounds are known exactly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class DenseInstance:
    """One symmetric input matrix and everything known about it exactly."""

    F: np.ndarray            # (n, n) float64, symmetric
    lam: np.ndarray          # (n,) eigenvalues, ascending
    Q: np.ndarray            # (n, n) eigenvectors: F = Q diag(lam) Q^T
    n_occ: int               # number of occupied states (lowest eigenvalues)
    lambda_min: float        # lower spectral bound handed to the method
    lambda_max: float        # upper spectral bound handed to the method
    homo: float              # lam[n_occ - 1]
    lumo: float              # lam[n_occ]
    label: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.F.shape[0]


def random_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Q from the QR factorisation of an n x n standard-normal matrix.

    Column signs are fixed by sign(diag R) so that Q is a deterministic
    function of the draws (and Haar distributed).
    """
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def two_band_spectrum(n: int, n_occ: int, lo: float, hi: float, gap: float,
                      rng: np.random.Generator | None = None,
                      equidistant: bool = False,
                      center: float = 0.0) -> np.ndarray:
    """Ascending eigenvalues: n_occ in [lo, c-gap/2], n-n_occ in [c+gap/2, hi].

    With ``equidistant`` the values are evenly spaced in each band (the
    paper's construction); otherwise they are uniform draws with both end
    points of each band pinned, so the gap and the extreme eigenvalues are
    exactly the requested ones.
    """
    a_hi = center - gap / 2.0
    b_lo = center + gap / 2.0

    def band(m: int, a: float, b: float) -> np.ndarray:
        if m <= 0:
            return np.empty(0)
        if m == 1:
            return np.array([b if b == a_hi else a])
        if equidistant:
            return np.linspace(a, b, m)
        inner = rng.uniform(a, b, size=m - 2) if m > 2 else np.empty(0)
        return np.sort(np.concatenate([[a], inner, [b]]))

    occ = band(n_occ, lo, a_hi)
    virt = band(n - n_occ, b_lo, hi)
    return np.concatenate([occ, virt])


def assemble(Q: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """F = Q diag(lam) Q^T, symmetrised so that F == F.T exactly."""
    F = (Q * lam[None, :]) @ Q.T
    return 0.5 * (F + F.T)


def dense_instance(n: int, n_occ: int, lo: float, hi: float, gap: float,
                   seed: int, equidistant: bool = False, center: float = 0.0,
                   label: str = "") -> DenseInstance:
    rng = np.random.default_rng(seed)
    lam = two_band_spectrum(n, n_occ, lo, hi, gap, rng, equidistant, center)
    Q = random_orthogonal(n, rng)
    F = assemble(Q, lam)
    homo = float(lam[n_occ - 1]) if n_occ > 0 else float("nan")
    lumo = float(lam[n_occ]) if n_occ < n else float("nan")
    return DenseInstance(F=F, lam=lam, Q=Q, n_occ=n_occ,
                         lambda_min=float(lo), lambda_max=float(hi),
                         homo=homo, lumo=lumo, label=label,
                         meta=dict(seed=seed, gap=gap, equidistant=equidistant))


def config_small(seed: int = 1001) -> DenseInstance:
    """N = 512, eigenvalues in [-1,-0.05] (256 occupied) and [0.05,1]."""
    return dense_instance(512, 256, -1.0, 1.0, 0.1, seed,
                          label="dense N=512 gap=0.1")


def config_mid(gap: float = 0.1, seed: int = 2001, n: int = 4096) -> DenseInstance:
    """N = 4096, n_occ = 2048, bands [-1,-gap/2] and [gap/2,1]."""
    return dense_instance(n, n // 2, -1.0, 1.0, gap, seed,
                          label=f"dense N={n} gap={gap:g}")


def config_metric(seed: int = 3001, n: int = 8192) -> DenseInstance:
    """N = 8192, n_occ = 4096, eigenvalues in [-2,-0.025] and [0.025,2]."""
    return dense_instance(n, n // 2, -2.0, 2.0, 0.05, seed,
                          label=f"dense N={n} gap=0.05 range [-2,2]")


def e5_instance(seed: int = 7, n: int = 1000) -> DenseInstance:
    """The paper's dense example of sec. 4.1 (figure fig:dense_1000_500).

    N = 1000, n_occ = 500, eigenvalues equidistant in [0, 0.495] and
    [0.505, 1]; spectral bounds 0 and 1.
    """
    return dense_instance(n, n // 2, 0.0, 1.0, 0.01, seed, equidistant=True,
                          center=0.5, label="paper sec. 4.1 example")


def e6_instance(seed: int = 11, n: int = 200) -> DenseInstance:
    """The paper's dense example of sec. 5: N = 200, n_occ = 100, gap 0.02
    around 0.5, equidistant eigenvalues in [0, 0.49] and [0.51, 1]."""
    return dense_instance(n, n // 2, 0.0, 1.0, 0.02, seed, equidistant=True,
                          center=0.5, label="paper sec. 5 example")


def diagonal_instance(diag: np.ndarray, n_occ: int, lambda_min: float,
                      lambda_max: float, perm_seed: int | None = None
                      ) -> DenseInstance:
    """F = P diag(d) P^T for a permutation P (identity if no seed)."""
    d = np.asarray(diag, dtype=np.float64)
    n = d.size
    if perm_seed is None:
        perm = np.arange(n)
    else:
        perm = np.random.default_rng(perm_seed).permutation(n)
    Q = np.eye(n)[:, perm]
    F = np.zeros((n, n))
    F[perm, perm] = d
    order = np.argsort(d, kind="stable")
    lam = d[order]
    Qs = Q[:, order]
    homo = float(lam[n_occ - 1]) if n_occ > 0 else float("nan")
    lumo = float(lam[n_occ]) if n_occ < n else float("nan")
    return DenseInstance(F=F, lam=lam, Q=Qs, n_occ=n_occ,
                         lambda_min=float(lambda_min),
                         lambda_max=float(lambda_max), homo=homo, lumo=lumo,
                         label="diagonal")


def symmetric_gaussian_perturbation(n: int, spectral_norm: float,
                                    rng: np.random.Generator) -> np.ndarray:
    """Random symmetric matrix with normal entries scaled to a given 2-norm.

    The paper perturbs its dense examples in every iteration with such a
    matrix (sec. 4.1 and sec. 5).
    """
    G = rng.standard_normal((n, n))
    G = 0.5 * (G + G.T)
    s = np.max(np.abs(np.linalg.eigvalsh(G)))
    return G * (spectral_norm / s)
