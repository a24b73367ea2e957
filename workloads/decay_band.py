"""Banded matrix with exponentially decaying entries: the block-sparse
workload (N = 32768, 32 x 32 blocks, truncation threshold 1e-6).

The paper's sparse inputs (Fock matrices of the alkane and water systems of
sec. 5 and sec. 6) are not available. The stand-in is a symmetric matrix
whose entries decay away from the diagonal like those of a local basis:

    F_ij = exp(-|i - j| / 8) z_ij      for 0 < |i - j| <= 192,
    F_ii = -Delta (i even),  +Delta (i odd),

with z_ij independent standard normal (drawn for the upper triangle, one
diagonal offset after the other, and mirrored), and zero outside the band.
The alternating diagonal splits the spectrum into a lower and an upper band;
Delta is chosen so that the gap between eigenvalue n_occ and n_occ + 1
(n_occ = N / 2) is 0.1 within 1e-4.

Eigenvalues are located by inertia: the number of eigenvalues of F below
sigma is the number of negative pivots of an LDL^T factorisation of
F - sigma I (Sylvester's law of inertia), computed without pivoting in the
natural (banded) order, and the eigenvalues nearest sigma come from
shift-invert Lanczos with the same factorisation. The spectral bounds handed
to the method are the extreme Ritz values of a Lanczos run, widened by their
residual norms plus 1e-6.

This module draws random numbers and assembles the input only; it holds
none of the purification arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla


@dataclass
class DecayBandInstance:
    F: sps.csr_matrix        # (n, n) float64, symmetric, half-bandwidth 192
    n_occ: int
    lambda_min: float        # lower bound of the spectrum handed to the method
    lambda_max: float
    delta: float             # alternating diagonal shift
    homo: float              # eigenvalue n_occ (1-based) of F
    lumo: float              # eigenvalue n_occ + 1
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.F.shape[0]

    @property
    def gap(self) -> float:
        return self.lumo - self.homo


def decay_band(n: int, half_width: int, decay: float,
               rng: np.random.Generator) -> sps.csr_matrix:
    """exp(-d / decay) z on the diagonal offsets d = 1 .. half_width (z
    standard normal, drawn offset by offset for the upper triangle),
    mirrored; zero diagonal."""
    offs, vals = [], []
    for d in range(1, min(half_width, n - 1) + 1):
        offs.append(d)
        vals.append(rng.standard_normal(n - d) * np.exp(-d / decay))
    if not offs:
        return sps.csr_matrix((n, n))
    U = sps.diags(vals, offs, shape=(n, n), format="csr")
    return (U + U.T).tocsr()


def alternating_diagonal(n: int) -> np.ndarray:
    """-1 on even, +1 on odd positions."""
    return np.where(np.arange(n) % 2 == 0, -1.0, 1.0)


def _factor(F: sps.spmatrix, sigma: float):
    """LDL^T of F - sigma I in the natural order without pivoting (SuperLU
    with diagonal pivots only): returns the factorisation and the number of
    negative pivots, i.e. of eigenvalues of F below sigma."""
    n = F.shape[0]
    M = (F - sigma * sps.identity(n, format="csr")).tocsc()
    lu = spla.splu(M, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    if not (np.array_equal(lu.perm_r, np.arange(n))
            and np.array_equal(lu.perm_c, np.arange(n))):
        raise RuntimeError("factorisation pivoted: inertia not available")
    d = lu.U.diagonal()
    if np.any(d == 0.0):
        raise RuntimeError("zero pivot: sigma is an eigenvalue of a leading block")
    return lu, int(np.count_nonzero(d < 0.0))


def count_below(F: sps.spmatrix, sigma: float) -> int:
    """Number of eigenvalues of the symmetric F below sigma."""
    return _factor(F, sigma)[1]


def _nearest(F: sps.spmatrix, sigma: float, lu, k: int) -> np.ndarray:
    """The k eigenvalues of F nearest sigma (shift-invert Lanczos with the
    factorisation of F - sigma I; fixed start vector)."""
    n = F.shape[0]
    op = spla.LinearOperator((n, n), matvec=lu.solve, dtype=np.float64)
    v0 = np.cos(np.arange(n) * 0.7548776662466927)   # deterministic start
    w = spla.eigsh(F, k=min(k, n - 1), sigma=sigma, which="LM", OPinv=op,
                   v0=v0, return_eigenvectors=False, tol=1e-14)
    return np.sort(w)


def occupation_gap(F: sps.spmatrix, n_occ: int, sigma: float = 0.0,
                   k: int = 8):
    """(homo, lumo, sigma): eigenvalues n_occ and n_occ + 1 (1-based) of F and
    a point sigma between them. Starting from the given sigma, sigma is moved
    across the eigenvalues that separate it from the gap until exactly n_occ
    eigenvalues lie below it."""
    for _ in range(200):
        lu, c = _factor(F, sigma)
        w = _nearest(F, sigma, lu, k)
        below, above = w[w < sigma][::-1], w[w >= sigma]
        if c == n_occ and below.size and above.size:
            return float(below[0]), float(above[0]), sigma
        if c > n_occ:            # move down across c - n_occ eigenvalues
            m = c - n_occ
            if below.size > m:
                sigma = 0.5 * (below[m - 1] + below[m])
            elif below.size:
                sigma = below[-1] - (sigma - below[-1])
            else:
                sigma -= max(abs(sigma), 1.0) * 1e-3
        elif c < n_occ:          # move up across n_occ - c eigenvalues
            m = n_occ - c
            if above.size > m:
                sigma = 0.5 * (above[m - 1] + above[m])
            elif above.size:
                sigma = above[-1] + (above[-1] - sigma)
            else:
                sigma += max(abs(sigma), 1.0) * 1e-3
        else:                    # in the gap, but one side not in reach
            k *= 2
    raise RuntimeError("gap at the occupation not located")


def spectral_bounds(F: sps.spmatrix, pad: float = 1e-6):
    """(lambda_min, lambda_max): the extreme Ritz values of a Lanczos run,
    widened by their residual norms plus `pad`."""
    n = F.shape[0]
    v0 = np.cos(np.arange(n) * 0.3819660112501051)
    out = []
    for which in ("SA", "LA"):
        w, V = spla.eigsh(F, k=1, which=which, v0=v0, tol=1e-12)
        res = float(np.linalg.norm(F @ V[:, 0] - w[0] * V[:, 0]))
        out.append((float(w[0]), res + pad))
    (lo, rlo), (hi, rhi) = out
    return lo - rlo, hi + rhi


def decay_band_instance(n: int = 32768, half_width: int = 192,
                        decay: float = 8.0, gap: float = 0.1,
                        n_occ: int | None = None, seed: int = 5001,
                        tol: float = 1e-4, delta0: float = 3.3) -> DecayBandInstance:
    """The seeded banded workload with the diagonal shift Delta that puts a
    gap of `gap` (within `tol`) between eigenvalues n_occ and n_occ + 1.
    Delta is found by regula falsi (Illinois variant) on the gap, which is a
    continuous function of Delta, and rounded to 1e-7 so that the input does
    not depend on the rounding of the search."""
    n_occ = n // 2 if n_occ is None else n_occ
    rng = np.random.default_rng(seed)
    A = decay_band(n, half_width, decay, rng)
    alt = sps.diags(alternating_diagonal(n))
    sigma = [0.0]

    def g(delta):
        F = (A + delta * alt).tocsr()
        homo, lumo, s = occupation_gap(F, n_occ, sigma[0])
        sigma[0] = 0.5 * (homo + lumo)
        return lumo - homo - gap

    # bracket: the gap grows with Delta on the whole (the bands separate)
    a, fa = delta0, g(delta0)
    step = 0.25
    b, fb = (a + step, None) if fa < 0 else (a - step, None)
    fb = g(b)
    while fa * fb > 0:
        step *= 2.0
        a, fa = b, fb
        b = b + step if fb < 0 else b - step
        fb = g(b)
        if step > 64:
            raise RuntimeError("no diagonal shift gives the requested gap")
    side = 0
    delta = b
    for _ in range(100):
        delta = (a * fb - b * fa) / (fb - fa)
        fd = g(delta)
        if abs(fd) <= 0.5 * tol:
            break
        if fd * fb < 0:
            a, fa = b, fb
            b, fb = delta, fd
            side = 0
        else:
            b, fb = delta, fd
            if side == 1:
                fa *= 0.5
            side = 1
    delta = round(delta, 7)
    F = (A + delta * alt).tocsr()
    F.sum_duplicates()
    homo, lumo, _ = occupation_gap(F, n_occ, sigma[0])
    if abs(lumo - homo - gap) > tol:
        raise RuntimeError(f"gap {lumo - homo} outside {gap} +- {tol}")
    lmin, lmax = spectral_bounds(F)
    return DecayBandInstance(F=F, n_occ=n_occ, lambda_min=lmin, lambda_max=lmax,
                             delta=delta, homo=homo, lumo=lumo, seed=seed,
                             meta=dict(half_width=half_width, decay=decay,
                                       gap_target=gap))
