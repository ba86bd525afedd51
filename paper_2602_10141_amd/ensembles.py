"""Seeded synthetic inputs: the random-matrix ensembles and geodesic points.

Inputs only -- no permanent arithmetic lives here.  Both the GPU path's
tests/benchmark and the oracle's tests draw their matrices from this module,
so the two sides see identical bytes.

Seeding: ``rng(cfg, sub)`` is numpy's PCG64 seeded with
SeedSequence([260210141, cfg, sub]).

Ensembles (paper Sec. 3.1, 5.1 and 6):

* complex Ginibre  -- i.i.d. CN(0,1): real and imaginary parts i.i.d. N(0, 1/2),
* real Ginibre     -- i.i.d. N(0,1),
* GUE = (A + A^*)/2 with A complex Ginibre, GOE = (A + A^T)/2 with A real Ginibre,
* Haar U(n)        -- Q R = complex Ginibre, U = Q diag(R_ii / |R_ii|),
* Haar O(n)        -- Q R = real Ginibre,    O = Q diag(sign R_ii).

Geodesics from I to the n-cycle C_n, (C_n)_{ij} = [i = j+1 mod n] (Sec. 4.1):

* ``cycle_geodesic``           principal branch gamma(t) = exp(t Log C_n), whose
  eigen-angles 2 pi k / n are taken in (-pi, pi]; for odd n the matrix is real:
  gamma(t)_{jl} = (-1)^{l-j} sin(pi t) / (n sin(pi (l - j + t) / n)),
  with gamma(0) = I and gamma(1) = C_n (the formula is 0/0 there);
* ``cycle_geodesic_circulant`` the paper's circulant formula, eigen-angles
  2 pi k / n with k = 0..n-1: gamma(t)_{jl} = (e^{2 pi i t} - 1) /
  (n (e^{2 pi i (l - j + t)/n} - 1)).

Geodesic from I to the unitary DFT matrix F_n = (w^{jk} / sqrt n),
w = e^{2 pi i / n} (Sec. 4.2): ``dft_geodesic``.  F_n^4 = I, so its
eigenvalues lie in {1, i, -1, -i} and P_lam = (1/4) sum_k lam^{-k} F_n^k
projects onto the eigenspace of lam.  gamma(t) = sum_lam e^{t log lam} P_lam
with log 1 = 0, log(+-i) = +-i pi/2 and log(-1) = branch * i pi: the paper
does not say which logarithm of -1 it takes, so the branch (+1 or -1) is an
argument.
"""
import numpy as np

ROOT_SEED = 260210141


def rng(cfg: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, cfg, sub])))


def ginibre_complex(n, g, count=None):
    shape = (n, n) if count is None else (count, n, n)
    s = np.sqrt(0.5)
    return g.standard_normal(shape) * s + 1j * (g.standard_normal(shape) * s)


def ginibre_real(n, g, count=None):
    shape = (n, n) if count is None else (count, n, n)
    return g.standard_normal(shape)


def gue(n, g, count=None):
    A = ginibre_complex(n, g, count)
    return (A + np.conj(np.swapaxes(A, -1, -2))) / 2


def goe(n, g, count=None):
    A = ginibre_real(n, g, count)
    return (A + np.swapaxes(A, -1, -2)) / 2


def haar_unitary(n, g, count=None):
    Z = ginibre_complex(n, g, count)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    return Q * ph[..., None, :]


def haar_orthogonal(n, g, count=None):
    Z = ginibre_real(n, g, count)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    return Q * np.sign(d)[..., None, :]


def cycle_matrix(n):
    C = np.zeros((n, n))
    for j in range(n):
        C[(j + 1) % n, j] = 1.0
    return C


def cycle_geodesic(n: int, t: float) -> np.ndarray:
    """Principal-branch point gamma(t) on the geodesic I -> C_n, n odd, complex128."""
    if n % 2 == 0:
        raise ValueError("the principal branch is real only for odd n")
    if t == 0.0:
        return np.eye(n, dtype=np.complex128)
    if t == 1.0:
        return cycle_matrix(n).astype(np.complex128)
    d = (np.arange(n)[None, :] - np.arange(n)[:, None])      # l - j
    sign = np.where(d % 2 == 0, 1.0, -1.0)
    G = sign * np.sin(np.pi * t) / (n * np.sin(np.pi * (d + t) / n))
    return G.astype(np.complex128)


def cycle_geodesic_circulant(n: int, t: float) -> np.ndarray:
    """gamma(t) by the paper's circulant formula (eigen-angles 2 pi k/n, k=0..n-1)."""
    if t == 0.0:
        return np.eye(n, dtype=np.complex128)
    d = (np.arange(n)[None, :] - np.arange(n)[:, None])
    num = np.exp(2j * np.pi * t) - 1.0
    den = n * (np.exp(2j * np.pi * (d + t) / n) - 1.0)
    return num / den


def dft_matrix(n: int) -> np.ndarray:
    """Unitary DFT matrix F_n = (w^{jk} / sqrt n), w = e^{2 pi i / n}."""
    j = np.arange(n)
    return np.exp(2j * np.pi * np.outer(j, j) / n) / np.sqrt(n)


def dft_geodesic(n: int, t: float, branch: int = 1) -> np.ndarray:
    """gamma(t) = exp(t log F_n), log(-1) = branch * i pi, complex128."""
    if branch not in (1, -1):
        raise ValueError("branch must be +1 or -1")
    F = dft_matrix(n)
    powers = [np.eye(n, dtype=complex)]
    for _ in range(3):
        powers.append(powers[-1] @ F)
    out = np.zeros((n, n), dtype=complex)
    for lam, angle in ((1, 0.0), (1j, np.pi / 2), (-1, branch * np.pi), (-1j, -np.pi / 2)):
        proj = sum(lam ** (-k) * powers[k] for k in range(4)) / 4
        out += np.exp(1j * angle * t) * proj
    return out


def geodesic_grid(points: int = 64):
    """t_i = i / (points - 1), i = 0..points-1 (both ends included)."""
    return [i / (points - 1) for i in range(points)]


def schur_complex(n: int) -> np.ndarray:
    """S_n = (e^{2 pi i jk/n}) over C."""
    j = np.arange(n)
    return np.exp(2j * np.pi * np.outer(j, j) / n)


def random_residues(n, p, g, count=None):
    """Uniform residues in [0, p) as uint32."""
    shape = (n, n) if count is None else (count, n, n)
    return g.integers(0, p, size=shape, dtype=np.uint64).astype(np.uint32)
