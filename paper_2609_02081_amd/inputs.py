"""Seeded synthetic inputs for biquaternion products.

This module only draws numbers and lays them out as eight real component
blocks [M1..M8] (unit coefficients 1:(M1+iM5), i:(M2+iM6), j:(M3+iM7),
k:(M4+iM8)).  It contains none of the product's arithmetic, imports neither
the HIP binding nor the oracle, and serves both sides of every comparison.

Recipes
-------
uniform    i.i.d. uniform[-1, 1]
normal     i.i.d. N(0, 1)
logspread  sign * 10**U(-6, 6): magnitudes spread over 1e-6..1e6
int        i.i.d. integers in [-bound, bound]; products of such inputs are
           exact in FP64 while n * bound**2 * 64 < 2**53
hermitian  Z = U diag(lambda) U^H on the 2n x 2n complex isomorph, U a product
           of six seeded complex Householder reflectors, 2n eigenvalues
           lambda_i = 10**(-8 i / (2n - 1)); "fock" gives each a seeded sign,
           "density" keeps them positive.  The components are read off Z with
           the isomorphic map of the paper (Sec. III, eq. mapping-formulas).

Host draws use numpy's PCG64 (default_rng(seed)); A's active blocks are drawn
in component order, then B's.  Large device-resident inputs are drawn on the
device with a seeded torch generator (different stream from the host one:
such inputs are copied back to the host when the oracle needs them).
"""
from __future__ import annotations

import math

import numpy as np

FULL = 0xFF          # all eight components active
REAL_QUAT = 0x0F     # M1..M4 (real quaternion, [1,1,1,1,0,0,0,0])
COMPLEX = 0x11       # M1, M5 (complex scalar field)
REAL = 0x01          # M1 only

MASKS = {"biquaternion": FULL, "real_quaternion": REAL_QUAT, "complex": COMPLEX, "real": REAL}


def _draw(rng: np.random.Generator, shape, dist: str, bound: int = 1024) -> np.ndarray:
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=shape)
    if dist == "normal":
        return rng.standard_normal(size=shape)
    if dist == "logspread":
        mag = 10.0 ** rng.uniform(-6.0, 6.0, size=shape)
        sgn = np.where(rng.random(size=shape) < 0.5, -1.0, 1.0)
        return sgn * mag
    if dist == "int":
        return rng.integers(-bound, bound + 1, size=shape).astype(np.float64)
    raise ValueError(f"unknown distribution {dist!r}")


def blocks(rng: np.random.Generator, rows: int, cols: int, dist: str = "uniform",
           mask: int = FULL, bound: int = 1024) -> np.ndarray:
    """(8, rows, cols) float64; components outside `mask` are zero."""
    out = np.zeros((8, rows, cols), dtype=np.float64)
    for c in range(8):
        if mask >> c & 1:
            out[c] = _draw(rng, (rows, cols), dist, bound)
    return out


def pair(m: int, k: int, n: int, dist: str = "uniform", seed: int = 1,
         mask_a: int = FULL, mask_b: int = FULL, bound: int = 1024):
    """A (8, m, k) and B (8, k, n) from one seeded stream, A first."""
    rng = np.random.default_rng(seed)
    A = blocks(rng, m, k, dist, mask_a, bound)
    B = blocks(rng, k, n, dist, mask_b, bound)
    return A, B


def batch_sizes(count: int = 512, lo: int = 64, hi: int = 1536, seed: int = 5) -> list[int]:
    """Square sizes drawn log-uniformly from [lo, hi]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [int(min(hi, max(lo, round(math.exp(x))))) for x in u]


# ---------------------------------------------------------------------------
# Hermitian-structured inputs (Fock-like and density-like)
# ---------------------------------------------------------------------------
def hermitian_params(n: int, seed: int, kind: str = "density", reflectors: int = 6) -> dict:
    """Eigenvalues and Householder vectors for Z = U diag(lambda) U^H (size 2n)."""
    rng = np.random.default_rng(seed)
    N = 2 * n
    lam = 10.0 ** (-8.0 * np.arange(N) / max(N - 1, 1))
    if kind == "fock":
        lam = lam * np.where(rng.random(N) < 0.5, -1.0, 1.0)
    elif kind != "density":
        raise ValueError("kind must be 'fock' or 'density'")
    vs = rng.standard_normal((reflectors, N)) + 1j * rng.standard_normal((reflectors, N))
    return {"n": n, "lam": lam, "v": vs}


def hermitian_blocks(params: dict, device="cpu"):
    """Build the (8, n, n) float64 torch tensor of a Hermitian biquaternion.

    Runs with torch on `device`; on a GPU this is input plumbing only.
    Peak extra memory: one 2n x 2n complex128 matrix.
    """
    import torch

    n = params["n"]
    N = 2 * n
    lam = torch.as_tensor(params["lam"], dtype=torch.float64, device=device)
    Z = torch.diag(lam.to(torch.complex128))
    for v_np in params["v"][::-1]:
        v = torch.as_tensor(v_np, dtype=torch.complex128, device=device)
        beta = -2.0 / float(np.vdot(v_np, v_np).real)
        # Z <- H Z H with H = I - 2 v v^H / (v^H v): two rank-1 updates.
        w = v.conj() @ Z                      # v^H Z
        Z.addr_(v, w, alpha=beta)
        w = Z @ v                             # Z v
        Z.addr_(w, v.conj(), alpha=beta)
        del w
    Z = 0.5 * (Z + Z.conj().T)                # remove rounding asymmetry
    out = torch.empty((8, n, n), dtype=torch.float64, device=device)
    a, b = Z[:n, :n], Z[:n, n:]
    c, d = Z[n:, :n], Z[n:, n:]
    # E=(a+d*)/2, F=(b-c*)/2, G=(a-d*)/2, H=(b+c*)/2 ;
    # [M1..M8] = [E_R, E_I, F_R, F_I, G_I, -G_R, H_I, -H_R]
    out[0] = 0.5 * (a.real + d.real)
    out[1] = 0.5 * (a.imag - d.imag)
    out[2] = 0.5 * (b.real - c.real)
    out[3] = 0.5 * (b.imag + c.imag)
    out[4] = 0.5 * (a.imag + d.imag)
    out[5] = -0.5 * (a.real - d.real)
    out[6] = 0.5 * (b.imag - c.imag)
    out[7] = -0.5 * (b.real + c.real)
    del Z
    return out


def hermitian_random(n: int, mask: int = FULL, seed: int = 1, dist: str = "normal") -> np.ndarray:
    """(8, n, n) float64 Hermitian biquaternion (A^dagger = A): components 1
    and 6..8 symmetric, 2..5 antisymmetric (the dagger sign pattern);
    components outside `mask` are zero."""
    rng = np.random.default_rng(seed)
    out = np.zeros((8, n, n), dtype=np.float64)
    for c in range(8):
        if mask >> c & 1:
            X = _draw(rng, (n, n), dist, 1024)
            out[c] = 0.5 * (X + X.T) if c in (0, 5, 6, 7) else 0.5 * (X - X.T)
    return out


def device_uniform(n_rows: int, n_cols: int, seed: int, device, count: int = 8):
    """(count, rows, cols) float64 uniform[-1, 1] drawn on `device`."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.empty((count, n_rows, n_cols), dtype=torch.float64, device=device)
    t.uniform_(-1.0, 1.0, generator=g)
    return t


def device_logspread(n_rows: int, n_cols: int, seed: int, device, count: int = 8):
    """(count, rows, cols) float64 sign * 10^U(-6, 6) drawn on `device` (the
    log-spread recipe at sizes the host would take long to draw)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.empty((count, n_rows, n_cols), dtype=torch.float64, device=device)
    t.uniform_(-6.0, 6.0, generator=g)
    torch.pow(10.0, t, out=t)
    sign = torch.empty((count, n_rows, n_cols), dtype=torch.float64, device=device)
    sign.uniform_(-1.0, 1.0, generator=g)
    t.mul_(torch.sign(sign))
    del sign
    return t


def hermitian_pair(n: int, seed: int, device="cpu"):
    """A Fock-like (signed spectrum, `seed`) and B density-like (positive
    spectrum, `seed + 1`) Hermitian biquaternions, each (8, n, n)."""
    A = hermitian_blocks(hermitian_params(n, seed, "fock"), device)
    B = hermitian_blocks(hermitian_params(n, seed + 1, "density"), device)
    return A, B
