"""Pins for the eigenproblem oracle (oracle.heev): the isomorph of a
Hermitian biquaternion diagonalized by a library eigensolver.  Pinned to a
known spectrum, Kramers degeneracy of time-reversal-symmetric (real
quaternion) matrices, the +-mu spectrum of the block anti-diagonal (pure j or
pure k) case, the trace rule, and the complex scalar field against a direct
eigensolve."""
import numpy as np
import pytest

import oracle
from paper_2609_02081_amd import inputs


def test_known_spectrum():
    """Z = U diag(lambda) U^H built on the complex side (generator), mapped to
    components by the inverse map: the oracle recovers lambda."""
    torch = pytest.importorskip("torch")
    p = inputs.hermitian_params(24, seed=31, kind="fock")
    A = inputs.hermitian_blocks(p).numpy()
    w, V = oracle.heev(A)
    assert np.allclose(w, np.sort(p["lam"]), rtol=0, atol=1e-13)


def test_hermitian_generator_is_hermitian():
    A = inputs.hermitian_random(17, inputs.FULL, seed=32)
    assert np.array_equal(oracle.herm(A), A)
    Z = oracle.iso(A)
    assert np.allclose(Z, Z.conj().T, rtol=0, atol=0)


def test_kramers_pairs_for_real_quaternions():
    """Time-reversal-symmetric (real quaternion) Hermitian matrices have
    doubly degenerate spectra."""
    A = inputs.hermitian_random(20, inputs.REAL_QUAT, seed=33)
    w, _ = oracle.heev(A)
    assert np.allclose(w[0::2], w[1::2], rtol=0, atol=1e-12)
    assert np.min(np.diff(w[0::2])) > 1e-6   # and only doubly


@pytest.mark.parametrize("mask", [0x44, 0x88])
def test_pure_j_or_k_spectrum_is_symmetric(mask):
    """Block anti-diagonal isomorph (only j or only k components): the
    spectrum is +-mu."""
    A = inputs.hermitian_random(19, mask, seed=34)
    w, _ = oracle.heev(A)
    assert np.allclose(w, -w[::-1], rtol=0, atol=1e-12)


def test_trace_rule():
    """sum of the eigenvalues = Tr Z = 2 (Tr c1 + i Tr c5), real for Hermitian A."""
    A = inputs.hermitian_random(23, inputs.FULL, seed=35)
    w, _ = oracle.heev(A)
    assert abs(w.sum() - oracle.trace(A).real) <= 1e-11
    assert abs(oracle.trace(A).imag) == 0.0


def test_complex_scalar_field():
    """Only c1 and c5: Z = diag(c1 + i c5, c1 + i c5), each eigenvalue of
    the complex Hermitian c1 + i c5 twice."""
    A = inputs.hermitian_random(15, inputs.COMPLEX, seed=36)
    w, _ = oracle.heev(A)
    ref = np.linalg.eigvalsh(A[0] + 1j * A[4])
    assert np.allclose(w, np.repeat(ref, 2), rtol=0, atol=1e-12)


def test_eigenvectors():
    A = inputs.hermitian_random(12, inputs.FULL, seed=37)
    w, V = oracle.heev(A)
    Z = oracle.iso(A)
    assert np.allclose(Z @ V, V * w, rtol=0, atol=1e-12)
    assert np.allclose(V.conj().T @ V, np.eye(24), rtol=0, atol=1e-12)
