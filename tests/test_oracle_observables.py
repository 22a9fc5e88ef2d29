"""Pins of the oracle's overlap <a|b> = dV sum conj(a) b (the inner product
behind the fidelity loss of the Sec. V ramp and the adjoint seed), fixed by
the algebra of a Hermitian inner product and by closed forms, not by
re-typing its formula.  A conjugate taken on the wrong argument, a dropped
dV or a real part taken too early fails at least one of them."""
import numpy as np

from oracle import observables as ob


def _rand(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_overlap_conjugate_symmetry_and_sesquilinearity():
    rng = np.random.default_rng(11)
    a, b, c = _rand(rng, 257), _rand(rng, 257), _rand(rng, 257)
    dV = 0.37
    alpha = 0.3 - 1.7j
    ab = ob.overlap(a, b, dV)
    # <a|b> = conj(<b|a>)
    assert abs(ab - np.conj(ob.overlap(b, a, dV))) <= 1e-13 * abs(ab)
    # linear in the second argument, antilinear in the first
    assert abs(ob.overlap(a, alpha * b, dV) - alpha * ab) <= 1e-13 * abs(ab) * abs(alpha)
    assert abs(ob.overlap(alpha * a, b, dV) - np.conj(alpha) * ab) <= 1e-13 * abs(ab) * abs(alpha)
    # <a|i b> = i <a|b> (a swapped conjugation would give -i)
    assert abs(ob.overlap(a, 1j * b, dV) - 1j * ab) <= 1e-13 * abs(ab)
    # additive in the second argument
    assert abs(ob.overlap(a, b + c, dV) - (ab + ob.overlap(a, c, dV))) <= 1e-12 * (abs(ab) + 1)


def test_overlap_with_itself_is_the_norm_and_real_positive():
    rng = np.random.default_rng(12)
    a = _rand(rng, 300)
    dV = 0.125
    aa = ob.overlap(a, a, dV)
    assert abs(aa.imag) <= 1e-13 * abs(aa.real)
    assert aa.real > 0
    assert abs(aa.real - ob.norm(a, dV)) <= 1e-13 * aa.real
    # Cauchy-Schwarz
    b = _rand(rng, 300)
    assert abs(ob.overlap(a, b, dV)) ** 2 <= ob.overlap(a, a, dV).real * ob.overlap(b, b, dV).real


def test_overlap_closed_forms_of_discrete_fourier_modes():
    """Plane waves e^{2 pi i k m / M} on M points: <e_k|e_q> = M dV if k = q
    and 0 otherwise; a constant against i times a constant gives i M dV."""
    M, dV = 96, 0.05
    m = np.arange(M)
    for k in (0, 1, 5, 17):
        ek = np.exp(2j * np.pi * k * m / M)
        assert abs(ob.overlap(ek, ek, dV) - M * dV) <= 1e-12
        for q in (k + 1, k + 7, M - 3):
            eq = np.exp(2j * np.pi * q * m / M)
            assert abs(ob.overlap(ek, eq, dV)) <= 1e-12
    # e_1 against e_1 shifted in phase by theta: <e|e^{i theta} e> = e^{i theta} M dV
    e1 = np.exp(2j * np.pi * m / M)
    theta = 0.9
    assert abs(ob.overlap(e1, np.exp(1j * theta) * e1, dV) - np.exp(1j * theta) * M * dV) <= 1e-12
    one = np.ones(M, dtype=complex)
    assert abs(ob.overlap(one, 1j * one, dV) - 1j * M * dV) <= 1e-13
