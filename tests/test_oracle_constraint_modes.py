"""Pins for box 2 of Fig. 1 (the complex constraint, Eq. 9-11 and 19) and for
the mixed-state mode orthogonalisation."""

import math

import numpy as np
import pytest
import scipy.linalg

import oracle as ora


def _obj(rng, shape=(30, 30)):
    a = 0.6 + 0.4 * rng.random(shape)
    ph = rng.uniform(-1.2, 1.2, shape)
    return a * np.exp(1j * ph)


def test_zero_alphas_identity(rng):
    O = _obj(rng)
    p = ora.Params(n=8, alpha1=0.0, alpha2=0.0)
    out, cbar = ora.complex_constraint(O, [(0, 0), (10, 12)], 8, p)
    np.testing.assert_allclose(out, O, atol=1e-14)
    assert cbar is not None


@pytest.mark.parametrize("alphas", [(1.0, 0.0), (0.0, 1.0), (0.4, 0.7)])
def test_homogeneous_object_is_fixed_point(alphas, rng):
    """Eq. (17)-(19): ln A = c phi with c = beta/delta; C-bar recovers c and the
    constraint leaves the object unchanged for any alphas."""
    c = 0.25
    tau = rng.random((30, 30)) * 2.0
    phi = -0.9 * tau
    O = np.exp(c * phi) * np.exp(1j * phi)
    p = ora.Params(n=10, alpha1=alphas[0], alpha2=alphas[1])
    out, cbar = ora.complex_constraint(O, [(2, 3), (15, 9)], 10, p)
    assert abs(cbar - c) < 1e-12
    np.testing.assert_allclose(out, O, atol=1e-12)


def test_amplitude_and_phase_closed_forms(rng):
    O = _obj(rng)
    boxes = [(1, 1), (12, 14)]
    n = 9
    mask = np.zeros(O.shape, bool)
    for r, c in boxes:
        mask[r:r + n, c:c + n] = True
    sa = sum(np.sum(np.abs(np.log(np.abs(O[r:r + n, c:c + n])))) for r, c in boxes)
    sp = sum(np.sum(np.abs(np.angle(O[r:r + n, c:c + n]))) for r, c in boxes)
    cb = sa / sp
    # alpha1 = 0, alpha2 = 1 (amplitude object, Sec. 4.6): A kept, phi = ln A / C
    out, cbar = ora.complex_constraint(O, boxes, n, ora.Params(n=n, alpha1=0.0, alpha2=1.0))
    assert abs(cbar - cb) < 1e-12
    np.testing.assert_allclose(np.abs(out[mask]), np.abs(O[mask]), rtol=1e-12)
    np.testing.assert_allclose(np.angle(out[mask]), np.log(np.abs(O[mask])) / cb, atol=1e-12)
    # alpha1 = 1, alpha2 = 0 (phase object, Sec. 3.1): phi kept, A = exp(C phi)
    out, _ = ora.complex_constraint(O, boxes, n, ora.Params(n=n, alpha1=1.0, alpha2=0.0))
    np.testing.assert_allclose(np.abs(out[mask]), np.exp(cb * np.angle(O[mask])), rtol=1e-12)
    np.testing.assert_allclose(np.angle(out[mask]), np.angle(O[mask]), atol=1e-12)
    # pixels outside the boxes are untouched
    np.testing.assert_array_equal(out[~mask], O[~mask])


def test_cbar_clamped_and_degenerate(rng):
    O = 0.5 * np.exp(1j * 1e-4 * np.ones((20, 20)))  # tiny phase: ratio huge -> clamp
    out, cbar = ora.complex_constraint(O, [(0, 0)], 8, ora.Params(n=8, cbar_max=3.0))
    assert cbar == 3.0
    O = 0.5 * np.ones((20, 20), complex)  # zero phase: skipped
    out, cbar = ora.complex_constraint(O, [(0, 0)], 8, ora.Params(n=8))
    assert cbar is None
    np.testing.assert_array_equal(out, O)


def test_windows():
    p = ora.Params(n=8, cc_start=5, cc_end=35)
    assert [t for t in range(1, 40) if ora.in_window(t, p)] == list(range(5, 36))
    p = ora.Params(n=8, cc_start=5, cc_end=35, cc_period=100)
    assert ora.in_window(105, p) and ora.in_window(235, p) and not ora.in_window(140, p)
    assert not ora.in_window(3, ora.Params(n=8))


def test_orthogonalization_properties(rng):
    k, n = 4, 10
    P = rng.standard_normal((k, n, n)) + 1j * rng.standard_normal((k, n, n))
    Q, lam = ora.orthogonalize_modes(P)
    flat = Q.reshape(k, -1)
    gram = np.conj(flat) @ flat.T
    np.testing.assert_allclose(gram, np.diag(lam), atol=1e-10)
    assert np.all(np.diff(lam) <= 0)
    np.testing.assert_allclose(np.sum(np.abs(Q) ** 2, axis=0), np.sum(np.abs(P) ** 2, axis=0),
                               rtol=1e-12)
    pf = P.reshape(k, -1)
    ref = np.sort(scipy.linalg.eigvalsh(np.conj(pf) @ pf.T))[::-1]
    np.testing.assert_allclose(lam, ref, rtol=1e-12)


def test_orthogonal_modes_are_kept_up_to_order(rng):
    n = 12
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b -= np.vdot(a, b) / np.vdot(a, a) * a
    a *= 1.0 / np.linalg.norm(a)
    b *= 2.0 / np.linalg.norm(b)
    Q, lam = ora.orthogonalize_modes(np.stack([a, b]))
    np.testing.assert_allclose(lam, [4.0, 1.0], rtol=1e-12)
    # same modes, order by power, each up to a unit phase
    for q, ref in ((Q[0], b), (Q[1], a)):
        ph = np.vdot(ref, q) / abs(np.vdot(ref, q))
        np.testing.assert_allclose(q, ref * ph, atol=1e-12)


def test_orthogonalization_phase_rule(rng):
    """The remix Q = V^T P of the R11 reading: recover V from Q and P by least squares
    (independently of the eigensolver) and check each column's largest-magnitude entry
    is real and positive, the columns are orthonormal, and the powers are descending."""
    k, n = 5, 9
    P = rng.standard_normal((k, n, n)) + 1j * rng.standard_normal((k, n, n))
    P *= np.array([3.0, 1.0, 2.0, 0.5, 1.5])[:, None, None]
    Q, lam = ora.orthogonalize_modes(P)
    pf, qf = P.reshape(k, -1), Q.reshape(k, -1)
    # qf = V^T pf  <=>  pf^T V = qf^T
    v, *_ = np.linalg.lstsq(pf.T, qf.T, rcond=None)
    np.testing.assert_allclose(pf.T @ v, qf.T, atol=1e-10)
    np.testing.assert_allclose(np.conj(v.T) @ v, np.eye(k), atol=1e-10)
    for j in range(k):
        i = int(np.argmax(np.abs(v[:, j])))
        assert abs(v[i, j].imag) < 1e-10 and v[i, j].real > 0, (j, v[:, j])
    powers = np.sum(np.abs(qf) ** 2, axis=1)
    np.testing.assert_allclose(powers, lam, rtol=1e-10)
    assert np.all(np.diff(powers) < 0)


def test_orthogonalization_phase_rule_flags_a_wrong_rule(rng):
    """A rule that leaves the eigensolver's phases (or fixes the first entry instead of
    the largest) fails the check above, so the pin is not vacuous."""
    k, n = 4, 6
    P = rng.standard_normal((k, n, n)) + 1j * rng.standard_normal((k, n, n))
    pf = P.reshape(k, -1)
    gram = np.conj(pf) @ pf.T
    lam, vec = np.linalg.eigh(gram)
    vec = vec[:, ::-1] * np.exp(1j * np.arange(1, k + 1))[None, :]  # arbitrary phases
    bad = []
    for j in range(k):
        i = int(np.argmax(np.abs(vec[:, j])))
        bad.append(abs(vec[i, j].imag) < 1e-10 and vec[i, j].real > 0)
    assert not all(bad)
