"""Plain FP64 pc-DM (test infrastructure only): the difference map of ref. [26]
of the paper (Thibault et al.) with the two changes of Sec. 2 -- box 1, the
blurred modulus constraint, in its Fourier projection, and box 2, the complex
constraint of Eq. (9)-(11), on the object after each overlap projection inside
the windows -- which Sec. 4.5 calls pc-DM (Fig. 11).

Notation as in oracle.pcepie.  The state holds one exit wave psi_{n,k} per scan
position n and probe mode k besides the object O and the K probe modes P_k.

One iteration t (1-based):
  1. Overlap projection (one alternation; reading): the object that best
     explains the exit waves for the current probe, then the probe that best
     explains them for the new object, each a least-squares problem with a
     small Tikhonov pull towards the current estimate (reading: without it the
     pixels that no probe intensity reaches are undetermined):
       O <- argmin sum_n sum_k ||P_k o_n - psi_{n,k}||^2 + delta max(W) ||O - O_cur||^2
         = (N_O + delta max W O_cur) / (W + delta max W),
       N_O(r) = sum_n sum_k conj(P_k(r - r_n)) psi_{n,k}(r - r_n),  W(r) = sum_n sum_k |P_k(r - r_n)|^2,
     over the union of the boxes; inside a constraint window the complex
     constraint follows (C-bar pooled over every box of the scan); then, when
     t >= probe_update_start,
       P_k <- (N_P,k + delta max V P_k) / (V + delta max V),
       N_P,k = sum_n conj(o_n) psi_{n,k},  V = sum_n |o_n|^2,
     with o_n the boxes of the new object.
  2. z_{n,k} = P_k o_n, the exit waves of the projected state.
  3. The difference-map step with the pc Fourier projection (box 1):
       psi_{n,k} <- psi_{n,k} + F^-1[ M( F(2 z_n - psi_n) ) ]_k - z_{n,k},
     where M applies the blurred modulus constraint to the K modes of a position.
  4. The data error E_t = sum_n sum_q (sqrt(I_n) - A^G_n)^2 / sum_n sum_q I_n of
     the Fourier projection's input estimates 2 z_n - psi_n (reading; at the map's
     fixed point psi differs from z, so E_t levels off above zero even on
     consistent data while the object converges).
The modes are not orthogonalised (reading: each mode's exit waves are state).
Library primitives: numpy's FFT through oracle.pcepie.propagate.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import pcepie as pe


@dataclasses.dataclass
class DMState:
    O: np.ndarray    # [H, W] complex128
    P: np.ndarray    # [K, N, N] complex128
    psi: np.ndarray  # [n_pos, K, N, N] complex128
    t: int = 0


def exit_waves(O, P, positions):
    """psi_{n,k} = P_k o_n for every scan position (the projected exit waves z)."""
    n = P.shape[-1]
    out = np.zeros((len(positions),) + P.shape, dtype=np.complex128)
    for i, (r, c) in enumerate(positions):
        out[i] = O[int(r):int(r) + n, int(c):int(c) + n][None] * P
    return out


def initial_state(O, P, positions):
    """Start of the iteration: the exit waves of the initial object and probe."""
    O = np.asarray(O, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    return DMState(O=O.copy(), P=P.copy(), psi=exit_waves(O, P, positions))


def project_object(psi, O, P, positions, delta):
    """The regularised least-squares object of the overlap projection (step 1)."""
    n = P.shape[-1]
    n_o = np.zeros(O.shape, dtype=np.complex128)
    w = np.zeros(O.shape, dtype=np.float64)
    mask = np.zeros(O.shape, dtype=bool)
    p2 = np.sum(np.abs(P) ** 2, axis=0)
    for i, (r, c) in enumerate(positions):
        r, c = int(r), int(c)
        n_o[r:r + n, c:c + n] += np.sum(np.conj(P) * psi[i], axis=0)
        w[r:r + n, c:c + n] += p2
        mask[r:r + n, c:c + n] = True
    reg = delta * np.max(w)
    out = O.copy()
    out[mask] = (n_o[mask] + reg * O[mask]) / (w[mask] + reg)
    return out, mask


def project_probe(psi, O, P, positions, delta):
    """The regularised least-squares probe modes of the overlap projection (step 1)."""
    n = P.shape[-1]
    n_p = np.zeros(P.shape, dtype=np.complex128)
    v = np.zeros((n, n), dtype=np.float64)
    for i, (r, c) in enumerate(positions):
        o = O[int(r):int(r) + n, int(c):int(c) + n]
        n_p += np.conj(o)[None] * psi[i]
        v += np.abs(o) ** 2
    reg = delta * np.max(v)
    return (n_p + reg * P) / (v + reg)[None]


def dm_iteration(state: DMState, sqrt_I, positions, params: pe.Params, delta=1e-3, g=None):
    """One pc-DM iteration (steps 1-4 above).  Returns (new DMState, err_num)."""
    if g is None:
        g = pe.gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    t = state.t + 1
    n = params.n
    O, _ = project_object(state.psi, state.O, state.P, positions, delta)
    if pe.in_window(t, params):
        O, _ = pe.complex_constraint(O, [(int(r), int(c)) for r, c in positions], n, params)
    P = state.P
    if t >= params.probe_update_start:
        P = project_probe(state.psi, O, state.P, positions, delta)
    psi = state.psi.copy()
    err = 0.0
    for i, (r, c) in enumerate(positions):
        z = O[int(r):int(r) + n, int(c):int(c) + n][None] * P
        Psi = pe.propagate(2.0 * z - state.psi[i], params)
        Psi_new, _, ag = pe.modulus_constraint(Psi, sqrt_I[i], params, g)
        psi[i] = state.psi[i] + (pe.backpropagate(Psi_new, params) - z)
        err += float(np.sum((sqrt_I[i] - ag) ** 2))
    return DMState(O=O, P=P, psi=psi, t=t), err


def dm_iterate(state: DMState, intensities, positions, params: pe.Params, n_iter, delta=1e-3, sqrt_I=None):
    """n_iter pc-DM iterations; returns (state, [E_t])."""
    if sqrt_I is None:
        sqrt_I = pe.measured_amplitude(intensities, params)
    g = pe.gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    denom = float(np.sum(sqrt_I ** 2))
    errs = []
    for _ in range(n_iter):
        state, e = dm_iteration(state, sqrt_I, positions, params, delta, g)
        errs.append(e / denom if denom > 0 else 0.0)
    return state, errs
