"""Plain FP64 pc-LSQML (test infrastructure only): the least-squares maximum-
likelihood engine of ref. [27] of the paper (Odstrcil, Menzel, Guizar-Sicairos
2018) with the two changes of Sec. 2 -- box 1, the blurred modulus constraint,
gives the exit-wave update, and box 2, the complex constraint of Eq. (9)-(11),
follows the object update inside the windows -- which Sec. 3.2 and Sec. 4.1
call pc-LSQML (Figs. 5 and 6), with K incoherent probe modes for the
mixed-state form.

The paper does not print LSQML.  Reading (the published method restated, in
its Gaussian-noise form; each step is one of ref. [27]'s):
  For each batch S of positions (the batches of oracle.pcepie.iterate), all
  starting from the same (O, P):
  1. chi_{j,k} = psi'_{j,k} - psi_{j,k}: the exit-wave update of box 1 (the same
     quantity pc-ePIE calls dpsi), with psi_{j,k} = o_j P_k.
  2. Update directions averaged over the batch, preconditioned by the summed
     illumination with the rPIE-form regularisation (gamma in (0, 1]; any
     positive scale of a direction is absorbed by step 3):
       dO   = N_O / ((1 - gamma_obj) W + gamma_obj max W)          on the union of the boxes
       dP_k = N_P,k / ((1 - gamma_probe) V + gamma_probe max V)      (zero before probe_update_start)
     with N_O, W, N_P,k, V the sums of oracle.pcepie.batch_step.
  3. Per position j, the real step pair (a_j, b_j) that minimises
       sum_k || chi_{j,k} - a dO_j P_k - b o_j dP_k ||^2
     (dO_j: the box of dO at position j), from its 2x2 normal equations
       [M11 M12; M12 M22] [a; b] = [r1; r2],
       M11 = sum |dO_j P_k|^2, M12 = Re sum conj(dO_j P_k) o_j dP_k, M22 = sum |o_j dP_k|^2,
       r1 = Re sum conj(dO_j P_k) chi_{j,k},  r2 = Re sum conj(o_j dP_k) chi_{j,k}
     (sums over the frame's pixels and the modes), damped on the diagonal,
     M11 <- (1 + lam) M11 and M22 <- (1 + lam) M22 (lam = lsq_damping >= 0;
     with lam > 0 the damped matrix is positive definite whenever both
     diagonals are nonzero, by Cauchy-Schwarz).  A direction with zero norm
     gets a zero step; without probe update, or when the damped matrix is
     singular (possible only without damping), b = 0 and a = r1 / M11.
  4. The batch moves by the mean steps (a_bar, b_bar) over its positions:
       O <- O + obj_step a_bar dO  on the union;  P_k <- P_k + probe_step b_bar dP_k.
  5. Inside a constraint window the complex constraint (box 2) follows, as in
     pc-ePIE.
  After the last batch of an iteration the K > 1 modes are orthogonalised and
  E_t is recorded, as in oracle.pcepie.iterate.
Library primitives: numpy's FFT through oracle.pcepie, numpy.linalg.solve on 2x2.
"""

from __future__ import annotations

import numpy as np

from . import pcepie as pe

__all__ = ["lsq_normal_equations", "lsq_steps", "batch_step", "iterate"]


def lsq_normal_equations(chi, dO_j, P, o_j, dP):
    """The 2x2 real normal equations of step 3 for one position.

    chi: [K, N, N] exit-wave updates; dO_j: [N, N] the object direction on the
    box; P, dP: [K, N, N] probe modes and probe direction; o_j: [N, N] the box.
    Returns (M [2, 2], r [2]).
    """
    a = dO_j[None] * P   # the object direction's exit-wave change per mode
    b = o_j[None] * dP   # the probe direction's exit-wave change per mode
    m11 = float(np.sum(np.abs(a) ** 2))
    m22 = float(np.sum(np.abs(b) ** 2))
    m12 = float(np.real(np.sum(np.conj(a) * b)))
    r1 = float(np.real(np.sum(np.conj(a) * chi)))
    r2 = float(np.real(np.sum(np.conj(b) * chi)))
    return np.array([[m11, m12], [m12, m22]]), np.array([r1, r2])


def lsq_steps(M, r, lam, probe_on):
    """Step 3's damped solve: (a, b) for one position."""
    m11 = M[0, 0] * (1.0 + lam)
    m22 = M[1, 1] * (1.0 + lam)
    if m11 <= 0.0 and (not probe_on or m22 <= 0.0):
        return 0.0, 0.0
    if not probe_on or m22 <= 0.0:
        return r[0] / m11, 0.0
    if m11 <= 0.0:
        return 0.0, r[1] / m22
    if m11 * m22 - M[0, 1] * M[1, 0] <= 0.0:
        # singular (only without damping, when the two directions change the exit
        # waves in parallel): the object step alone
        return r[0] / m11, 0.0
    sol = np.linalg.solve(np.array([[m11, M[0, 1]], [M[1, 0], m22]]), r)
    return float(sol[0]), float(sol[1])


def batch_step(O, P, sqrt_I, positions, batch, t, params: pe.Params, lam=0.1, g=None, capture=False):
    """One pc-LSQML step over a batch of scan positions (steps 1-5 of the module
    reading).  Returns (O_new, P_new, err_num, capture dict or None)."""
    n = params.n
    if g is None:
        g = pe.gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    n_o = np.zeros(O.shape, dtype=np.complex128)
    w = np.zeros(O.shape, dtype=np.float64)
    n_p = np.zeros(P.shape, dtype=np.complex128)
    v = np.zeros((n, n), dtype=np.float64)
    mask = np.zeros(O.shape, dtype=bool)
    err_num = 0.0
    boxes, chis = [], []
    for pos in batch:
        r, c = int(positions[pos][0]), int(positions[pos][1])
        boxes.append((r, c))
        o_b = O[r:r + n, c:c + n]
        psi = o_b[None] * P
        Psi = pe.propagate(psi, params)
        Psi_new, _, ag = pe.modulus_constraint(Psi, sqrt_I[pos], params, g)
        chi = pe.backpropagate(Psi_new, params) - psi
        chis.append(chi)
        err_num += float(np.sum((sqrt_I[pos] - ag) ** 2))
        n_o[r:r + n, c:c + n] += np.sum(np.conj(P) * chi, axis=0)
        w[r:r + n, c:c + n] += np.sum(np.abs(P) ** 2, axis=0)
        n_p += np.conj(o_b)[None] * chi
        v += np.abs(o_b) ** 2
        mask[r:r + n, c:c + n] = True
    probe_on = t >= params.probe_update_start
    go, gp = params.gamma_obj, params.gamma_probe
    dO = np.zeros(O.shape, dtype=np.complex128)
    dO[mask] = n_o[mask] / ((1.0 - go) * w[mask] + go * np.max(w))
    dP = np.zeros(P.shape, dtype=np.complex128)
    if probe_on:
        dP = n_p / ((1.0 - gp) * v + gp * np.max(v))[None]
    steps = []
    for (r, c), chi in zip(boxes, chis):
        M, rhs = lsq_normal_equations(chi, dO[r:r + n, c:c + n], P, O[r:r + n, c:c + n], dP)
        steps.append(lsq_steps(M, rhs, lam, probe_on))
    steps = np.array(steps)
    a_bar, b_bar = float(np.mean(steps[:, 0])), float(np.mean(steps[:, 1]))
    O_new = O.copy()
    O_new[mask] = O[mask] + params.obj_step * a_bar * dO[mask]
    P_new = P + params.probe_step * b_bar * dP if probe_on else P
    cbar = None
    if pe.in_window(t, params):
        O_new, cbar = pe.complex_constraint(O_new, boxes, n, params)
    cap = None
    if capture:
        cap = dict(chi=np.stack(chis), dO=dO, dP=dP, steps=steps, a_bar=a_bar, b_bar=b_bar, n_o=n_o, w=w,
                   n_p=n_p, v=v, mask=mask, cbar=cbar)
    return O_new, P_new, err_num, cap


def iterate(state: pe.State, intensities, positions, params: pe.Params, n_iter, lam=0.1, orders=None,
            sqrt_I=None):
    """n_iter pc-LSQML iterations over the batches of each iteration's order;
    mode orthogonalisation and E_t as in oracle.pcepie.iterate.
    Returns (new State, list of E_t)."""
    if sqrt_I is None:
        sqrt_I = pe.measured_amplitude(intensities, params)
    g = pe.gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    denom = float(np.sum(sqrt_I ** 2))
    O, P, t = state.O.copy(), state.P.copy(), state.t
    n_pos = len(positions)
    errs = []
    for it in range(n_iter):
        t += 1
        order = pe.permutation(params.seed, t, n_pos) if orders is None else np.asarray(orders[it])
        num = 0.0
        for s in range(0, n_pos, params.batch):
            O, P, e, _ = batch_step(O, P, sqrt_I, positions, order[s:s + params.batch], t, params, lam, g)
            num += e
        if P.shape[0] > 1 and params.orthogonalize:
            P, _ = pe.orthogonalize_modes(P)
        errs.append(num / denom if denom > 0 else 0.0)
    return pe.State(O=O, P=P, t=t), errs
