"""Plain FP64 implementation of one pc-ePIE reconstruction (test infrastructure only).

Notation follows the paper (Sec. 2): O is the object transmission function,
o_n the object box extracted at scan position n, P the probe (here K incoherent
modes P_k), Psi the diffracted wave estimate, I the recorded intensity, g the
normalised 2D Gaussian of Eq. (7), and A^G the blurred amplitude of Eq. (6).

Arrays are complex128 / float64.  Library primitives used as single steps:
numpy.fft (the unitary 2D DFT), numpy.linalg.eigh (a Hermitian eigensolve).
No blocking, fusion or reordering is applied beyond what the definitions state.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "FAR_FIELD", "NEAR_FIELD", "BLUR_AMPLITUDE", "BLUR_INTENSITY",
    "Params", "fft2u", "ifft2u", "transfer_function", "propagate", "backpropagate",
    "gaussian_kernel", "blur_periodic", "modulus_constraint", "in_window",
    "complex_constraint", "orthogonalize_modes", "batch_step", "iterate",
    "splitmix64_stream", "permutation", "measured_amplitude", "nmse",
    "illumination_roi", "State",
]

FAR_FIELD = 0
NEAR_FIELD = 1
BLUR_AMPLITUDE = 0
BLUR_INTENSITY = 1
LN_FLOOR = 1e-20  # amplitude floor before the logarithm of Eq. (9)-(11)


@dataclasses.dataclass
class Params:
    """Reconstruction parameters (the same fields the C library takes).

    sigma1 acts along x (columns, horizontal) and sigma2 along y (rows,
    vertical), as stated below Eq. (7).  kernel_size is the side of the square
    Gaussian support (11 in all of the paper's reconstructions, Sec. 3.1).
    alpha1/alpha2 weight Eq. (9)/(10); cc_start..cc_end is the 1-based inclusive
    window of iterations in which the complex constraint is applied (Sec. 3.1:
    "5th-35th"), repeated every cc_period iterations when cc_period > 0
    (Sec. 4.6: "in every 100 iterations").
    """

    n: int
    n_modes: int = 1
    geometry: int = FAR_FIELD
    fresnel_px: float = 0.0
    sigma1: float = 1.0
    sigma2: float = 1.0
    kernel_size: int = 11
    blur_domain: int = BLUR_AMPLITUDE
    eps: float = 1e-6
    alpha1: float = 1.0
    alpha2: float = 0.0
    cbar_min: float = 0.01
    cbar_max: float = 10.0
    cc_start: int = 0
    cc_end: int = -1
    cc_period: int = 0
    obj_step: float = 1.0
    probe_step: float = 1.0
    gamma_obj: float = 1.0
    gamma_probe: float = 1.0
    probe_update_start: int = 1
    batch: int = 1
    orthogonalize: int = 1
    seed: int = 0


# ----------------------------------------------------------------------------
# Propagators (Eq. 1 and the near-field geometry of Sec. 3.1)
# ----------------------------------------------------------------------------

def fft2u(x):
    """Unitary 2D DFT over the last two axes: the Fourier propagator of Eq. (1).

    Psi[u, v] = N^-1 sum_{y,x} psi[y, x] exp(-2 pi i (u x + v y) / N), FFT order.
    """
    return np.fft.fft2(x, axes=(-2, -1), norm="ortho")


def ifft2u(x):
    """Inverse of :func:`fft2u`."""
    return np.fft.ifft2(x, axes=(-2, -1), norm="ortho")


def transfer_function(n, fresnel_px):
    """Paraxial free-space transfer function for the near-field geometry.

    Sec. 3.1 places the detector 19.9 mm behind the sample with no optics in
    between; the paper does not print the propagator.  Reading: the paraxial
    angular-spectrum transfer function H(f) = exp(-i pi lambda z |f|^2), which
    on an N-point grid of pitch dx is exp(-i pi (u~^2 + v~^2) / (N^2 F_px)) with
    the signed frequency index u~ and the pixel Fresnel number
    F_px = dx^2 / (lambda z).
    """
    k = np.fft.fftfreq(n, d=1.0 / n)  # signed integer index, FFT order
    h1 = np.exp(-1j * math.pi * k.astype(np.float64) ** 2 / (n * n * fresnel_px))
    return h1[:, None] * h1[None, :]


def propagate(psi, params: Params):
    """Sample plane -> detector plane (Eq. 1's propagator; far or near field)."""
    if params.geometry == FAR_FIELD:
        return fft2u(psi)
    h = transfer_function(params.n, params.fresnel_px)
    return ifft2u(h * fft2u(psi))


def backpropagate(Psi, params: Params):
    """Detector plane -> sample plane, the adjoint (= inverse) of :func:`propagate`."""
    if params.geometry == FAR_FIELD:
        return ifft2u(Psi)
    h = transfer_function(params.n, params.fresnel_px)
    return ifft2u(np.conj(h) * fft2u(Psi))


# ----------------------------------------------------------------------------
# Box 1 of Fig. 1: Gaussian convolution of the estimated amplitude (Eq. 6-7)
# ----------------------------------------------------------------------------

def gaussian_kernel(sigma1, sigma2, kernel_size):
    """The normalised kernel g of Eq. (7) on a kernel_size x kernel_size support.

    g[dy, dx] = exp(-(dx^2 / 2 sigma1^2 + dy^2 / 2 sigma2^2)) / Z, with x the
    horizontal (column) offset and y the vertical (row) offset; Z makes the
    entries sum to one ("normalized", Sec. 2).  A zero sigma makes that axis a
    delta (the fully coherent limit, where the normalised MCF is unity, Eq. 5).
    Returned with index [dy + h, dx + h], h = (kernel_size - 1) / 2.
    """
    if kernel_size < 1 or kernel_size % 2 == 0:
        raise ValueError("kernel_size must be odd and positive")
    h = (kernel_size - 1) // 2
    d = np.arange(-h, h + 1, dtype=np.float64)
    g = np.zeros((kernel_size, kernel_size))
    for iy, dy in enumerate(d):
        for ix, dx in enumerate(d):
            ex = 0.0 if dx == 0 else (math.inf if sigma1 == 0 else dx * dx / (2 * sigma1 * sigma1))
            ey = 0.0 if dy == 0 else (math.inf if sigma2 == 0 else dy * dy / (2 * sigma2 * sigma2))
            g[iy, ix] = math.exp(-(ex + ey))
    return g / g.sum()


def blur_periodic(a, g):
    """(a (x) g)[y, x] = sum_{dy,dx} g[dy, dx] a[y - dy, x - dx], indices mod N.

    The convolution of Eq. (6) with a periodic boundary (reading: the paper
    does not state the boundary; periodic makes the blur commute with the
    centring shift of a far-field pattern).
    """
    h = (g.shape[0] - 1) // 2
    out = np.zeros(a.shape, dtype=np.float64)
    for iy in range(g.shape[0]):
        for ix in range(g.shape[1]):
            out += g[iy, ix] * np.roll(a, shift=(iy - h, ix - h), axis=(-2, -1))
    return out


def modulus_constraint(Psi, sqrt_I, params: Params, g=None):
    """Partially coherent modulus constraint (box 1 of Fig. 1; Eq. 2 and 6).

    Psi: [K, N, N] detector-plane estimates of the K incoherent modes;
    sqrt_I: [N, N] measured amplitude sqrt(max(I, 0)) in the same pixel order.
    The modelled amplitude is the incoherent mode sum A = sqrt(sum_k |Psi_k|^2)
    (mixed-state model, Sec. 1 and Sec. 4.1).  Reading of the unprinted update:
      AMPLITUDE (Eq. 6): A^G = A (x) g,            factor = sqrt(I) / (A^G + eps)
      INTENSITY (Eq. 2): I^G = (sum_k|Psi_k|^2) (x) g, factor = sqrt(I / (I^G + eps^2))
    and Psi'_k = factor * Psi_k.  Returns (Psi', factor, A^G); A^G is
    sqrt(I^G) in the intensity domain and feeds the data error.
    """
    if g is None:
        g = gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    i_mod = np.sum(np.abs(Psi) ** 2, axis=0)
    if params.blur_domain == BLUR_AMPLITUDE:
        ag = blur_periodic(np.sqrt(i_mod), g)
        factor = sqrt_I / (ag + params.eps)
    else:
        ig = blur_periodic(i_mod, g)
        ag = np.sqrt(ig)
        factor = sqrt_I / np.sqrt(ig + params.eps ** 2)
    return Psi * factor[None], factor, ag


# ----------------------------------------------------------------------------
# Box 2 of Fig. 1: the complex constraint (Eq. 8-11)
# ----------------------------------------------------------------------------

def in_window(t, params: Params):
    """True when 1-based iteration t lies in a complex-constraint window.

    The paper applies the constraint in early windows only, e.g. the 5th-35th
    iterations (Sec. 3.1), or the 5th-35th of every 100 (Sec. 4.6).
    """
    if params.cc_end < params.cc_start or params.cc_start < 1:
        return False
    tt = t
    if params.cc_period > 0:
        tt = (t - 1) % params.cc_period + 1
    return params.cc_start <= tt <= params.cc_end


def complex_constraint(O, boxes, n, params: Params):
    """Eq. (9)-(11) applied to the object after an update.

    C-bar (Eq. 11) is the ratio of sum |ln A'| to sum |phi'| over the M pixels
    of the object box; for a batch of boxes both sums run over every box
    (pixels covered twice count twice; with one box this is Eq. 11 exactly).
    Readings: amplitudes are floored at 1e-20 before the logarithm; phi' is the
    principal argument in (-pi, pi]; C-bar is confined to [cbar_min, cbar_max]
    (the threshold of Sec. 4.8, whose values the paper does not give); when
    sum |phi'| = 0 the constraint is skipped.  Eq. (9)-(10) are then applied to
    every pixel in the union of the boxes:
      A^c   = exp[(1 - alpha1) ln A' + alpha1 C phi']
      phi^c = (1 - alpha2) phi' + alpha2 C^-1 ln A'
    Returns (O_new, C-bar or None when skipped).
    """
    sa = 0.0
    sp = 0.0
    mask = np.zeros(O.shape, dtype=bool)
    for (r, c) in boxes:
        box = O[r:r + n, c:c + n]
        sa += np.sum(np.abs(np.log(np.maximum(np.abs(box), LN_FLOOR))))
        sp += np.sum(np.abs(np.angle(box)))
        mask[r:r + n, c:c + n] = True
    if sp == 0.0:
        return O, None
    cbar = min(max(sa / sp, params.cbar_min), params.cbar_max)
    a1, a2 = params.alpha1, params.alpha2
    vals = O[mask]
    ln_a = np.log(np.maximum(np.abs(vals), LN_FLOOR))
    phi = np.angle(vals)
    amp_c = np.exp((1.0 - a1) * ln_a + a1 * cbar * phi)
    phi_c = (1.0 - a2) * phi + a2 * ln_a / cbar
    out = O.copy()
    out[mask] = amp_c * np.exp(1j * phi_c)
    return out, cbar


# ----------------------------------------------------------------------------
# Mixed-state probe modes (Sec. 4.1 / 4.4: the mixed-state method)
# ----------------------------------------------------------------------------

def orthogonalize_modes(P):
    """Orthogonalise K probe modes (reading: the mixed-state treatment the paper
    combines pc with, Sec. 4.1, keeps mutually orthogonal modes).

    G_ij = <P_i, P_j> = sum_r conj(P_i) P_j;  G V = V diag(lam);  Q_j = sum_i V_ij P_i,
    sorted by power lam descending; each eigenvector's phase is fixed so that
    its largest-magnitude entry (the first, on ties) is real and positive.
    The map is unitary, so sum_k |P_k(r)|^2 is preserved at every pixel.
    """
    k = P.shape[0]
    flat = P.reshape(k, -1)
    gram = np.conj(flat) @ flat.T
    lam, vec = np.linalg.eigh(gram)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    vec = vec[:, order]
    for j in range(k):
        i = int(np.argmax(np.abs(vec[:, j])))
        vec[:, j] *= np.conj(vec[i, j]) / abs(vec[i, j])
    q = vec.T @ flat
    return q.reshape(P.shape), lam


# ----------------------------------------------------------------------------
# One batch step and one iteration of pc-ePIE (Fig. 1)
# ----------------------------------------------------------------------------

def measured_amplitude(intensities, params: Params):
    """sqrt(max(I, 0)) in the pixel order the propagator produces.

    Far-field patterns arrive with the zero frequency at (N/2, N/2) and are
    moved to FFT order once; near-field patterns are real-space images.
    """
    a = np.sqrt(np.maximum(np.asarray(intensities, dtype=np.float64), 0.0))
    if params.geometry == FAR_FIELD:
        a = np.fft.ifftshift(a, axes=(-2, -1))
    return a


@dataclasses.dataclass
class State:
    O: np.ndarray
    P: np.ndarray
    t: int = 0  # number of completed iterations


def batch_step(O, P, sqrt_I, positions, batch, t, params: Params, g=None, capture=False):
    """One step of pc-ePIE over a batch of scan positions (Fig. 1, boxes 1 and 2).

    For every position b in the batch, starting from the same (O, P):
      o_b = O[box_b]; psi_bk = o_b P_k; Psi = propagate(psi); Psi' = modulus
      constraint (box 1); psi' = backpropagate(Psi'); dpsi_bk = psi' - psi.
    The ePIE update of ref. [24] (not printed in the paper; reading) uses the
    pre-update o_b and P:
      N_O(r) = sum_b sum_k conj(P_k(r - r_b)) dpsi_bk(r - r_b),  W(r) = sum_b sum_k |P_k(r - r_b)|^2
      N_P,k  = sum_b conj(o_b) dpsi_bk,                         V    = sum_b |o_b|^2
      O += obj_step N_O / ((1 - gamma_obj) W + gamma_obj max W)   on the union of the boxes
      P_k += probe_step N_P,k / ((1 - gamma_probe) V + gamma_probe max V)   if t >= probe_update_start
    With one position and gamma = 1 this is exactly the ePIE loop of Fig. 1
    (object step alpha P*/max|P|^2, probe step beta o*/max|o|^2).  Batches of
    B > 1 positions are this library's reading (the paper is sequential).
    Inside a constraint window the complex constraint (box 2) follows.
    Returns (O_new, P_new, err_num, capture dict or None).
    """
    n = params.n
    if g is None:
        g = gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    n_o = np.zeros(O.shape, dtype=np.complex128)
    w = np.zeros(O.shape, dtype=np.float64)
    n_p = np.zeros(P.shape, dtype=np.complex128)
    v = np.zeros((n, n), dtype=np.float64)
    mask = np.zeros(O.shape, dtype=bool)
    err_num = 0.0
    cap = {"psi": [], "psi_new": [], "factor": []} if capture else None
    boxes = []
    for pos in batch:
        r, c = int(positions[pos][0]), int(positions[pos][1])
        boxes.append((r, c))
        o_b = O[r:r + n, c:c + n]
        psi = o_b[None] * P
        Psi = propagate(psi, params)
        Psi_new, factor, ag = modulus_constraint(Psi, sqrt_I[pos], params, g)
        psi_new = backpropagate(Psi_new, params)
        dpsi = psi_new - psi
        err_num += float(np.sum((sqrt_I[pos] - ag) ** 2))
        n_o[r:r + n, c:c + n] += np.sum(np.conj(P) * dpsi, axis=0)
        w[r:r + n, c:c + n] += np.sum(np.abs(P) ** 2, axis=0)
        n_p += np.conj(o_b)[None] * dpsi
        v += np.abs(o_b) ** 2
        mask[r:r + n, c:c + n] = True
        if capture:
            cap["psi"].append(psi)
            cap["psi_new"].append(psi_new)
            cap["factor"].append(factor)
    go, gp = params.gamma_obj, params.gamma_probe
    O_new = O.copy()
    denom_o = (1.0 - go) * w[mask] + go * np.max(w)
    O_new[mask] = O[mask] + params.obj_step * n_o[mask] / denom_o
    P_new = P
    if t >= params.probe_update_start:
        denom_p = (1.0 - gp) * v + gp * np.max(v)
        P_new = P + params.probe_step * n_p / denom_p[None]
    cbar = None
    if in_window(t, params):
        O_new, cbar = complex_constraint(O_new, boxes, n, params)
    if capture:
        for key in ("psi", "psi_new", "factor"):
            cap[key] = np.stack(cap[key])
        cap.update(n_o=n_o, w=w, n_p=n_p, v=v, cbar=cbar, mask=mask)
    return O_new, P_new, err_num, cap


def splitmix64_stream(state, count):
    """`count` outputs of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) from `state`."""
    mask = (1 << 64) - 1
    out = []
    s = state & mask
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & mask
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def permutation(seed, t, n_pos):
    """The random sequence S_n of Fig. 1 for 1-based iteration t (reading: the
    paper names no generator).  Fisher-Yates over 0..n_pos-1 driven by
    SplitMix64 seeded with seed XOR t: for i = n_pos-1 down to 1, j = next % (i+1),
    swap a[i], a[j]."""
    a = list(range(n_pos))
    draws = splitmix64_stream(seed ^ t, max(n_pos - 1, 0))
    for idx, i in enumerate(range(n_pos - 1, 0, -1)):
        j = draws[idx] % (i + 1)
        a[i], a[j] = a[j], a[i]
    return np.array(a, dtype=np.int64)


def iterate(state: State, intensities, positions, params: Params, n_iter, orders=None,
            sqrt_I=None):
    """Run n_iter pc-ePIE iterations (Fig. 1: one iteration is N loops over a
    random sequence S_n), split into consecutive batches of params.batch.

    After the last batch of an iteration the K > 1 probe modes are
    orthogonalised (reading) and the data error
      E_t = sum_n sum_q (sqrt(I_n) - A^G_n)^2 / sum_n sum_q I_n
    is recorded (reading of the NRMSE of Sec. 4.2, evaluated from the
    pre-update estimates).  Returns (new State, list of E_t).
    """
    if sqrt_I is None:
        sqrt_I = measured_amplitude(intensities, params)
    g = gaussian_kernel(params.sigma1, params.sigma2, params.kernel_size)
    denom = float(np.sum(sqrt_I ** 2))
    O, P, t = state.O.copy(), state.P.copy(), state.t
    n_pos = len(positions)
    errs = []
    for it in range(n_iter):
        t += 1
        order = permutation(params.seed, t, n_pos) if orders is None else np.asarray(orders[it])
        num = 0.0
        for s in range(0, n_pos, params.batch):
            batch = order[s:s + params.batch]
            O, P, e, _ = batch_step(O, P, sqrt_I, positions, batch, t, params, g)
            num += e
        if P.shape[0] > 1 and params.orthogonalize:
            P, _ = orthogonalize_modes(P)
        errs.append(num / denom if denom > 0 else 0.0)
    return State(O=O, P=P, t=t), errs


# ----------------------------------------------------------------------------
# Harness metrics (outside the method)
# ----------------------------------------------------------------------------

def illumination_roi(positions, P, obj_shape, frac=0.1):
    """Pixels where the summed illumination sum_n sum_k |P_k(r - r_n)|^2 >= frac * max."""
    n = P.shape[-1]
    illum = np.zeros(obj_shape)
    p2 = np.sum(np.abs(P) ** 2, axis=0)
    for (r, c) in positions:
        illum[int(r):int(r) + n, int(c):int(c) + n] += p2
    return illum >= frac * illum.max()


def nmse(o_rec, o_true, roi):
    """min_c sum_ROI |c o_rec - o_true|^2 / sum_ROI |o_true|^2 (global complex scalar removed)."""
    a = o_rec[roi]
    b = o_true[roi]
    den = np.vdot(a, a).real
    c = np.vdot(a, b) / den if den > 0 else 0.0
    return float(np.sum(np.abs(c * a - b) ** 2) / np.sum(np.abs(b) ** 2))
