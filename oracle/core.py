"""FP64 oracle of the MAGPIE hot path (arXiv 2504.10118).  Test infrastructure only.

Notation follows the paper: object ``z`` (n x n), probe ``Q`` (m x m), scan
extraction ``P_k`` given by top-left offsets, data ``d_k`` (here passed as
``sqrt_d`` = sqrt(d_k)), revised exit wave ``R_k``, regularisation vector ``u``,
restriction ``I_h^H`` (``restrict``) and prolongation ``I_H^h`` (``prolong``).

Readings of points the paper leaves open (each also listed in the design notes):

* DFT convention (Section 2.1 says only "2-D DFT"): numpy's, i.e. forward
  kernel exp(-2 pi i (a x + b y) / m), unnormalised, zero frequency at [0, 0];
  the inverse is F^* / m^2 as Appendix A derives.
* theta(0) := 0 (Definition 2.1 footnote), so the revised exit wave takes the
  measured modulus with zero phase where F(Q z_k) vanishes exactly.  The
  phase-recycling rule of eq. (3.2) is an option of the driver (``phases``):
  where F(Q z_k) vanishes, the phase of position k's previous visit is used,
  and theta = 0 before its first visit; "iteration j" of eq. (3.2) is read as
  the j-th visit of position k.
* Objective is reported in exit-wave form, eq. (2.1); the amplitude form
  printed before it is m^2 times larger (Appendix B.1).
* Restriction is 2x2 average pooling on bins aligned to the patch origin
  (the matrix of eq. (2.5) is garbled in print; the text calls it binning by
  average pooling and Lemma E.4's proof uses bins of 4 entries).
* "L levels" means L grids in total: the fine grid and L-1 coarse grids, so
  L = 1 is rPIE (Alg 1) and L = 2 is the two-level MAGPS of Section 4.1.
* Division by zero in the weights of eq. (4.4): where the bin sum of |Q|^2
  vanishes, W_z := 1 and W_R := 0; where it vanishes on the coarse grid,
  W_u := 0; where u + |Q|^2 vanishes the proximal coefficient
  conj(Q) / (u + |Q|^2) := 0.  W_R is evaluated with Q's singular division
  cancelled: (I_H^h Q_H) conj(Q) / (I_H^h I_h^H |Q|^2), as Section 4.1's
  "Well-definedness" paragraph intends.
* Minibatches (the paper is sequential; a minibatch variant is named as future
  work in the Conclusion): all positions of a minibatch read the same z, each
  runs Alg 3, and the per-pixel precision-weighted average of the updates is
  applied: z <- z + sum_k P_k^T(w0 * dz_k) / sum_k P_k^T w0, w0 = u + |Q|^2,
  on pixels with a positive denominator.  With one position per minibatch this
  is Alg 4 exactly; with one level it is the exact proximal minimiser of the
  minibatch surrogate (eqs. (3.4)-(3.5)).

Pins (tests/test_oracle_*.py): brute-force DFT, Parseval, the objective
identity, finite-difference gradients, Lemma C.1 / Prop 3.1 majorisation,
Prop 3.2 descent, Prop 3.3 bound, Lemmas E.1-E.4, Props 4.1, 4.2, 4.4
(as an inequality), Thm 4.3 and eq. (4.6), the rPIE special case, literal
Alg 3 == gradient form, fixed point at the truth, recovery, the
splitmix64 published test vector, and u^rPIE and the stopping statistic of
Section 5 on hand-worked values.  The minibatch combination for L >= 2 and
B >= 2 is "parity unpinned" beyond its two pinned special cases (B = 1 and
L = 1); the probe update is beyond the paper and likewise unpinned except by
its own descent property.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "fft2", "ifft2", "extract", "scatter_add", "forward_model",
    "phase_factor", "revised_exit_wave", "phi_k", "objective",
    "objective_amplitude", "grad_k", "full_gradient", "surrogate_k",
    "pie_surrogate_k", "surrogate", "u_rpie", "rpie_update", "restrict",
    "prolong", "weights", "weights_literal", "magps", "level_constants",
    "magps_gradient_form", "minibatch_step", "run_epochs",
    "magpie_sequential", "rpie_sequential", "stopping_statistic",
    "illumination", "error_paper", "error_relative", "splitmix64",
    "library_permutation", "batches", "full_batch_surrogate_minimiser",
    "probe_update_step", "blind_minibatch_step", "run_epochs_blind",
    "phase_factor_recycled", "revised_exit_wave_recycled", "initial_phases", "error_scaled",
]

M64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# Discrete Fourier transform (Section 2.1; Appendix A: F^{-1} = F^* / m^2)
# --------------------------------------------------------------------------
def fft2(v: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D DFT over the last two axes (library primitive)."""
    return np.fft.fft2(np.asarray(v, dtype=np.complex128), axes=(-2, -1))


def ifft2(v: np.ndarray) -> np.ndarray:
    """Inverse 2-D DFT, F^* / m^2 (Appendix A)."""
    return np.fft.ifft2(np.asarray(v, dtype=np.complex128), axes=(-2, -1))


# --------------------------------------------------------------------------
# Scan extraction P_k and its transpose (Section 2.1)
# --------------------------------------------------------------------------
def extract(z: np.ndarray, off, m: int) -> np.ndarray:
    """z_k = P_k z: the m x m window whose top-left corner is ``off``."""
    r, c = int(off[0]), int(off[1])
    return np.array(z[r:r + m, c:c + m], dtype=np.complex128, copy=True)


def scatter_add(acc: np.ndarray, off, patch: np.ndarray) -> None:
    """acc += P_k^T patch (in place)."""
    m = patch.shape[0]
    r, c = int(off[0]), int(off[1])
    acc[r:r + m, c:c + m] += patch


def forward_model(z: np.ndarray, Q: np.ndarray, offsets) -> np.ndarray:
    """Noiseless intensities d_k = |F(Q * P_k z)|^2 (Section 2.1), float64 [N, m, m]."""
    m = Q.shape[0]
    return np.stack([np.abs(fft2(Q * extract(z, o, m))) ** 2 for o in offsets])


# --------------------------------------------------------------------------
# Revised exit wave (Definition 2.1, theta(0) := 0 per its footnote)
# --------------------------------------------------------------------------
def phase_factor(Psi: np.ndarray) -> np.ndarray:
    """exp(i theta(Psi)) elementwise, with theta(0) = 0."""
    out = np.ones_like(Psi, dtype=np.complex128)
    nz = Psi != 0
    out[nz] = Psi[nz] / np.abs(Psi[nz])
    return out


def revised_exit_wave(zk: np.ndarray, Q: np.ndarray, sqrt_dk: np.ndarray) -> np.ndarray:
    """R_k(z_k) = F^{-1}(sqrt(d_k) * exp(i theta(F(Q * z_k))))."""
    Psi = fft2(Q * zk)
    return ifft2(sqrt_dk * phase_factor(Psi))


def phase_factor_recycled(Psi: np.ndarray, previous: np.ndarray) -> np.ndarray:
    """exp(i theta) with the specification of eq. (3.2): Psi / |Psi| where Psi is
    nonzero, and where it vanishes the factor of the position's previous visit
    (``previous``; all ones before the first visit, i.e. theta = 0)."""
    out = np.array(previous, dtype=np.complex128, copy=True)
    nz = Psi != 0
    out[nz] = Psi[nz] / np.abs(Psi[nz])
    return out


def revised_exit_wave_recycled(zk, Q, sqrt_dk, previous):
    """(R_k(z_k), phase factor used) under eq. (3.2)."""
    ph = phase_factor_recycled(fft2(Q * zk), previous)
    return ifft2(sqrt_dk * ph), ph


# --------------------------------------------------------------------------
# Objective (eq. 2.1) and its amplitude form (Section 2.1)
# --------------------------------------------------------------------------
def phi_k(zk, Q, sqrt_dk) -> float:
    """Phi_k(z_k) = 1/2 ||Q * z_k - R_k(z_k)||^2 (eq. 2.1)."""
    return 0.5 * float(np.sum(np.abs(Q * zk - revised_exit_wave(zk, Q, sqrt_dk)) ** 2))


def objective(z, Q, offsets, sqrt_d) -> float:
    """Phi(z) = sum_k Phi_k(P_k z) (eq. 2.1)."""
    m = Q.shape[0]
    return float(sum(phi_k(extract(z, o, m), Q, sqrt_d[k]) for k, o in enumerate(offsets)))


def objective_amplitude(z, Q, offsets, sqrt_d) -> float:
    """1/2 sum_k || |F(Q * P_k z)| - sqrt(d_k) ||^2, the form printed before eq. 2.1."""
    m = Q.shape[0]
    tot = 0.0
    for k, o in enumerate(offsets):
        tot += 0.5 * float(np.sum((np.abs(fft2(Q * extract(z, o, m))) - sqrt_d[k]) ** 2))
    return tot


# --------------------------------------------------------------------------
# Gradients (eq. 2.2 and the full gradient after it)
# --------------------------------------------------------------------------
def grad_k(zk, Q, sqrt_dk) -> np.ndarray:
    """nabla_{z_k} Phi_k = conj(Q) * (Q * z_k - R_k(z_k)) (eq. 2.2)."""
    return np.conj(Q) * (Q * zk - revised_exit_wave(zk, Q, sqrt_dk))


def full_gradient(z, Q, offsets, sqrt_d) -> np.ndarray:
    """nabla Phi(z) = sum_k P_k^T nabla Phi_k(P_k z)."""
    m = Q.shape[0]
    g = np.zeros(z.shape, dtype=np.complex128)
    for k, o in enumerate(offsets):
        scatter_add(g, o, grad_k(extract(z, o, m), Q, sqrt_d[k]))
    return g


# --------------------------------------------------------------------------
# Surrogates (eq. 2.4 PIE surrogate, eq. 3.1 quadratic surrogate)
# --------------------------------------------------------------------------
def surrogate_k(zk, zk_j, Q, sqrt_dk) -> float:
    """Phi~_k(z_k; z_k^(j)) = 1/2 ||Q * z_k - R_k(z_k^(j))||^2 (eq. 3.1)."""
    return 0.5 * float(np.sum(np.abs(Q * zk - revised_exit_wave(zk_j, Q, sqrt_dk)) ** 2))


def pie_surrogate_k(zk, zk_j, Q, sqrt_dk, u) -> float:
    """Phi^PIE_k = Phi~_k + 1/2 u^T |z_k - z_k^(j)|^2 (eq. 2.4)."""
    return surrogate_k(zk, zk_j, Q, sqrt_dk) + 0.5 * float(np.sum(u * np.abs(zk - zk_j) ** 2))


def surrogate(z, zj, Q, offsets, sqrt_d) -> float:
    """Phi~(z; z^(j)) = sum_k Phi~_k(P_k z; P_k z^(j)) (eq. 3.1)."""
    m = Q.shape[0]
    return float(sum(surrogate_k(extract(z, o, m), extract(zj, o, m), Q, sqrt_d[k])
                     for k, o in enumerate(offsets)))


# --------------------------------------------------------------------------
# rPIE (Section 2.1: u^rPIE, eq. 2.3, Alg 1)
# --------------------------------------------------------------------------
def u_rpie(Q, alpha) -> np.ndarray:
    """u^rPIE = alpha (||Q||_inf^2 J - |Q|^2)."""
    A = np.abs(Q) ** 2
    return alpha * (A.max() - A)


def rpie_update(zk, Q, Rk, u) -> np.ndarray:
    """z_k^+ = z_k + conj(Q) / (u + |Q|^2) * (R_k - Q * z_k) (eq. 2.3)."""
    return zk + np.conj(Q) / (u + np.abs(Q) ** 2) * (Rk - Q * zk)


# --------------------------------------------------------------------------
# Restriction and prolongation (eqs. 2.5, 2.6)
# --------------------------------------------------------------------------
def restrict(a: np.ndarray) -> np.ndarray:
    """I_h^H: average of each 2x2 bin (bins aligned to index 0)."""
    return 0.25 * (a[0::2, 0::2] + a[1::2, 0::2] + a[0::2, 1::2] + a[1::2, 1::2])


def prolong(a: np.ndarray) -> np.ndarray:
    """I_H^h = 4 (I_h^H)^T: copy each coarse value into its 2x2 bin."""
    return np.repeat(np.repeat(a, 2, axis=0), 2, axis=1)


# --------------------------------------------------------------------------
# Weights (eq. 4.4; Alg 3 coarse-level preparation)
# --------------------------------------------------------------------------
def weights(Q):
    """Q_H, W_z, W_R, W_u^H of eq. (4.4), with the zero-division readings above."""
    A = np.abs(Q) ** 2
    S = restrict(A)                      # I_h^H |Q|^2
    QH = restrict(Q)                     # Q_H = I_h^H Q
    PS = prolong(S)                      # I_H^h I_h^H |Q|^2
    pos = PS > 0
    Wz = np.ones_like(A)
    Wz[pos] = A[pos] / PS[pos]
    WR = np.zeros_like(Q, dtype=np.complex128)
    WR[pos] = prolong(QH)[pos] * np.conj(Q[pos]) / PS[pos]
    Wu = np.zeros_like(S)
    Wu[S > 0] = np.abs(QH[S > 0]) ** 2 / S[S > 0]
    return QH, Wz, WR, Wu


def weights_literal(Q):
    """Eq. (4.4) exactly as printed: W_R = (I_H^h Q_H) * W_z / Q.  Needs Q != 0."""
    A = np.abs(Q) ** 2
    S = restrict(A)
    QH = restrict(Q)
    Wz = A / prolong(S)
    WR = prolong(QH) * Wz / Q
    Wu = np.abs(QH) ** 2 / S
    return QH, Wz, WR, Wu


# --------------------------------------------------------------------------
# MAGPS (Alg 3), literal recursive form
# --------------------------------------------------------------------------
def _prox_coefficient(Q, u):
    w = u + np.abs(Q) ** 2
    C = np.zeros_like(Q, dtype=np.complex128)
    pos = w > 0
    C[pos] = np.conj(Q[pos]) / w[pos]
    return C


def magps(zk, Q, Rk, u, levels: int) -> np.ndarray:
    """Alg 3 on one patch.  ``levels`` = grids left including this one (1 = coarsest)."""
    C = _prox_coefficient(Q, u)
    if levels <= 1:
        # coarsest level: one proximal (rPIE) step
        return zk + C * (Rk - Q * zk)
    # coarse-level preparation
    QH, Wz, WR, Wu = weights(Q)
    zH = restrict(Wz * zk)
    RH = restrict(WR * Rk)
    uH = Wu * restrict(u)
    # recursive coarse solve
    zH_hat = magps(zH, QH, RH, uH, levels - 1)
    # coarse-to-fine update
    eH = zH_hat - zH
    z_tilde = zk + prolong(eH)
    # post-smoothing
    return z_tilde + C * (Rk - Q * z_tilde)


# --------------------------------------------------------------------------
# MAGPS, gradient form (what the GPU computes).  Derived from the proof of
# Thm 4.3 (Appendix H): Q_H z_H - R_H = (Q_H / I|Q|^2) * I(g) by Lemma E.1,
# so each level only needs the restricted gradient.  Equality with ``magps``
# is pinned by a test.
# --------------------------------------------------------------------------
def level_constants(Q, u, levels: int):
    """Per-level constants of the gradient form.

    Returns dict with w0 = u + |Q|^2, u0 = u and, for l = 1..L-1, tuples
    (V_l, rho_l, r_l): V_l = W_u at the transfer into level l, and with
    hat-quantities u^_l = I(u_{l-1}), w^_l = I(w_{l-1}):
    rho_l = u^_l / w^_l, r_l = 1 / w^_l where V_l > 0 and w^_l > 0, else
    rho_l = 1, r_l = 0 (the literal step then has a zero proximal coefficient).
    """
    out = {"w0": u + np.abs(Q) ** 2, "u0": np.array(u, dtype=np.float64), "levels": []}
    Ql, ul = Q, np.array(u, dtype=np.float64)
    for _ in range(1, levels):
        QH, _, _, Wu = weights(Ql)
        wl = ul + np.abs(Ql) ** 2
        w_hat = restrict(wl)
        u_hat = restrict(ul)
        ok = (Wu > 0) & (w_hat > 0)
        rho = np.ones_like(w_hat)
        r = np.zeros_like(w_hat)
        rho[ok] = u_hat[ok] / w_hat[ok]
        r[ok] = 1.0 / w_hat[ok]
        out["levels"].append((Wu, rho, r))
        Ql, ul = QH, Wu * u_hat
    return out


def magps_gradient_form(zk, Q, Rk, consts) -> np.ndarray:
    """Returns c_k = w0 * (MAGPS(z_k) - z_k) computed from the gradient g0 = conj(Q)(Q z_k - R_k)."""
    g0 = np.conj(Q) * (Q * zk - Rk)
    lv = consts["levels"]
    L = len(lv) + 1
    if L == 1:
        return -g0
    ghat = [None] * L
    ghat[1] = restrict(g0)
    for l in range(1, L - 1):
        V = lv[l - 1][0]
        ghat[l + 1] = restrict(V * ghat[l])
    _, rho, r = lv[L - 2]
    e = -r * ghat[L - 1]
    for l in range(L - 2, 0, -1):
        _, rho, r = lv[l - 1]
        e = rho * prolong(e) - r * ghat[l]
    return consts["u0"] * prolong(e) - g0


# --------------------------------------------------------------------------
# Stochastic driver: Alg 4 (sequential) and the minibatch reading
# --------------------------------------------------------------------------
def batches(order, B: int):
    """Consecutive chunks of B positions of an epoch's permutation (last one short)."""
    order = list(order)
    return [order[t:t + B] for t in range(0, len(order), B)]


def minibatch_step(z, Q, offsets, sqrt_d, u, levels: int, batch, use_gradient_form=False, phases=None):
    """One minibatch step: every k in ``batch`` runs Alg 3 on the same z, updates are
    averaged with precision weights w0 = u + |Q|^2 and applied where the weight sum > 0.
    ``phases`` ([N][m][m] complex, updated in place): eq. (3.2) phase recycling."""
    m = Q.shape[0]
    w0 = u + np.abs(Q) ** 2
    num = np.zeros(z.shape, dtype=np.complex128)
    den = np.zeros(z.shape, dtype=np.float64)
    consts = level_constants(Q, u, levels) if use_gradient_form else None
    for k in batch:
        o = offsets[k]
        zk = extract(z, o, m)
        if phases is None:
            Rk = revised_exit_wave(zk, Q, sqrt_d[k])
        else:
            Rk, phases[k] = revised_exit_wave_recycled(zk, Q, sqrt_d[k], phases[k])
        if use_gradient_form:
            ck = magps_gradient_form(zk, Q, Rk, consts)
        else:
            ck = w0 * (magps(zk, Q, Rk, u, levels) - zk)
        scatter_add(num, o, ck)
        scatter_add(den, o, w0)
    znew = np.array(z, dtype=np.complex128, copy=True)
    pos = den > 0
    znew[pos] += num[pos] / den[pos]
    return znew


def initial_phases(n_pos: int, m: int) -> np.ndarray:
    """Phase factors before any visit: theta = 0 (eq. 3.2, j = 0)."""
    return np.ones((n_pos, m, m), dtype=np.complex128)


def run_epochs(z0, Q, offsets, sqrt_d, u, levels: int, orders, B: int,
               use_gradient_form=False, callback=None, phases=None):
    """Epochs of minibatch MAGPIE over the given permutations (one per epoch); with
    ``phases`` (see ``initial_phases``, updated in place) eq. (3.2) phase recycling."""
    z = np.array(z0, dtype=np.complex128, copy=True)
    for e, order in enumerate(orders):
        for batch in batches(order, B):
            z = minibatch_step(z, Q, offsets, sqrt_d, u, levels, batch, use_gradient_form, phases)
        if callback is not None:
            callback(e, z)
    return z


def magpie_sequential(z0, Q, offsets, sqrt_d, u, levels: int, orders):
    """Alg 4: for each epoch, visit positions in the given order and replace z_k by MAGPS_k."""
    m = Q.shape[0]
    z = np.array(z0, dtype=np.complex128, copy=True)
    for order in orders:
        for k in order:
            o = offsets[k]
            zk = extract(z, o, m)
            Rk = revised_exit_wave(zk, Q, sqrt_d[k])
            r, c = int(o[0]), int(o[1])
            z[r:r + m, c:c + m] = magps(zk, Q, Rk, u, levels)
    return z


def rpie_sequential(z0, Q, offsets, sqrt_d, alpha, orders):
    """Alg 1 (rPIE) written as the textbook loop with eq. (2.3)."""
    m = Q.shape[0]
    u = u_rpie(Q, alpha)
    z = np.array(z0, dtype=np.complex128, copy=True)
    for order in orders:
        for k in order:
            o = offsets[k]
            zk = extract(z, o, m)
            Rk = revised_exit_wave(zk, Q, sqrt_d[k])
            r, c = int(o[0]), int(o[1])
            z[r:r + m, c:c + m] = rpie_update(zk, Q, Rk, u)
    return z


def full_batch_surrogate_minimiser(z, Q, offsets, sqrt_d):
    """Exact minimiser of eq. (3.1) with u = 0 (eq. 3.3): z_p = sum P^T conj(Q) R / sum P^T |Q|^2.

    Pixels never illuminated keep their value.
    """
    m = Q.shape[0]
    num = np.zeros(z.shape, dtype=np.complex128)
    den = np.zeros(z.shape, dtype=np.float64)
    for k, o in enumerate(offsets):
        zk = extract(z, o, m)
        scatter_add(num, o, np.conj(Q) * revised_exit_wave(zk, Q, sqrt_d[k]))
        scatter_add(den, o, np.abs(Q) ** 2)
    znew = np.array(z, dtype=np.complex128, copy=True)
    pos = den > 0
    znew[pos] = num[pos] / den[pos]
    return znew


# --------------------------------------------------------------------------
# Probe update (beyond the paper: blind ptychography is future work in its
# Conclusion).  Simultaneous with the object step, from the same z and R_k:
#   Q <- Q + sum_k conj(z_k) (R_k - Q z_k) / sum_k (|z_k|^2 + beta max|z_k|^2)
# The denominator is the per-pixel curvature of sum_k Phi~_k in Q plus a
# proximal term, so for one minibatch the probe step is the proximal
# minimiser of the minibatch surrogate in Q (parity unpinned beyond that).
# --------------------------------------------------------------------------
def probe_update_step(z, Q, offsets, sqrt_d, batch, beta):
    m = Q.shape[0]
    num = np.zeros(Q.shape, dtype=np.complex128)
    den = np.zeros(Q.shape, dtype=np.float64)
    for k in batch:
        zk = extract(z, offsets[k], m)
        Rk = revised_exit_wave(zk, Q, sqrt_d[k])
        a = np.abs(zk) ** 2
        num += np.conj(zk) * (Rk - Q * zk)
        den += a + beta * a.max()
    Qn = np.array(Q, dtype=np.complex128, copy=True)
    pos = den > 0
    Qn[pos] += num[pos] / den[pos]
    return Qn


def blind_minibatch_step(z, Q, offsets, sqrt_d, alpha, levels: int, batch, beta, u=None, alternate=False):
    """Object step (minibatch MAGPS) and probe step.  Simultaneous (default): both from the
    same (z, Q).  Alternating: the probe step is taken at the new object, so each half step
    is a proximal majorisation-minimisation step in its own variable (Lemma C.1 applied to
    z, then to Q) and, with one grid, the minibatch's partial objective cannot increase.

    u = u^rPIE(Q, alpha) of the current probe unless a fixed u is given.
    """
    uu = u_rpie(Q, alpha) if u is None else u
    znew = minibatch_step(z, Q, offsets, sqrt_d, uu, levels, batch)
    Qnew = probe_update_step(znew if alternate else z, Q, offsets, sqrt_d, batch, beta)
    return znew, Qnew


def run_epochs_blind(z0, Q0, offsets, sqrt_d, alpha, levels: int, orders, B: int, beta, u=None,
                     alternate=False):
    """Epochs of minibatch MAGPIE with the probe step after every minibatch."""
    z = np.array(z0, dtype=np.complex128, copy=True)
    Q = np.array(Q0, dtype=np.complex128, copy=True)
    for order in orders:
        for batch in batches(order, B):
            z, Q = blind_minibatch_step(z, Q, offsets, sqrt_d, alpha, levels, batch, beta, u, alternate)
    return z, Q


# --------------------------------------------------------------------------
# Evaluation (Section 5: stopping criterion, quality metrics)
# --------------------------------------------------------------------------
def stopping_statistic(z, Q, offsets, sqrt_d) -> float:
    """(1 / (N m)) sum_k ||nabla_{z_k} Phi_k(z_k)||_2 (Section 5, "Stopping criterion")."""
    m = Q.shape[0]
    N = len(offsets)
    tot = 0.0
    for k, o in enumerate(offsets):
        tot += float(np.linalg.norm(grad_k(extract(z, o, m), Q, sqrt_d[k])))
    return tot / (N * m)


def illumination(shape, Q, offsets) -> np.ndarray:
    """sum_k P_k^T |Q|^2 (the quantity in Prop 3.3)."""
    acc = np.zeros(shape, dtype=np.float64)
    A = np.abs(Q) ** 2
    for o in offsets:
        scatter_add(acc, o, A)
    return acc


def error_paper(z, z_true, mask=None) -> float:
    """|| |z| - |z*| ||_2 (Section 5, "Quality metrics"), optionally on a mask."""
    d = np.abs(z) - np.abs(z_true)
    if mask is not None:
        d = d[mask]
    return float(np.linalg.norm(d))


def error_relative(z, z_true, mask) -> float:
    """min_phi ||e^{i phi} z - z*||_M / ||z*||_M with phi = arg <z, z*>_M (global phase removed)."""
    a = z[mask]
    b = z_true[mask]
    ip = np.vdot(a, b)
    ph = np.exp(1j * np.angle(ip)) if ip != 0 else 1.0
    return float(np.linalg.norm(ph * a - b) / np.linalg.norm(b))


def error_scaled(z, z_true, mask) -> float:
    """min_c ||c z - z*||_M / ||z*||_M over complex scalars c: with the probe also unknown,
    (c z, Q / c) explain the same data, so only z up to a complex scale is determined;
    c = <z, z*>_M / <z, z>_M (least squares)."""
    a = z[mask]
    b = z_true[mask]
    den = np.vdot(a, a)
    c = np.vdot(a, b) / den if den != 0 else 0.0
    return float(np.linalg.norm(c * a - b) / np.linalg.norm(b))


# --------------------------------------------------------------------------
# splitmix64 (Steele, Lea, Flood 2014) and the library's epoch permutation
# --------------------------------------------------------------------------
def splitmix64(state: int):
    """Yields (new_state, output) pairs of the splitmix64 generator."""
    while True:
        state = (state + 0x9E3779B97F4A7C15) & M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        yield z ^ (z >> 31)


def library_permutation(seed: int, epoch: int, n: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1 driven by splitmix64 seeded with seed XOR epoch.

    For i = n-1 down to 1: j = next() mod (i + 1); swap(perm[i], perm[j]).
    """
    gen = splitmix64((int(seed) ^ int(epoch)) & M64)
    perm = list(range(n))
    for i in range(n - 1, 0, -1):
        j = next(gen) % (i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return np.array(perm, dtype=np.int32)
