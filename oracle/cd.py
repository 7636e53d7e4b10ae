"""Contour-deformation G0W0 quantities in plain FP64 (oracle; test
infrastructure only).

Paper sections cited: "Theory - Contour Deformation" (the split
Sigma = R - I, the residue term R and the imaginary-axis term I) and
"Implementation - Contour Deformation" (W in the auxiliary basis, the
polarizability Pi_PQ(omega), the dielectric matrix 1 - Pi, the imaginary-axis
integral I_nn, the residue term R_nn) and Algorithm 1 (CD-GW).

Closed shell, Hartree units.  Occupied states are 0..n_occ-1, virtual states
n_occ..n_mo-1, eps ascending.  B_ov[P, i*n_virt + a] = (P|ia) and
b = B_rows[r, m, :] = (P|nm) for the state n = row_ids[r].

Readings of the paper:
  * Pi carries the closed-shell spin sum (factor 2) and eta -> 0+, so at
    omega = i xi it is -4 sum_ia B_ia B_ia^T D/(D^2 + xi^2) and at real
    omega it is -4 sum_ia B_ia B_ia^T D/(D^2 - omega^2), D = eps_a - eps_i.
  * Only the correlation part W^c = W - v enters both terms
    (W^c = b^T [(1 - Pi)^-1 - 1] b); the bare part is the exchange
    self-energy, handled outside (dsig_x).
  * Real part of -I: -(1/pi) int_0^inf W^c(i xi) a/(a^2 + xi^2) d xi per m
    with a = omega - eps_m (the Sigma update of Algorithm 1).
  * Residue set (the equation for R): occupied m with eps_m > omega carry
    -W^c(eps_m - omega), virtual m with eps_m < omega carry
    +W^c(eps_m - omega); the step function takes the half-maximum value 1/2
    at 0 (Theory, Hedin equations paragraph).
"""
import numpy as np


def transition_energies(eps, n_occ):
    """D[i*n_virt + a] = eps_a - eps_i (the ia ordering of B_ov)."""
    eps = np.asarray(eps, dtype=np.float64)
    return (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)


def pi_imag(eps, n_occ, B_ov, xi):
    """Pi(i xi) = -4 B_ov diag(D / (D^2 + xi^2)) B_ov^T  [N_aux, N_aux]."""
    D = transition_energies(eps, n_occ)
    return -4.0 * (B_ov * (D / (D * D + xi * xi))) @ B_ov.T


def pi_real(eps, n_occ, B_ov, w):
    """Pi(w) for real w (principal value, eta -> 0+):
    -4 B_ov diag(D / (D^2 - w^2)) B_ov^T."""
    D = transition_energies(eps, n_occ)
    return -4.0 * (B_ov * (D / (D * D - w * w))) @ B_ov.T


def dpi_real_quadratic(eps, n_occ, B_ov, w, x):
    """x^T (dPi/dw) x at real w, from d/dw [D/(D^2 - w^2)] = 2 D w/(D^2 - w^2)^2."""
    D = transition_energies(eps, n_occ)
    u = B_ov.T @ x
    return -4.0 * float(np.sum(u * u * (2.0 * D * w / (D * D - w * w) ** 2)))


def screened_from_pi(Pi, b):
    """W^c = b^T [(1 - Pi)^-1 - 1] b with an explicit inverse.  b: [..., N_aux].

    The quadratic form is the row sum of (b X) * b: one matrix product with
    X = (1 - Pi)^-1 - 1, then a dot product of each row with its own b."""
    n = Pi.shape[0]
    X = np.linalg.inv(np.eye(n) - Pi) - np.eye(n)
    return np.sum((b @ X) * b, axis=-1)


def w_table(eps, n_occ, B_ov, B_rows, xi):
    """W^c_{nm}(i xi_g) for every supplied row n, every m and every grid point:
    array [n_rows, n_mo, G] (Algorithm 1: W(i omega') for all grid points)."""
    n_rows, n_mo, _ = B_rows.shape
    out = np.empty((n_rows, n_mo, len(xi)))
    for g, x in enumerate(xi):
        out[:, :, g] = screened_from_pi(pi_imag(eps, n_occ, B_ov, x), B_rows)
    return out


def step_half(x):
    """Heaviside step with the half-maximum convention theta(0) = 1/2."""
    return 1.0 if x > 0 else (0.5 if x == 0 else 0.0)


def residue_weights(eps, n_occ, omega):
    """f_m of the residue term R_nn(omega): -theta(eps_i - omega) for occupied,
    +theta(omega - eps_a) for virtual."""
    eps = np.asarray(eps, dtype=np.float64)
    f = np.zeros(eps.size)
    for m in range(eps.size):
        if m < n_occ:
            f[m] = -step_half(eps[m] - omega)
        else:
            f[m] = step_half(omega - eps[m])
    return f


def residue_value(eps, n_occ, B_ov, b, w):
    """W^c(w) = b^T[(1 - Pi(w))^-1 - 1] b and dW^c/dw at a real frequency w,
    by building 1 - Pi(w) and inverting it (what the paper's iterative solver
    avoids; here it is the definition).  eps: the eigenvalues in Pi."""
    n = B_ov.shape[0]
    Pi = pi_real(eps, n_occ, B_ov, w)
    Ainv = np.linalg.inv(np.eye(n) - Pi)
    x = Ainv @ b
    wc = float(b @ x - b @ b)
    # d/dw b^T A^-1 b = -b^T A^-1 (dA/dw) A^-1 b = x^T (dPi/dw) x
    dwc = dpi_real_quadratic(eps, n_occ, B_ov, w, x)
    return wc, dwc


def sigma_c(eps, n_occ, B_ov, b_row, wtab_row, xi, z, omega, derivative=True, eps_w=None,
            w0_row=None):
    """Re Sigma^c_nn(omega) and d/d omega of it for one state.

    eps:      the energies in G (poles eps_m: the quadrature's a = omega - eps_m,
              the residue set and the residue frequencies eps_m - omega)
    eps_w:    the energies in W (transition energies of Pi); None: eps
    b_row:    [n_mo, N_aux]  (P|nm) for every m
    wtab_row: [n_mo, G]      W^c_nm(i xi_g), built from eps_w
    w0_row:   [n_mo] W^c_nm(0), or None.  When given, the static part of each
              I integrand is integrated exactly, int_0^inf a/(a^2 + xi^2) d xi
              = (pi/2) sgn(a), and only W^c(i xi) - W^c(0) goes through the
              quadrature, which stays accurate as omega approaches a pole eps_m
    Returns (sigma, dsigma, n_residues).
    """
    if eps_w is None:
        eps_w = eps
    eps = np.asarray(eps, dtype=np.float64)
    a = omega - eps                                   # [n_mo]
    den = a[:, None] ** 2 + xi[None, :] ** 2          # [n_mo, G]
    wq = wtab_row if w0_row is None else wtab_row - np.asarray(w0_row)[:, None]
    sig = -(1.0 / np.pi) * float(np.sum(z[None, :] * wq * a[:, None] / den))
    if w0_row is not None:
        sig += -0.5 * float(np.sum(np.sign(a) * np.asarray(w0_row)))
    dsig = 0.0
    if derivative:
        dsig = -(1.0 / np.pi) * float(
            np.sum(z[None, :] * wq * (xi[None, :] ** 2 - a[:, None] ** 2) / den ** 2))
    f = residue_weights(eps, n_occ, omega)
    nres = 0
    for m in range(eps.size):
        if f[m] == 0.0:
            continue
        nres += 1
        wc, dwc = residue_value(eps_w, n_occ, B_ov, b_row[m], eps[m] - omega)
        sig += f[m] * wc
        # the residue frequency eps_m - omega moves opposite to omega
        dsig += -f[m] * dwc
    return sig, dsig, nres
