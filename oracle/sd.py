"""Spectral-decomposition (Casida RPA) route (oracle; test infrastructure
only).  It does not touch the contour-deformation code and serves as the
independent pin for it.

Paper: "Theory - Spectral Decomposition" (Casida equations, W from the
excitation vectors, Sigma_nn as a sum over poles) and "Implementation -
Spectral Decomposition" (the Hermitian form
(A-B)^1/2 (A+B) (A-B)^1/2 T = Omega^2 T with A - B = D diagonal and
A + B = D + 4 B_ov^T B_ov in the fitted basis).

With T orthonormal and (X+Y)_s = D^1/2 T_s / Omega_s^1/2, the correlation
part of W becomes, for every frequency z (z^2 = -xi^2 on the imaginary axis),
  W^c_nm(z) = -sum_s rho_s^2 / (Omega_s^2 - z^2),  rho_s = 2 b^T B_ov D^1/2 T_s,
i.e. pole weights (w^s_nm)^2 = rho_s^2 / (2 Omega_s) in the paper's pole form
(the factor 2 over the paper's open-shell w is the closed-shell spin sum), and
  Re Sigma^c_nn(omega) = sum_s [ sum_i w_ni^2 / (omega - eps_i + Omega_s)
                                + sum_a w_na^2 / (omega - eps_a - Omega_s) ].
"""
import numpy as np


def casida(eps, n_occ, B_ov):
    """Excitation energies Omega [N_ov] and orthonormal T [N_ov, N_ov]."""
    eps = np.asarray(eps, dtype=np.float64)
    D = (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)
    sD = np.sqrt(D)
    M = np.diag(D * D) + 4.0 * sD[:, None] * (B_ov.T @ B_ov) * sD[None, :]
    om2, T = np.linalg.eigh(M)
    if om2.min() <= 0:
        raise ValueError("RPA instability: non-positive Omega^2")
    return np.sqrt(om2), T, D


def pole_strengths(B_ov, D, T, b):
    """rho[..., s] = 2 b^T B_ov D^1/2 T_s for b [..., N_aux]."""
    return 2.0 * ((b @ B_ov) * np.sqrt(D)) @ T


def screened(rho, Omega, z2):
    """W^c(z) = -sum_s rho_s^2 / (Omega_s^2 - z^2), z2 = z^2 (real)."""
    return -np.sum(rho * rho / (Omega * Omega - z2), axis=-1)


def sigma_c(eps, n_occ, rho_row, Omega, omega):
    """Re Sigma^c_nn(omega) and its derivative from the pole form.

    rho_row: [n_mo, N_ov] pole strengths of b = (P|nm) for every m.
    """
    eps = np.asarray(eps, dtype=np.float64)
    w2 = rho_row * rho_row / (2.0 * Omega[None, :])
    sig = 0.0
    dsig = 0.0
    for m in range(eps.size):
        if m < n_occ:
            den = omega - eps[m] + Omega
        else:
            den = omega - eps[m] - Omega
        sig += float(np.sum(w2[m] / den))
        dsig += float(np.sum(-w2[m] / (den * den)))
    return sig, dsig


def casida_uhf(eps, n_occ, B_ov):
    """Open-shell excitations from the spin-block Casida equations ("Theory -
    Spectral Decomposition"): with K_{ia s1, jb s2} = (ia s1|jb s2) =
    sum_P B^P_{ia s1} B^P_{jb s2} over both spins, A = D + K and B = K, so
    A - B = D and A + B = D + 2 K in the stacked (up, down) transition space.
    Returns Omega, orthonormal T, the stacked D and the stacked B_ov
    [N_aux, N_ov_up + N_ov_down]."""
    Ds, Bs = [], []
    for s in (0, 1):
        e = np.asarray(eps[s], dtype=np.float64)
        Ds.append((e[None, n_occ[s]:] - e[:n_occ[s], None]).reshape(-1))
        Bs.append(np.asarray(B_ov[s], dtype=np.float64))
    D = np.concatenate(Ds)
    Bc = np.concatenate(Bs, axis=1)
    sD = np.sqrt(D)
    M = np.diag(D * D) + 2.0 * sD[:, None] * (Bc.T @ Bc) * sD[None, :]
    om2, T = np.linalg.eigh(M)
    if om2.min() <= 0:
        raise ValueError("RPA instability: non-positive Omega^2")
    return np.sqrt(om2), T, D, Bc


def pole_strengths_uhf(Bc, D, T, b):
    """rho[..., s] with rho_s^2 / (2 Omega_s) = (w^s)^2, the paper's open-shell
    pole weight w^s = sum (mn|ia s')(X + Y)^s_{ia s'}, (X + Y) = D^1/2 T
    Omega^-1/2: rho_s = sqrt(2) b^T B D^1/2 T_s."""
    return np.sqrt(2.0) * ((b @ Bc) * np.sqrt(D)) @ T


def poles(eps, n_occ, Omega):
    """All pole positions of Sigma^c: eps_i - Omega_s and eps_a + Omega_s."""
    eps = np.asarray(eps, dtype=np.float64)
    return np.sort(np.concatenate([(eps[:n_occ, None] - Omega[None, :]).ravel(),
                                   (eps[n_occ:, None] + Omega[None, :]).ravel()]))
