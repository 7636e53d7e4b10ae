"""Open-shell (spin-resolved) contour-deformation G0W0 in plain FP64 (oracle;
test infrastructure only).

Paper: "Implementation - Contour Deformation": the polarizability
Pi_PQ(omega) carries an explicit sum over the spin sigma of the transitions
i sigma -> a sigma, the screened interaction W_{mn sigma, mn sigma} is formed
from (mn sigma|P) in the same auxiliary basis, and I_{nn sigma} sums over the
orbitals m of the state's own spin; "Theory - Spectral Decomposition": the
Kohn-Sham Green's function is diagonal in spin.

Spin 0 is up, spin 1 down.  Per spin s: eps[s] [n_mo] (ascending), n_occ[s]
occupied levels, B_ov[s] [N_aux, n_occ_s * n_virt_s] with column
i * n_virt_s + a.  A state is named by its spin-orbital index s * n_mo + n;
its row b = (P|n m s) [n_mo, N_aux] runs over the orbitals m of spin s.

Readings:
  * Pi(i xi) = -2 sum_s B_s diag(D_s / (D_s^2 + xi^2)) B_s^T: the two
    time orderings of each spin's transitions give the 2; closed shell (both
    spins equal) gives the -4 of the closed-shell reading;
  * W^c does not depend on the state's spin beyond its row b;
  * the residue set, the residue frequencies and the quadrature of state
    (n, s) use the levels and the occupation of spin s only.
"""
import numpy as np

from . import cd


def _D(eps_s, n_occ_s):
    eps_s = np.asarray(eps_s, dtype=np.float64)
    return (eps_s[None, n_occ_s:] - eps_s[:n_occ_s, None]).reshape(-1)


def pi_imag(eps, n_occ, B_ov, xi):
    """Pi(i xi) = -2 sum_s B_s diag(D_s / (D_s^2 + xi^2)) B_s^T."""
    out = 0.0
    for s in (0, 1):
        D = _D(eps[s], n_occ[s])
        out = out - 2.0 * (B_ov[s] * (D / (D * D + xi * xi))) @ B_ov[s].T
    return out


def pi_real(eps, n_occ, B_ov, w):
    """Pi(w) at real w (principal value): -2 sum_s B_s diag(D_s/(D_s^2 - w^2)) B_s^T."""
    out = 0.0
    for s in (0, 1):
        D = _D(eps[s], n_occ[s])
        out = out - 2.0 * (B_ov[s] * (D / (D * D - w * w))) @ B_ov[s].T
    return out


def dpi_real_quadratic(eps, n_occ, B_ov, w, x):
    """x^T (dPi/dw) x at real w."""
    tot = 0.0
    for s in (0, 1):
        D = _D(eps[s], n_occ[s])
        u = B_ov[s].T @ x
        tot += -2.0 * float(np.sum(u * u * (2.0 * D * w / (D * D - w * w) ** 2)))
    return tot


def w_table(eps, n_occ, B_ov, B_rows, xi):
    """W^c [n_rows, n_mo, G] from an explicit inverse of 1 - Pi(i xi_g)."""
    n_rows, n_mo, _ = B_rows.shape
    out = np.empty((n_rows, n_mo, len(xi)))
    for g, x in enumerate(xi):
        out[:, :, g] = cd.screened_from_pi(pi_imag(eps, n_occ, B_ov, x), B_rows)
    return out


def residue_value(eps, n_occ, B_ov, b, w):
    """W^c(w) and dW^c/dw at a real frequency, explicit inverse."""
    n = b.shape[-1]
    Ainv = np.linalg.inv(np.eye(n) - pi_real(eps, n_occ, B_ov, w))
    x = Ainv @ b
    return float(b @ x - b @ b), dpi_real_quadratic(eps, n_occ, B_ov, w, x)


def sigma_c(eps, n_occ, B_ov, spin, b_row, wtab_row, xi, z, omega):
    """Re Sigma^c of a state of spin `spin` at omega, and its derivative:
    -(1/pi) sum_m sum_g z_g W^c_nm(i xi_g) a/(a^2 + xi_g^2), a = omega - eps_m,
    plus the residues f_m W^c(eps_m - omega), m over the orbitals of `spin`.
    Returns (sigma, dsigma, n_residues)."""
    e = np.asarray(eps[spin], dtype=np.float64)
    a = omega - e
    den = a[:, None] ** 2 + xi[None, :] ** 2
    sig = -(1.0 / np.pi) * float(np.sum(z[None, :] * wtab_row * a[:, None] / den))
    dsig = -(1.0 / np.pi) * float(
        np.sum(z[None, :] * wtab_row * (xi[None, :] ** 2 - a[:, None] ** 2) / den ** 2))
    f = cd.residue_weights(e, n_occ[spin], omega)
    nres = 0
    for m in range(e.size):
        if f[m] == 0.0:
            continue
        nres += 1
        wc, dwc = residue_value(eps, n_occ, B_ov, b_row[m], e[m] - omega)
        sig += f[m] * wc
        dsig += -f[m] * dwc
    return sig, dsig, nres


def solve(eps, n_occ, B_ov, row_ids, B_rows, states, xi, z, dsig_x=None, tol=1e-10,
          max_iter=100):
    """G0W0 QP energies of open-shell states (spin-orbital indices), each
    solved with the step tree of oracle/qp.py from its own level.  dsig_x:
    optional [2 * n_mo] (Sigma^x - V^xc per spin-orbital)."""
    from . import qp
    n_mo = np.asarray(eps).shape[1]
    row_ids = [int(r) for r in row_ids]
    wtab = w_table(eps, n_occ, B_ov, B_rows, xi)
    out = []
    for p in states:
        p = int(p)
        s, n = divmod(p, n_mo)
        r = row_ids.index(p)
        dx = 0.0 if dsig_x is None else float(dsig_x[p])
        e_n = float(eps[s][n])

        def fe(w, r=r, s=s, e_n=e_n, dx=dx):
            sg, ds, _ = sigma_c(eps, n_occ, B_ov, s, B_rows[r], wtab[r], xi, z, w)
            return e_n + dx + sg - w, ds - 1.0

        res = qp.step_tree(fe, e_n, tol=tol, max_iter=max_iter)
        res.update(state=p, sigma_c=res["f"] - (e_n + dx - res["E"]))
        out.append(res)
    return out
