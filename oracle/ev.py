"""Eigenvalue self-consistent GW (oracle; test infrastructure only).

Paper: Algorithm 1, the outer loop over iter = 0..maxeviter: once the QP
equations of the requested states are solved, their QP energies replace the
eigenvalues and the next cycle recomputes the transition energies and W;
the Introduction distinguishes updating the eigenvalues in G only (evGW0)
from updating them in G and W (evGW).

Readings:
  * only the requested states' eigenvalues are replaced, all at the end of a
    cycle; the other states keep their reference values (the paper states no
    shift for them);
  * the QP equation keeps the mean-field eigenvalue as its constant term
    (eps^QP = eps + Re Sigma(eps^QP) - V^xc); the updated energies enter the
    poles of G (the residue set, the residue frequencies eps_m - omega and the
    quadrature's a = omega - eps_m) and, for evGW, the transition energies of
    Pi (so W^c is rebuilt every cycle);
  * each cycle's QP solve starts from the state's current energy in G;
  * from the second cycle on a state's root lies close to its own moved G
    pole, where the plain quadrature of the I term cannot follow the
    integrand a/(a^2 + xi^2); the static part W^c(0) of that integrand is
    therefore integrated exactly in every cycle (cd.sigma_c with w0_row),
    which changes nothing in the limit of an exact quadrature;
  * cycles stop after n_cycles, or earlier once max |E - E_previous cycle| <
    ev_tol (ev_tol = 0: always n_cycles).
"""
import numpy as np

from . import cd, cluster, qp


def evgw(eps, n_occ, B_ov, row_ids, B_rows, states, xi, z, mode="evgw0", n_cycles=3,
         ev_tol=0.0, dsig_x=None, tol=1e-10, max_iter=100, cluster_width=0.0):
    """QP energies of `states` after eigenvalue self-consistency.

    mode: "evgw0" (G only) or "evgw" (G and W).  cluster_width > 0 applies the
    cluster initial-guess layer (oracle/cluster.py) in every cycle, with the
    clusters formed from the current energies in G.  Returns (results of the
    last cycle as qp.solve returns them, number of cycles run, energies per
    cycle)."""
    if mode not in ("evgw0", "evgw"):
        raise ValueError(mode)
    eps_ref = np.array(eps, dtype=np.float64)
    eps_g = eps_ref.copy()
    row_ids = [int(r) for r in row_ids]
    wtab = cd.w_table(eps_ref, n_occ, B_ov, B_rows, xi)
    w0 = cd.w_table(eps_ref, n_occ, B_ov, B_rows, np.zeros(1))[:, :, 0]
    history = []
    res = []
    cycles = 0
    for cyc in range(n_cycles):
        eps_w = eps_ref if mode == "evgw0" else eps_g.copy()
        if mode == "evgw" and cyc > 0:
            wtab = cd.w_table(eps_w, n_occ, B_ov, B_rows, xi)
            w0 = cd.w_table(eps_w, n_occ, B_ov, B_rows, np.zeros(1))[:, :, 0]
        fevals, dxs = [], []
        for n in states:
            r = row_ids.index(int(n))
            dx = 0.0 if dsig_x is None else float(dsig_x[n])
            fevals.append(qp.make_feval(eps_g, n_occ, B_ov, B_rows[r], wtab[r], xi, z, int(n),
                                        dx, eps_ref_n=eps_ref[n], eps_w=eps_w, w0_row=w0[r]))
            dxs.append(dx)
        # width 0: every state is its own cluster and starts at its energy in G
        res = cluster.solve_states(fevals, [float(eps_g[int(n)]) for n in states],
                                   cluster_width, tol=tol, max_iter=max_iter)
        for k, n in enumerate(states):
            res[k].update(state=int(n),
                          sigma_c=res[k]["f"] - (eps_ref[n] + dxs[k] - res[k]["E"]))
        E = np.array([o["E"] for o in res])
        cycles = cyc + 1
        converged = bool(history) and float(np.max(np.abs(E - history[-1]))) < ev_tol
        history.append(E)
        for k, n in enumerate(states):
            eps_g[n] = E[k]
        if converged:
            break
    return res, cycles, history
