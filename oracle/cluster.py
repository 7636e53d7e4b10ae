"""Cluster initial-guess layer of the QP solver (oracle; test infrastructure
only).

Paper: "Implementation - Solution of the Quasiparticle Equations", the layer
described after the step-selection tree: in a molecule with many nuclei of
one kind the QP energies of the requested states gather in a few narrow
regions; once one state of a region is solved, its result gives the other
states of that region a good start for the iterative solver.

Readings:
  * clusters are formed from the requested states' energies in G (the
    mean-field eigenvalues for G0W0): sorted ascending, a new cluster starts
    wherever the gap to the previous state exceeds `width` (Ha); width <= 0
    disables the layer (every state is its own cluster);
  * the member of median energy (the lower median for an even count; among
    equal energies the one requested first) is the cluster's representative
    and is solved first, from its own energy;
  * every other member starts the step tree at eps_n + (E_rep - eps_rep), i.e.
    it takes over the representative's QP shift; a representative that hit
    the iteration cap passes no guess (its members start at eps_n);
  * the step tree itself is unchanged (its first step is still the scaled
    residual), so a member's result depends only on its start.
"""
import numpy as np

from . import cd, qp


def clusters(energies, width):
    """Clusters of positions into `energies` (lists in ascending energy order)."""
    e = np.asarray(energies, dtype=np.float64)
    order = sorted(range(len(e)), key=lambda k: (e[k], k))
    out = []
    for k in order:
        if out and width > 0 and e[k] - e[out[-1][-1]] <= width:
            out[-1].append(k)
        else:
            out.append([k])
    return out


def representative(cluster):
    """The member of median energy (clusters are in ascending order)."""
    return cluster[(len(cluster) - 1) // 2]


def solve_states(fevals, starts, width, tol=1e-10, max_iter=100):
    """Step-tree solves of several states with the cluster layer.

    fevals[k](w) -> (f, df/dw) of state k; starts[k]: its energy in G.
    Returns the step_tree results in input order, each also carrying its
    start frequency w0 and whether it was its cluster's representative."""
    out = [None] * len(starts)

    def run(k, w0):
        res = qp.step_tree(fevals[k], w0, tol=tol, max_iter=max_iter)
        res["w0"] = w0
        return res

    for cl in clusters(starts, width):
        rep = representative(cl)
        out[rep] = run(rep, float(starts[rep]))
        out[rep]["representative"] = True
        shift = (None if out[rep]["status"] & qp.STATUS_MAXITER
                 else out[rep]["E"] - float(starts[rep]))
        for k in cl:
            if k == rep:
                continue
            w0 = float(starts[k]) if shift is None else float(starts[k]) + shift
            out[k] = run(k, w0)
            out[k]["representative"] = False
    return out


def solve(eps, n_occ, B_ov, row_ids, B_rows, states, xi, z, width, dsig_x=None, tol=1e-10,
          max_iter=100):
    """G0W0 QP energies of `states` with the cluster initial-guess layer.

    Returns qp.solve's result list (in the order of `states`), each entry
    also carrying w0 and `representative` (see solve_states)."""
    row_ids = [int(r) for r in row_ids]
    eps = np.asarray(eps, dtype=np.float64)
    wtab = cd.w_table(eps, n_occ, B_ov, B_rows, xi)
    fevals, counters, dxs = [], [], []
    for n in states:
        r = row_ids.index(int(n))
        dx = 0.0 if dsig_x is None else float(dsig_x[int(n)])
        calls = []
        fevals.append(qp.make_feval(eps, n_occ, B_ov, B_rows[r], wtab[r], xi, z, int(n), dx,
                                    calls))
        counters.append(calls)
        dxs.append(dx)
    out = solve_states(fevals, [float(eps[int(n)]) for n in states], width, tol, max_iter)
    for k, n in enumerate(states):
        r = out[k]
        r.update(state=int(n), sigma_c=r["f"] - (eps[int(n)] + dxs[k] - r["E"]),
                 n_evals=len(counters[k]))
    return out
