"""Quasiparticle equation solvers (oracle; test infrastructure only).

Paper: "Implementation - Solution of the Quasiparticle Equations": the QP
equation eps_QP = eps + Re Sigma(eps_QP) - V^xc, the residual
f(xi) = eps + Re Sigma(xi) - V^xc - xi, Z = -(df/dxi)^-1, the step-selection
tree figure, the scaled-Newton factor 0.7 and the scaled-residual factor
(adaptive, at most 0.1), and the bracket definition (a sign change of f, or
the same sign with growing magnitude between consecutive steps).  The
graphical solver (scan on a fine real-frequency grid) is the paper's
alternative solver and serves as the brute-force pin.

Here f(w) = eps_n + dsig_x_n + Re Sigma^c_n(w) - w, where dsig_x_n stands
for Sigma^x_nn - V^xc_nn (0 unless given).

Readings:
  * scaled residual: dw = alpha f with alpha = min(0.1, 0.1/|f|), so the
    step never exceeds 0.1 Ha;
  * iteration 0 is always a scaled residual (no derivative is used there);
  * Newton: dw = Z f when Z >= 0.3; scaled Newton: dw = 0.7 Z f when
    0.1 <= Z < 0.3 and no bracket exists;
  * a bracket is a pair of evaluated points.  It is created from the
    previous and current point when f changes sign with f > 0 on the left
    end (a root between them), or when f keeps its sign, grows in magnitude,
    and the step went in the direction of the residual (a pole was crossed,
    so a root was skipped).  A point that lands strictly inside an existing
    bracket replaces one of its ends (see _shrink);
  * "golden section" on a bracket: with s the end of smaller |f| and e the
    other, the next point is s + 0.381966 (e - s);
  * convergence: |f| < qp_tol.  Between poles df/dw <= -1, so the root is
    then within qp_tol of w;
  * at the iteration cap the last evaluated point is returned, flagged.

Parity unpinned: when the scan finds several roots in the window (core levels
near a dense pole band), which one the step tree returns is fixed only by
this deterministic rule; tests record whether the returned root is the
unique one in its scan window.
"""
import math

import numpy as np

from . import cd

GOLD = (3.0 - math.sqrt(5.0)) / 2.0   # 0.381966...

STATUS_MAXITER = 1
STATUS_SMALL_Z = 2


def _alpha(f):
    return min(0.1, 0.1 / abs(f)) if f != 0.0 else 0.1


def _sgn(x):
    return int(x > 0) - int(x < 0)


def _shrink(br, x, fx):
    """Replace one end of bracket br = (s, fs, e, fe) by the inner point x."""
    s, fs, e, fe = br
    if _sgn(fs) != _sgn(fe):
        # sign-change bracket: keep the ends of opposite sign
        if _sgn(fx) == _sgn(fs):
            s, fs = x, fx
        else:
            e, fe = x, fx
    else:
        # same-sign bracket (skipped root): x lies on s's branch beyond s when
        # f keeps its sign and shrinks in magnitude; otherwise past the pole
        if _sgn(fx) == _sgn(fs) and abs(fx) < abs(fs):
            s, fs = x, fx
        else:
            e, fe = x, fx
    if abs(fe) < abs(fs):
        s, fs, e, fe = e, fe, s, fs
    return (s, fs, e, fe)


def _make_bracket(wp, fp, wc, fc):
    """Bracket from consecutive points, or None."""
    if fp * fc < 0:
        lo, flo, hi, fhi = (wp, fp, wc, fc) if wp < wc else (wc, fc, wp, fp)
        if flo > 0 > fhi:
            br = (lo, flo, hi, fhi)
        else:
            return None     # f rises through a pole: no root between them
    elif fp * fc > 0 and abs(fc) > abs(fp) and _sgn(wc - wp) == _sgn(fp):
        br = (wp, fp, wc, fc)
    else:
        return None
    s, fs, e, fe = br
    if abs(fe) < abs(fs):
        s, fs, e, fe = e, fe, s, fs
    return (s, fs, e, fe)


def step_tree(feval, w0, tol=1e-10, max_iter=100):
    """Solve f(w) = 0 from w0 with the paper's step-selection tree.

    feval(w) -> (f, dfdw).  Returns dict(E, f, dfdw, Z, status, iters, trace).
    """
    if max_iter < 1:
        raise ValueError("max_iter must be >= 1")
    w = float(w0)
    prev = None
    br = None
    trace = []
    for it in range(max_iter):
        f, fp = feval(w)
        Z = -1.0 / fp if fp != 0.0 else math.inf
        if prev is not None:
            wp, fpv = prev
            if br is not None and min(br[0], br[2]) < w < max(br[0], br[2]):
                br = _shrink(br, w, f)
            else:
                nb = _make_bracket(wp, fpv, w, f)
                if nb is not None:
                    br = nb
        if abs(f) < tol:
            trace.append((w, f, "done"))
            st = STATUS_SMALL_Z if Z < 0.1 else 0
            return dict(E=w, f=f, dfdw=fp, Z=Z, status=st, iters=it + 1, trace=trace)
        if it == 0:
            kind, wn = "residual", w + _alpha(f) * f
        elif Z >= 0.3:
            kind, wn = "newton", w + Z * f
        elif br is not None:
            s, _, e, _ = br
            kind, wn = "golden", s + GOLD * (e - s)
        elif Z >= 0.1:
            kind, wn = "scaled-newton", w + 0.7 * Z * f
        else:
            kind, wn = "residual", w + _alpha(f) * f
        trace.append((w, f, kind))
        prev = (w, f)
        w = wn
    # iteration cap: the last evaluated point is the answer (f, Z as evaluated
    # there); the step computed after it is not taken
    st = STATUS_MAXITER | (STATUS_SMALL_Z if Z < 0.1 else 0)
    return dict(E=prev[0], f=f, dfdw=fp, Z=Z, status=st, iters=max_iter, trace=trace)


def make_feval(eps, n_occ, B_ov, b_row, wtab_row, xi, z, n, dsig_x_n=0.0, counter=None,
               eps_ref_n=None, eps_w=None, w0_row=None):
    """f(w) and df/dw for state n from the contour-deformation Sigma^c.

    eps are the energies in G; eps_w those in W (None: eps); eps_ref_n the
    constant term of the QP equation (None: eps[n]); w0_row the static
    W^c_nm(0) for the split quadrature of cd.sigma_c (None: plain quadrature)."""
    eps_n = float(eps[n] if eps_ref_n is None else eps_ref_n)

    def feval(w):
        s, ds, nres = cd.sigma_c(eps, n_occ, B_ov, b_row, wtab_row, xi, z, w, eps_w=eps_w,
                                 w0_row=w0_row)
        if counter is not None:
            counter.append((w, s, ds, nres))
        return float(eps_n + dsig_x_n + s - w), float(ds - 1.0)

    return feval


def solve(eps, n_occ, B_ov, row_ids, B_rows, states, xi, z, dsig_x=None,
          tol=1e-10, max_iter=100):
    """G0W0 QP energies for `states` (each must be in row_ids).

    Returns a list of dicts with E, sigma_c (Re Sigma^c at E), Z, status,
    iters and the number of Sigma evaluations."""
    row_ids = list(int(r) for r in row_ids)
    wtab = cd.w_table(eps, n_occ, B_ov, B_rows, xi)
    out = []
    for n in states:
        r = row_ids.index(int(n))
        dx = 0.0 if dsig_x is None else float(dsig_x[n])
        calls = []
        fe = make_feval(eps, n_occ, B_ov, B_rows[r], wtab[r], xi, z, int(n), dx, calls)
        res = step_tree(fe, eps[n], tol=tol, max_iter=max_iter)
        sig = res["f"] - (eps[n] + dx - res["E"])
        res.update(state=int(n), sigma_c=sig, n_evals=len(calls),
                   n_residues=[c[3] for c in calls])
        out.append(res)
    return out


def scan(feval, center, half_width=1.0, step=1e-3, tol=1e-12):
    """Graphical solution: evaluate f on a uniform grid over
    [center - half_width, center + half_width] and refine every downward sign
    change (f > 0 then f < 0) by bisection.  Upward sign changes are pole
    crossings.  Returns (roots, pole_crossings)."""
    ws = center + np.arange(-half_width, half_width + 0.5 * step, step)
    fs = np.array([feval(w)[0] for w in ws])
    roots, poles = [], []
    for k in range(len(ws) - 1):
        if fs[k] > 0 > fs[k + 1]:
            lo, hi, flo = ws[k], ws[k + 1], fs[k]
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                fm = feval(mid)[0]
                if fm > 0:
                    lo, flo = mid, fm
                else:
                    hi = mid
                if hi - lo < tol:
                    break
            roots.append(0.5 * (lo + hi))
        elif fs[k] < 0 < fs[k + 1]:
            poles.append(0.5 * (ws[k] + ws[k + 1]))
    return roots, poles
