"""Generate cf_nu14.inc: poles and residues of the degree-14
Caratheodory-Fejer (CF) approximant of e^x on (-inf, 0] (paper, Section 2),
as FP64 constants for the HIP library.

Build-time script of the library; run once, output committed.

Poles: the CF construction.  x = 9 (s-1)/(s+1) maps s in [-1, 1] onto
(-inf, 0]; the full Chebyshev coefficients a_k of f(s) = e^{x(s)} are taken
by Gauss-Chebyshev quadrature; the Hankel matrix [a_{1+i+j}] is symmetric and
its eigenvector for the 15th largest |eigenvalue| defines a polynomial whose
14 roots outside the unit disk, mapped by s = (z + 1/z)/2 and then to x, are
the poles.

Residues: with the poles fixed, r(x) = w0 + Re sum_j c_j/(x - tau_j) is
linear in (w0, c_j); the coefficients are the minimax ones on (-inf, 0],
found by a linear Remez exchange in 34-digit arithmetic.  The CF poles are
optimal to O(56^-14), so the minimax error equals the CF error level.
"""
import os

import mpmath as mp
import numpy as np

mp.mp.dps = 34
NU = 14
SC = mp.mpf(9)
KH = 80          # Hankel order
NQ = 640         # Gauss-Chebyshev nodes


def f_of_s(s):
    if s + 1 < mp.mpf(10) ** -30:
        return mp.mpf(0)
    return mp.exp(SC * (s - 1) / (s + 1))


def chebyshev_coefficients(nmax):
    nodes = [(j + mp.mpf(1) / 2) * mp.pi / NQ for j in range(NQ)]
    fv = [f_of_s(mp.cos(t)) for t in nodes]
    return [2 * mp.fsum(fv[j] * mp.cos(k * nodes[j]) for j in range(NQ)) / NQ
            for k in range(nmax + 1)]


def hankel_eigvec(a):
    Hf = np.array([[float(a[1 + i + j]) for j in range(KH)] for i in range(KH)])
    w, V = np.linalg.eigh(Hf)
    pick = np.argsort(-np.abs(w))[NU]
    H = mp.matrix(KH, KH)
    for i in range(KH):
        for j in range(KH):
            H[i, j] = a[1 + i + j]
    vec = mp.matrix([mp.mpf(x) for x in V[:, pick]])
    mu = mp.mpf(w[pick])
    for _ in range(4):                      # Rayleigh-quotient refinement
        sol = mp.lu_solve(H - mu * mp.eye(KH), vec)
        vec = sol / mp.norm(sol)
        mu = (vec.T * H * vec)[0]
    return [vec[i] for i in range(KH)], mu


def outer_roots(coef):
    """Roots of sum_j coef[j] z^(K-1-j) outside the unit disk, Newton-polished."""
    r0 = np.roots(np.array([float(x) for x in coef]))
    out = []
    for z0 in r0[np.abs(r0) > 1]:
        z = mp.mpc(z0.real, z0.imag)
        for _ in range(12):
            p = mp.mpc(0)
            dp = mp.mpc(0)
            for cc in coef:
                dp = dp * z + p
                p = p * z + cc
            z -= p / dp
        out.append(z)
    assert len(out) == NU, len(out)
    return out


def remez_residues(taus):
    """Linear minimax fit of (w0, c_j) with the poles fixed."""
    def basis(x):
        row = [mp.mpf(1)]
        for t in taus:
            q = 1 / (x - t)
            row += [q.real, -q.imag]
        return row

    ngrid = 6000
    svals = [mp.cos(mp.pi * (ngrid - i) / ngrid) for i in range(ngrid + 1)]
    xs = [mp.mpf("-1e40") if s + 1 < mp.mpf(10) ** -30 else SC * (s - 1) / (s + 1)
          for s in svals]
    fx = [mp.exp(x) for x in xs]
    rows = [basis(x) for x in xs]
    nb = 1 + 2 * len(taus)
    # start: nb+1 points equispaced in s.  Each step solves
    #   f(x_i) - r(x_i) = (-1)^i E
    # on the current alternating reference; once the error curve shows more
    # than nb+1 alternating extrema (the CF poles are near-optimal, so close
    # to 2*14+2 of them appear) every extremum is kept in the reference and
    # the system is solved in the least-squares sense.
    ref = [int(round(i * ngrid / nb)) for i in range(nb + 1)]
    best = None
    for it in range(30):
        A = mp.matrix(len(ref), nb + 1)
        rhs = mp.matrix(len(ref), 1)
        for r, gi in enumerate(ref):
            for k in range(nb):
                A[r, k] = rows[gi][k]
            A[r, nb] = (-1) ** r
            rhs[r] = fx[gi]
        if len(ref) == nb + 1:
            sol = mp.lu_solve(A, rhs)
        else:
            sol = mp.qr_solve(A, rhs)[0]
        coef = [sol[k] for k in range(nb)]
        err = [fx[i] - mp.fsum(rows[i][k] * coef[k] for k in range(nb)) for i in range(len(xs))]
        ext = []
        for i in range(len(err)):
            e = err[i]
            if e == 0:
                continue
            if ext and mp.sign(err[ext[-1]]) == mp.sign(e):
                if abs(e) > abs(err[ext[-1]]):
                    ext[-1] = i
            else:
                ext.append(i)
        emax = max(abs(e) for e in err)
        if best is None or emax < best[1]:
            best = (coef, emax)
        if len(ext) >= nb + 1:
            ref = ext
        else:
            gmax = max(range(len(err)), key=lambda i: abs(err[i]))
            ref = sorted(set(ref[1:] + [gmax]))[:nb + 1]
        spread = max(abs(err[i]) for i in ext) / min(abs(err[i]) for i in ext)
        if spread < 1 + mp.mpf("1e-4"):
            break
    coef, emax = best
    return coef, emax


def main():
    a = chebyshev_coefficients(2 * KH + 2)
    vec, mu = hankel_eigvec(a)
    zeta = outer_roots(vec)
    taus_all = [SC * (z - 1) ** 2 / (z + 1) ** 2 for z in zeta]
    up = sorted([t for t in taus_all if t.imag > 0], key=lambda t: t.real)
    coef, emax = remez_residues(up)
    w0 = coef[0]
    cs = [mp.mpc(coef[1 + 2 * j], coef[2 + 2 * j]) for j in range(len(up))]
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "cf_nu14.inc"), "w") as fh:
        fh.write("// Generated by gen_cf_table.py: degree-14 CF approximant of e^x on (-inf,0].\n")
        fh.write("// r(x) = CF_OMEGA0 + Re sum_j CF_C[j] / (x - CF_TAU[j]),  Im CF_TAU[j] > 0.\n")
        fh.write(f"// max |r(x) - e^x| on (-inf,0] (34-digit evaluation): {mp.nstr(emax, 6)}\n")
        fh.write("#define CF_NPOLE 7\n")
        fh.write(f"static const double CF_OMEGA0 = {mp.nstr(w0, 20)};\n")
        fh.write("static const double CF_TAU_RE[CF_NPOLE] = {" + ", ".join(mp.nstr(t.real, 20) for t in up) + "};\n")
        fh.write("static const double CF_TAU_IM[CF_NPOLE] = {" + ", ".join(mp.nstr(t.imag, 20) for t in up) + "};\n")
        fh.write("static const double CF_C_RE[CF_NPOLE] = {" + ", ".join(mp.nstr(x.real, 20) for x in cs) + "};\n")
        fh.write("static const double CF_C_IM[CF_NPOLE] = {" + ", ".join(mp.nstr(x.imag, 20) for x in cs) + "};\n")
    print("max error", mp.nstr(emax, 8))


if __name__ == "__main__":
    main()
