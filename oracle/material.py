"""Point constitutive laws P = P(F, alpha) and their tangents (oracle).

Sec. 2.1, Eq. 2 (a point law with internal variables), Eq. 13 (the tangent
K = dP/dF used by Newton) and Sec. 3.2, Eq. 22 (the power-law flow rule with
a back stress).  The paper cites the full cyclic law of its grains without
writing it out; the workloads use the flow rule of Eq. 22 with a constant
critical resolved shear stress g and an Armstrong-Frederick back stress.
Its discrete form is a reading fixed here:

Crystal plasticity (law 0), one time step dt from committed (Fp^-1_0, chi_0):
    A       = I - sum_a dgam_a S0_a
    Fp^-1   = Fp^-1_0 A                      (backward Euler on Fp)
    Fe      = F Fp^-1,   Ee = (Fe^T Fe - I)/2,   S = C : Ee
    tau_a   = S : S0_a
    chi_a   = (chi_0a + c dgam_a) / (1 + d |dgam_a|)
    R_a     = dgam_a - dt gdot0 |(tau_a - chi_a)/g|^n sign(tau_a - chi_a) = 0
    P       = Fe S Fp^-T
The 12 slip increments solve R = 0 by a damped Newton iteration.  The tangent
is consistent with the converged local solution:
    K = dP/dF|_dgam - (dP/ddgam) J^-1 (dR/dF),   J = dR/ddgam.

Isotropic St-Venant-Kirchhoff (law 1, the stiff particles of Sec. 4.4):
    E = (F^T F - I)/2,  S = lam tr(E) I + 2 mu E,  P = F S,
    K_ijkl = d_ik S_lj + F_ia C_ajld F_kd.

Pins: central finite differences of P(F) for the tangent; the elastic limit;
objectivity and cubic symmetry; the single-crystal uniaxial case against an
independent scalar backward-Euler solve.  Status: pinned.
"""

from __future__ import annotations

import numpy as np

# parameter block indices (same order as the C ABI constant block)
C11, C12, C44, GDOT0, GCRSS, NEXP, CAF, DAF, EPART, NUPART = range(10)

LOCAL_MAXIT = 60
LOCAL_RTOL = 1e-10
LOCAL_ATOL = 1e-18
LOCAL_RFLOOR = 1e-10

_I3 = np.eye(3)


def _sym(A):
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def _cp_eval(F, Fpi0, chi0, dg, S0, C, p, dt):
    """Residual and intermediates of the return mapping at given slips."""
    A = _I3 - np.einsum("ma,maij->mij", dg, S0)
    Fpi = Fpi0 @ A
    Fe = F @ Fpi
    Ee = 0.5 * (np.swapaxes(Fe, 1, 2) @ Fe - _I3)
    S = np.einsum("mijkl,mkl->mij", C, Ee)
    tau = np.einsum("mij,maij->ma", S, S0)
    den = 1.0 + p[DAF] * np.abs(dg)
    chi = (chi0 + p[CAF] * dg) / den
    x = (tau - chi) / p[GCRSS]
    ax = np.abs(x)
    rate = dt * p[GDOT0] * ax ** p[NEXP] * np.sign(x)
    R = dg - rate
    return dict(A=A, Fpi=Fpi, Fe=Fe, S=S, tau=tau, chi=chi, x=x, den=den, R=R)


def _cp_jacobian(F, Fpi0, dg, S0, C, p, dt, ev):
    """J = dR/ddgam (M, 12, 12) and the factor D = dt gdot0 n |x|^(n-1)/g."""
    Fe = ev["Fe"]
    Q = np.swapaxes(Fe, 1, 2) @ F @ Fpi0                     # Fe^T F Fp^-1_0
    V = _sym(np.einsum("mij,mbjk->mbik", Q, S0))             # sym(Q S0_b)
    CS0 = np.einsum("mijkl,makl->maij", C, S0)               # C : S0_a
    dtau = -np.einsum("maij,mbij->mab", CS0, V)              # dtau_a/ddg_b
    dchi = (p[CAF] - p[DAF] * np.sign(dg) * ev["chi"]) / ev["den"]
    D = dt * p[GDOT0] * p[NEXP] * np.abs(ev["x"]) ** (p[NEXP] - 1) / p[GCRSS]
    J = np.broadcast_to(np.eye(12), dtau.shape).copy()
    J -= D[:, :, None] * dtau
    J[:, np.arange(12), np.arange(12)] += D * dchi
    return J, D, CS0


def _asinh_pow(x, n):
    """asinh(|x|^n sign x) and its derivative in x, safe for large |x|.

    For y = |x|^n > 1, asinh(y) = n ln|x| + ln(1 + sqrt(1 + y^-2)), which
    never forms an overflowing power.
    """
    ax = np.abs(x)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        lnx = np.log(ax)
        big = lnx * n > 0.0
        y = np.where(big, 1.0, ax ** n)
        yinv = np.where(big, np.exp(-n * lnx), 1.0)
        val_big = n * lnx + np.log1p(np.sqrt(1.0 + yinv * yinv))
        val_small = np.arcsinh(y)
        val = np.sign(x) * np.where(big, val_big, val_small)
        d_big = (n / np.where(big, ax, 1.0)) / np.sqrt(1.0 + yinv * yinv)
        d_small = n * ax ** (n - 1) / np.sqrt(1.0 + y * y)
        der = np.where(big, d_big, d_small)
    return val, der


def _local_system(F, Fpi0, chi0, dg, S0, C, p, dt):
    """Residual and Jacobian of the local problem in asinh form.

    R_a = asinh(dgam_a / a) - asinh(|x_a|^n sign x_a),  a = dt gdot0,
    x_a = (tau_a - chi_a)/g.  asinh is odd and strictly increasing, so R = 0
    has exactly the roots of the rate form dgam_a = a |x_a|^n sign x_a.  The
    residual is linear in the slip for |dgam| << a and logarithmic beyond,
    which keeps Newton's linear model accurate under large overstress, where
    the rate form would shrink the overstress by only (1 - 1/n) per step.
    """
    ev = _cp_eval(F, Fpi0, chi0, dg, S0, C, p, dt)
    a = dt * p[GDOT0]
    n = p[NEXP]
    Fe = ev["Fe"]
    Q = np.swapaxes(Fe, 1, 2) @ F @ Fpi0
    V = _sym(np.einsum("mij,mbjk->mbik", Q, S0))
    CS0 = np.einsum("mijkl,makl->maij", C, S0)
    dx = -np.einsum("maij,mbij->mab", CS0, V)                  # dtau/ddg
    dchi = (p[CAF] - p[DAF] * np.sign(dg) * ev["chi"]) / ev["den"]
    dx[:, np.arange(12), np.arange(12)] -= dchi
    dx /= p[GCRSS]                                              # dx/ddg
    rhs, drhs = _asinh_pow(ev["x"], n)
    R = np.arcsinh(dg / a) - rhs
    J = -drhs[:, :, None] * dx
    J[:, np.arange(12), np.arange(12)] += 1.0 / np.sqrt(a * a + dg * dg)
    return ev, R, J


def cp_update(F, Fpi0, chi0, dg0, S0, C, params, dt, tangent=True):
    """Crystal-plasticity return mapping for M voxels.

    The local iteration starts from ``dg0``; voxels where that attempt fails
    are solved again from zero slips (same root, different start).
    """
    out = _cp_update_from(F, Fpi0, chi0, dg0, S0, C, params, dt, tangent)
    bad = np.nonzero(~out["ok"])[0]
    if bad.size and np.any(np.asarray(dg0)[bad] != 0.0):
        again = _cp_update_from(F[bad], Fpi0[bad], chi0[bad],
                                np.zeros((bad.size, 12)), S0[bad], C[bad],
                                params, dt, tangent)
        for k, v in again.items():
            if k == "iters":
                out[k][bad] += v
            else:
                out[k][bad] = v
    return out


def _cp_update_from(F, Fpi0, chi0, dg0, S0, C, params, dt, tangent=True):
    """One attempt of the return mapping from the starting slips ``dg0``.

    F, Fpi0: (M,3,3); chi0, dg0: (M,12) (dg0 = starting guess of the local
    Newton iteration); S0: (M,12,3,3); C: (M,3,3,3,3).
    Returns dict with P (M,3,3), K (M,3,3,3,3) if ``tangent``, trial state
    Fpi (M,3,3), chi (M,12), dg (M,12), tau (M,12), iterations and ok flags.
    """
    p = np.asarray(params, dtype=np.float64)
    M = F.shape[0]
    dg = np.array(dg0, dtype=np.float64, copy=True)
    active = np.ones(M, dtype=bool)
    iters = np.zeros(M, dtype=np.int64)
    ok = np.zeros(M, dtype=bool)
    for it in range(LOCAL_MAXIT):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        sl = (F[idx], Fpi0[idx], chi0[idx])
        _, R, J = _local_system(*sl, dg[idx], S0[idx], C[idx], p, dt)
        step = -np.linalg.solve(J, R[:, :, None])[:, :, 0]
        iters[idx] += 1
        small = np.all(np.isfinite(step), axis=1) & (
            np.max(np.abs(step), axis=1) <= LOCAL_ATOL + LOCAL_RTOL *
            np.max(np.abs(dg[idx] + step), axis=1))
        # backtracking on the merit 0.5 |R|^2 (Armijo with c = 1e-4)
        merit = 0.5 * np.sum(R * R, axis=1)
        lam = np.ones(idx.size)
        pending = ~small
        new = dg[idx] + step
        for _ in range(40):
            if not pending.any():
                break
            sub = np.nonzero(pending)[0]
            trial = dg[idx[sub]] + lam[sub, None] * step[sub]
            _, Rt, _ = _local_system(F[idx[sub]], Fpi0[idx[sub]],
                                     chi0[idx[sub]], trial, S0[idx[sub]],
                                     C[idx[sub]], p, dt)
            mt = 0.5 * np.sum(Rt * Rt, axis=1)
            good = np.isfinite(mt) & (mt <= (1.0 - 1e-4 * lam[sub]) *
                                      merit[sub])
            new[sub] = trial          # last tried step stands if none descends
            pending[sub[good]] = False
            lam[sub[~good]] *= 0.5
        dg[idx] = new
        # at the rounding floor no step descends; a tiny residual there is
        # as converged as the iteration can get
        floor = pending & (np.max(np.abs(R), axis=1) <= LOCAL_RFLOOR)
        done = (small | floor) & np.all(np.isfinite(dg[idx]), axis=1)
        ok[idx[done]] = True
        active[idx[done]] = False
        bad = ~np.all(np.isfinite(dg[idx]), axis=1)
        active[idx[bad]] = False
    ev = _cp_eval(F, Fpi0, chi0, dg, S0, C, p, dt)
    Fe, Fpi, S = ev["Fe"], ev["Fpi"], ev["S"]
    P = Fe @ S @ np.swapaxes(Fpi, 1, 2)
    out = dict(P=P, Fpi=Fpi, chi=ev["chi"], dg=dg, tau=ev["tau"],
               iters=iters, ok=ok & np.all(np.isfinite(P), axis=(1, 2)))
    if tangent:
        out["K"] = _cp_tangent(F, Fpi0, dg, S0, C, p, dt, ev)
    return out


def _cp_tangent(F, Fpi0, dg, S0, C, p, dt, ev):
    """Consistent tangent dP/dF at the converged slips (M,3,3,3,3)."""
    Fe, Fpi, S = ev["Fe"], ev["Fpi"], ev["S"]
    J, D, CS0 = _cp_jacobian(F, Fpi0, dg, S0, C, p, dt, ev)
    # dR_a/dF_kl = -D_a (Fe (C:S0_a) Fp^-T)_kl
    dtau_dF = np.einsum("mkb,mabc,mlc->makl", Fe, CS0, Fpi)
    dR_dF = -D[:, :, None, None] * dtau_dF
    # explicit part at fixed slips
    B = Fpi @ S @ np.swapaxes(Fpi, 1, 2)                        # Fp^-1 S Fp^-T
    K = np.einsum("ik,mlj->mijkl", _I3, B)
    K += np.einsum("mib,mjc,mbcde,mkd,mle->mijkl", Fe, Fpi, C, Fe, Fpi,
                   optimize=True)
    # slip part: dP/ddg_b
    Gb = -np.einsum("mij,mjk,mbkl->mbil", F, Fpi0, S0)          # dFe/ddg_b
    dFpi = -np.einsum("mij,mbjk->mbik", Fpi0, S0)               # dFp^-1/ddg_b
    dE = _sym(np.einsum("mji,mbjk->mbik", Fe, Gb))
    dS = np.einsum("mijkl,mbkl->mbij", C, dE)
    FpiT = np.swapaxes(Fpi, 1, 2)
    dP = (np.einsum("mbij,mjk,mkl->mbil", Gb, S, FpiT)
          + np.einsum("mij,mbjk,mkl->mbil", Fe, dS, FpiT)
          + np.einsum("mij,mjk,mblk->mbil", Fe, S, dFpi))
    M = F.shape[0]
    ddg_dF = -np.linalg.solve(J, dR_dF.reshape(M, 12, 9)).reshape(M, 12, 3, 3)
    K += np.einsum("mbij,mbkl->mijkl", dP, ddg_dF)
    return K


def svk_update(F, lam, mu, tangent=True):
    """Isotropic St-Venant-Kirchhoff: P = F S, S = lam tr(E) I + 2 mu E."""
    E = 0.5 * (np.swapaxes(F, 1, 2) @ F - _I3)
    trE = np.trace(E, axis1=1, axis2=2)
    S = lam * trE[:, None, None] * _I3 + 2 * mu * E
    P = F @ S
    out = dict(P=P, S=S)
    if tangent:
        d = _I3
        Ciso = (lam * np.einsum("ab,cd->abcd", d, d)
                + mu * (np.einsum("ac,bd->abcd", d, d)
                        + np.einsum("ad,bc->abcd", d, d)))
        K = np.einsum("ik,mlj->mijkl", d, S)
        K += np.einsum("mia,ajld,mkd->mijkl", F, Ciso, F, optimize=True)
        out["K"] = K
    return out
