"""Newton-CG load increments on a periodic RVE (oracle).

Follows Sec. 2.1 of Lucarini & Segurado:

* Eq. 1: F = Fbar + Ftilde with <F> = Fbar, Ftilde periodic.
* Eqs. 9-11: discrete equilibrium G(P(F)) = 0 on every voxel.
* Eqs. 12-16: Newton iterations F^i = F^{i-1} + dF, where dF solves the
  linear system G(K : dF) = -G(P) with the operator G_K.
* The linear system is solved with conjugate gradients (text after Eq. 16):
  it is rank deficient (null and Nyquist frequencies) and CG never needs the
  matrix.
* Internal variables are updated only after the increment has converged
  (end of Sec. 2.1).
* Sec. 3.3, Eqs. 23-24: fatigue indicator fields accumulated per cycle.
* Sec. 3.1: the macroscopic stress is the volume average of the microscopic
  stress.

Readings (listed in the design notes): the predictor is the converged field
of the previous increment plus the macroscopic increment; equilibrium is
reached when ||G(P)||_2 <= tol ||P||_2 over all 9N entries; CG starts from
zero and stops when ||r|| <= eta ||b|| or when p.Ap <= 0; the accumulated
plastic slip uses sqrt(2/3 dLp:dLp) per increment (the printed integrand
has units of 1/s) and the literal sum dLp:dLp/dt is kept beside it;
sigma_bar = P_bar Fbar^T / det Fbar.

Pins: homogeneous medium (one evaluation, zero CG iterations), laminate
closed form, dense brute-force Newton on tiny grids, directional finite
differences of the Newton Jacobian, Hill-Mandel, single-crystal FIPs.
Status: pinned.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import crystal, material, umat
from .projection import apply_G

OK, EINVAL, ENOTCONV, ELOCAL = 0, -1, -4, -5
CHUNK = 16384


@dataclass
class IncrementInfo:
    status: int = OK
    newton_iters: int = 0
    cg_iters: list = field(default_factory=list)
    residuals: list = field(default_factory=list)
    local_failures: int = 0
    P_bar: np.ndarray = None
    sigma_bar: np.ndarray = None

    @property
    def cg_iters_total(self) -> int:
        return int(sum(self.cg_iters))


def cg(apply_A, b, eta, maxit):
    """Conjugate gradients from x0 = 0; returns (x, iterations, breakdown)."""
    x = np.zeros_like(b)
    r = b.copy()
    rr = float(np.vdot(r, r))
    bnorm = np.sqrt(rr)
    if bnorm == 0.0:
        return x, 0, False
    p = r.copy()
    it = 0
    breakdown = False
    while it < maxit:
        Ap = apply_A(p)
        it += 1
        pAp = float(np.vdot(p, Ap))
        if not pAp > 0.0:
            breakdown = True
            break
        alpha = rr / pAp
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.vdot(r, r))
        if np.sqrt(rr_new) <= eta * bnorm:
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return x, it, breakdown


class OracleRVE:
    """Periodic RVE state and the increment algorithm, all in FP64 on CPU.

    Fields are stored voxel-major: F has shape (N, 3, 3) with the voxel index
    flattened as (a*n2 + b)*n3 + c.
    """

    def __init__(self, shape, phase, quat, law, params, operator="continuous",
                 L=(1.0, 1.0, 1.0)):
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.phase = np.asarray(phase, dtype=np.int64).reshape(-1)
        assert self.phase.size == self.N
        self.quat = np.asarray(quat, dtype=np.float64)
        self.law = np.asarray(law, dtype=np.int64)
        self.params = np.asarray(params, dtype=np.float64)
        self.operator = operator
        self.L = tuple(float(x) for x in L)
        S0g, Cg = crystal.grain_tables(self.quat, self.params)
        self.S0g, self.Cg = S0g, Cg
        self.lam, self.mu = crystal.lame_from_young(self.params[8],
                                                    self.params[9])
        vlaw = self.law[self.phase]
        self.cp_idx = np.nonzero(vlaw == 0)[0]
        self.el_idx = np.nonzero(vlaw == 1)[0]
        self.reset()

    # ----------------------------------------------------------------- state
    def reset(self):
        N = self.N
        self.F = np.broadcast_to(np.eye(3), (N, 3, 3)).copy()
        self.F_bar = np.eye(3)
        self.Fpi = np.broadcast_to(np.eye(3), (N, 3, 3)).copy()
        self.chi = np.zeros((N, 12))
        self.dg = np.zeros((N, 12))
        self.P = np.zeros((N, 3, 3))
        self.pcyc = np.zeros(N)
        self.pcyc_lit = np.zeros(N)
        self.wcyc = np.zeros((N, 12))
        self.t = 0.0
        self.increments = 0

    def reset_fips(self):
        """Start a new cycle: zero the per-cycle indicator accumulators."""
        self.pcyc[:] = 0.0
        self.pcyc_lit[:] = 0.0
        self.wcyc[:] = 0.0

    # ----------------------------------------------------------- field maps
    def to_field(self, A):
        """(N,3,3) -> (3,3,n1,n2,n3)."""
        return np.ascontiguousarray(np.moveaxis(A, 0, -1)).reshape(
            (3, 3) + self.shape)

    def from_field(self, B):
        return np.ascontiguousarray(np.moveaxis(B.reshape(3, 3, self.N), -1, 0))

    def G(self, A):
        """Eq. 11 on a voxel-major field."""
        return self.from_field(apply_G(self.to_field(A), self.L, self.operator))

    # -------------------------------------------------------- constitutive
    def constitutive(self, F, dt, dg_start):
        """P, K and trial state for every voxel at committed internal state."""
        N = self.N
        P = np.zeros((N, 3, 3))
        K = np.zeros((N, 3, 3, 3, 3))
        trial = dict(Fpi=self.Fpi.copy(), chi=self.chi.copy(),
                     dg=np.zeros((N, 12)), tau=np.zeros((N, 12)))
        fails = 0
        for s in range(0, self.cp_idx.size, CHUNK):
            idx = self.cp_idx[s:s + CHUNK]
            g = self.phase[idx]
            out = material.cp_update(F[idx], self.Fpi[idx], self.chi[idx],
                                     dg_start[idx], self.S0g[g], self.Cg[g],
                                     self.params, dt)
            P[idx] = out["P"]
            K[idx] = out["K"]
            trial["Fpi"][idx] = out["Fpi"]
            trial["chi"][idx] = out["chi"]
            trial["dg"][idx] = out["dg"]
            trial["tau"][idx] = out["tau"]
            fails += int(np.count_nonzero(~out["ok"]))
        if self.el_idx.size:
            out = material.svk_update(F[self.el_idx], self.lam, self.mu)
            P[self.el_idx] = out["P"]
            K[self.el_idx] = out["K"]
        return P, K, trial, fails

    # ------------------------------------------------------------ increment
    def increment(self, F_bar_new, dt, tol=1e-6, eta=1e-4, newton_max=25,
                  cg_max=2000, dF_start=None):
        """Solve one load increment; commit only on success.

        ``dF_start`` optionally adds a warm-start fluctuation to the
        homogeneous predictor; it is projected by G first so that it is
        compatible and has zero mean.
        """
        F_bar_new = np.asarray(F_bar_new, dtype=np.float64).reshape(3, 3)
        info = IncrementInfo()
        F = self.F + (F_bar_new - self.F_bar)[None]
        if dF_start is not None:
            F = F + self.G(np.asarray(dF_start, dtype=np.float64))
        dg_start = np.zeros((self.N, 12))
        for it in range(newton_max + 1):
            P, K, trial, fails = self.constitutive(F, dt, dg_start)
            if fails:
                info.status = ELOCAL
                info.local_failures = fails
                return info
            r = self.G(P)
            rn = float(np.sqrt(np.vdot(r, r)))
            Pn = float(np.sqrt(np.vdot(P, P)))
            rel = rn / Pn if Pn > 0 else 0.0
            info.residuals.append(rel)
            if rn <= tol * Pn:
                self._commit(F, F_bar_new, P, trial, dt)
                info.newton_iters = it
                info.P_bar = P.mean(axis=0)
                info.sigma_bar = info.P_bar @ F_bar_new.T / np.linalg.det(
                    F_bar_new)
                return info
            if it == newton_max:
                break
            Kv = K.reshape(self.N, 9, 9)

            def apply_A(x, Kv=Kv):
                y = np.einsum("vab,vb->va", Kv, x.reshape(self.N, 9))
                return self.G(y.reshape(self.N, 3, 3))

            x, ncg, _ = cg(apply_A, -r, eta, cg_max)
            info.cg_iters.append(ncg)
            F = F + x
            dg_start = trial["dg"]
        info.status = ENOTCONV
        info.newton_iters = newton_max
        return info

    def _commit(self, F, F_bar_new, P, trial, dt):
        """End of Sec. 2.1: accept the increment; Eqs. 23-24 accumulate."""
        g = self.phase
        dLp = np.einsum("va,vaij->vij", trial["dg"], self.S0g[g])
        dd = np.einsum("vij,vij->v", dLp, dLp)
        cp = self.law[g] == 0
        self.pcyc += np.where(cp, np.sqrt(2.0 / 3.0 * dd), 0.0)
        self.pcyc_lit += np.where(cp, dd / dt, 0.0)
        self.wcyc += np.where(cp[:, None], trial["tau"] * trial["dg"], 0.0)
        self.F = F
        self.F_bar = F_bar_new.copy()
        self.Fpi = trial["Fpi"]
        self.chi = trial["chi"]
        self.dg = trial["dg"]
        self.P = P
        self.t += dt
        self.increments += 1

    # ------------------------------------------------- time incrementation
    def increment_adaptive(self, F_bar_new, dt, max_cutbacks=6, grow_after=2,
                           **kw):
        """Automatic time incrementation (named in Sec. 2.3, no algorithm
        given; reading of this implementation): try the whole step; after a
        failed attempt (nothing committed) halve the sub-step, after
        ``grow_after`` converged sub-steps in a row double it (never past
        the rest of the step).  Sub-step targets lie on the straight path
        F_bar_0 + f (F_bar_new - F_bar_0) with time f dt; the last one is
        F_bar_new itself.  Fails when the sub-step would fall below
        2^-max_cutbacks of the step; the RVE then returns to its state
        before the call.  Returns (status, substeps, cutbacks, list of the
        sub-steps' (fraction, IncrementInfo))."""
        import copy
        F_bar_new = np.asarray(F_bar_new, dtype=np.float64).reshape(3, 3)
        F0 = self.F_bar.copy()
        done, h, streak, cutbacks = 0.0, 1.0, 0, 0
        snapshot = None
        steps = []
        while done < 1.0:
            h = min(h, 1.0 - done)
            f = done + h
            target = F_bar_new if f == 1.0 else F0 + f * (F_bar_new - F0)
            info = self.increment(target, h * dt, **kw)
            if info.status == OK:
                steps.append((h, info))
                done = f
                streak += 1
                if streak >= grow_after:
                    h *= 2.0
                    streak = 0
                continue
            cutbacks += 1
            streak = 0
            if snapshot is None:
                snapshot = copy.deepcopy(self.__dict__)
            h *= 0.5
            if h < 2.0 ** (-max_cutbacks):
                self.__dict__.update(snapshot)
                return info.status, len(steps), cutbacks, steps
        return OK, len(steps), cutbacks, steps

    # -------------------------------------------------------------- outputs
    def P_bar(self):
        return self.P.mean(axis=0)

    def sigma_bar(self):
        Fb = self.F_bar
        return self.P_bar() @ Fb.T / np.linalg.det(Fb)

    def cauchy(self):
        """Voxel Cauchy stress sigma = P F^T / det F."""
        J = np.linalg.det(self.F)
        return self.P @ np.swapaxes(self.F, 1, 2) / J[:, None, None]


class OracleUmatRVE(OracleRVE):
    """The same increment algorithm with a user material in the form of a
    commercial FE code's subroutine (Appendix A): the material returns the
    Cauchy stress and the Jaumann-rate tangent from (F at t_k, F at t_k-1,
    state variables at t_k-1, dt); P follows from Eq. A.1 and K from
    Eq. A.16.  State variables are committed with the increment; the
    fatigue indicators of the crystal law are not defined for such a
    material and stay zero.

    ``umat(F1, F0, statev, dt) -> (sigma6, ddsdde, statev_new, ok)``.
    """

    def __init__(self, shape, umat_fn, statev0, operator="continuous",
                 L=(1.0, 1.0, 1.0)):
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.umat = umat_fn
        self.statev0 = np.array(statev0, dtype=np.float64).reshape(self.N, -1)
        self.operator = operator
        self.L = tuple(float(x) for x in L)
        self.reset()

    def reset(self):
        super().reset()
        self.statev = self.statev0.copy()

    def constitutive(self, F, dt, dg_start):
        s6, D, sv, ok = self.umat(F, self.F, self.statev, dt)
        sig = umat.sym_from_voigt(s6)
        P = umat.piola_from_cauchy(F, sig)
        K = umat.tangent_from_jaumann(F, sig, umat.tensor_from_voigt(D))
        trial = dict(statev=sv, dg=np.zeros((self.N, 12)))
        return P, K, trial, int(np.count_nonzero(~ok))

    def _commit(self, F, F_bar_new, P, trial, dt):
        self.F = F
        self.F_bar = F_bar_new.copy()
        self.statev = trial["statev"]
        self.P = P
        self.t += dt
        self.increments += 1


def run_history(rve: OracleRVE, history, tol=1e-6, eta=1e-4, newton_max=25,
                cg_max=2000, callback=None):
    """Drive an RVE through a list of increments (see synthetic.loading).

    Per-cycle accumulators are reset at each cycle start.  Returns a list of
    (increment dict, IncrementInfo).
    """
    out = []
    for inc in history:
        if inc["cycle_start"]:
            rve.reset_fips()
        info = rve.increment(inc["F_bar"], inc["dt"], tol, eta, newton_max,
                             cg_max)
        out.append((inc, info))
        if callback is not None:
            callback(inc, info, rve)
        if info.status != OK:
            break
    return out
