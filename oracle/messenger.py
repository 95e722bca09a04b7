"""The multi-messenger Wiener-filter iteration, step by step (float64, CPU).

Follows Section 2 of the paper: equations (ew_t)-(ew_s) for one messenger,
(2mess_t1)-(2mess_s) for two, extended as the paper says (two more fields, a
data-like d and a messenger t, per extra noise term) to the three-term noise
N = N_1/f + N_stripe + N_white used here.  The chain of the hierarchical model
(Appendix A, Fig. 4) runs from the signal to the data:

    s --T_0-- t_0 --Nbar_0-- d_0 --T_1-- t_1 --Nbar_1-- d_1 --T_2-- t_2 --Nbar_2-- d

level 0 = 1/f noise (2-D Fourier diagonal), level 1 = stripes (row basis),
level 2 = white noise (pixel diagonal).  An absent term drops its level; with
only the white term the chain is the single-messenger method of Section 2.

Every field is kept in pixel space.  Each update is the mean of that field's
Gaussian conditional in the joint probability (eqn 2mess_prob), evaluated in the
basis of the one non-scalar covariance it touches:

    t_i = (Nbar_i^-1 + T_i^-1)^-1 (Nbar_i^-1 d_i + T_i^-1 d_{i-1})     (d_{-1} = s)
    d_i = (Nbar_i^-1 + T_{i+1}^-1)^-1 (Nbar_i^-1 t_i + T_{i+1}^-1 t_{i+1})
    s   = (S^-1 + T_0^-1)^-1 T_0^-1 t_0

in the order of the paper (data towards signal): t_2, d_1, t_1, d_0, t_0, s.
Cooling (Section 2) replaces every T_i = tau_i I by lambda tau_i I with the
Nbar_i held fixed; the adaptive schedule is the one of Section 3.3.

Readings where the paper is silent (all recorded in the design notes):
* tau_i = beta_i * (smallest eigenvalue of N_i), beta_i < 1 on levels whose
  both neighbours are free (a singular Nbar there freezes the pair), beta = 1
  allowed on the data-side level;
* the stripe covariance has zero eigenvalues off the row-constant modes, so a
  floor phi = alpha * min(N_pix over observed pixels) is moved from the white
  term to the stripe term (the total N is unchanged);
* one shared lambda for all levels; s in the t_0 update is the s of the
  previous sweep, i.e. S (S + lambda_prev tau_0)^-1 t_0,prev;
* a warm start sets every messenger and data-like field to s_init, and the
  starting s to S (S + lambda_0 tau_0)^-1 s_init;
* the residual uses the true N (Section 2, d_rec = (I + N S^-1) s), with
  S^-1 s formed as (S + T_0)^-1 t_0, on observed pixels; on masked pixels
  S^-1 s itself is reported (it vanishes at the Wiener solution).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from .bases import FourierDiag, PixelDiag, StripeDiag, irfft2u, rfft2u


class NotPositiveDefinite(ValueError):
    """Some messenger covariance tau_i is not positive (an empty noise term;
    the paper notes the method fails then, Section 3.1)."""


class InvalidInput(ValueError):
    pass


CHAINS = ("three", "merged", "augmented")


@dataclass
class Settings:
    beta: Sequence[float] = (0.9, 0.9, 1.0)  # tau fractions for 1/f, stripe, white
    floor_frac: float = 0.5                   # alpha: white floor lent to stripes
    chain: str = "three"                      # which chain of messengers (below)


@dataclass
class Level:
    name: str          # "oof", "stripe" or "white"
    tau: float         # messenger variance at lambda = 1
    nbar: object       # covariance Nbar_i = N_i - tau_i (basis object)
    n_true: object     # the noise term itself, for the residual


@dataclass
class Setup:
    levels: List[Level]
    S: FourierDiag          # signal covariance of the problem
    S_chain: FourierDiag    # covariance of the field at the signal end of the chain
    observed: np.ndarray
    phi: float
    d: np.ndarray
    n_pix: np.ndarray
    shape: tuple
    chain: str = "three"


# An infinite noise variance on a Fourier mode projects the mode out of the
# data (Section 4).  It is carried as this finite value, which every update of
# the multiplied form [B a + A b] / (A + B) turns into its A -> inf limit b up
# to a relative 1e-30 * (largest other covariance).
INFINITE_COV = 1.0e30


def _check_spectrum(name, p, allow_inf=False):
    p = np.asarray(p, dtype=np.float64)
    bad = np.isnan(p) | (p < 0) | (np.isinf(p) if not allow_inf else False)
    if np.any(bad):
        raise InvalidInput(f"{name} must be >= 0 and finite" + (" or +inf" if allow_inf else ""))
    if allow_inf:
        if np.all(np.isinf(p)):
            raise InvalidInput(f"{name}: every mode projected out")
        p = np.where(np.isinf(p), INFINITE_COV, p)
    return p


def setup(problem, settings: Settings = Settings()) -> Setup:
    """Section 2: N_i, tau_i and Nbar_i = N_i - T_i for each present term.

    chain = "three": one messenger level per noise term (1/f, stripe, white),
        the method of Section 2 extended to three terms.
    chain = "merged": the 1/f and stripe terms form one 2-D Fourier-diagonal
        term (stripes live on the k_x = 0 column), as the paper's Section 3.3
        test put the m = 0 stripe power into its harmonic noise term.
    chain = "augmented": every Fourier-diagonal term joins the signal,
        S' = S + N_1/f + N_stripe, and a single messenger carries the white
        noise; s = S S'^-1 u at the end.  This is the Appendix A shortcut
        s = (S^-1 + N_0^-1)^-1 N_0^-1 d_0, valid because S and those noise
        terms share a basis.
    All three have the Wiener filter as their fixed point at lambda = 1.
    """
    if settings.chain not in CHAINS:
        raise InvalidInput(f"unknown chain {settings.chain!r}")
    d = np.asarray(problem.d, dtype=np.float64)
    ny, nx = d.shape
    obs = (np.ones((ny, nx), dtype=bool) if problem.mask is None
           else np.asarray(problem.mask) != 0)
    if not obs.any():
        raise InvalidInput("no observed pixel")
    n_pix = np.asarray(problem.n_pix, dtype=np.float64)
    if not (np.all(np.isfinite(d[obs])) and np.all(np.isfinite(n_pix[obs]))):
        raise InvalidInput("non-finite data or pixel variance")
    s_k = _check_spectrum("signal spectrum", problem.s_k)
    p_oof = (None if problem.p_oof is None
             else _check_spectrum("1/f spectrum", problem.p_oof, allow_inf=True))
    p_st = None if problem.p_stripe is None else _check_spectrum("stripe spectrum", problem.p_stripe)
    b0, b1, b2 = settings.beta
    S = FourierDiag(s_k, (ny, nx))
    S_chain = S
    phi = 0.0
    levels: List[Level] = []

    if settings.chain == "three":
        if p_st is not None:
            phi = settings.floor_frac * float(n_pix[obs].min())
        if p_oof is not None:
            tau0 = b0 * float(p_oof.min())
            levels.append(Level("oof", tau0, FourierDiag(p_oof - tau0, (ny, nx)),
                                FourierDiag(p_oof, (ny, nx))))
        if p_st is not None:
            tau1 = b1 * phi  # smallest eigenvalue of N_stripe + phi I is phi
            levels.append(Level("stripe", tau1, StripeDiag(p_st, phi - tau1, (ny, nx)),
                                StripeDiag(p_st, phi, (ny, nx))))
    else:
        nf = np.zeros_like(s_k)
        if p_oof is not None:
            nf = nf + p_oof
        if p_st is not None:
            nf[:, 0] += nx * p_st
            if p_oof is None:
                phi = settings.floor_frac * float(n_pix[obs].min())
                nf = nf + phi
        if settings.chain == "merged":
            if p_oof is not None or p_st is not None:
                tau0 = b0 * float(nf.min())
                levels.append(Level("fourier", tau0, FourierDiag(nf - tau0, (ny, nx)),
                                    FourierDiag(nf, (ny, nx))))
        else:
            S_chain = FourierDiag(s_k + nf, (ny, nx))

    n2 = n_pix - phi
    tau2 = b2 * float(n2[obs].min())
    levels.append(Level("white", tau2, PixelDiag(n2 - tau2, obs),
                        PixelDiag(n2, obs)))
    for lv in levels:
        if not lv.tau > 0.0:
            raise NotPositiveDefinite(f"tau of level {lv.name} is {lv.tau}")
    return Setup(levels=levels, S=S, S_chain=S_chain, observed=obs, phi=phi,
                 d=d, n_pix=n_pix, shape=(ny, nx), chain=settings.chain)


@dataclass
class State:
    t: List[np.ndarray]       # t_0 .. t_{m-1}
    dd: List[np.ndarray]      # d_0 .. d_{m-2} (d_{m-1} is the data)
    s: np.ndarray


def init_state(st: Setup, lam0: float, s_init: Optional[np.ndarray] = None,
               chain_field: bool = False) -> State:
    """Zero start s = t = d = 0 (Section 2), or every field set to s_init.

    The field at the signal end of the chain is then S_c (S_c + lam0 tau_0)^-1
    s_init (one signal update of the messenger s_init), or s_init itself when
    ``chain_field`` says that s_init already is that field and the chain has
    no Fourier-diagonal messenger level (a chain with one recomputes its
    signal end from t_0 in every sweep, so both readings start alike)."""
    m = len(st.levels)
    if s_init is None:
        z = np.zeros(st.shape)
        return State(t=[z.copy() for _ in range(m)],
                     dd=[z.copy() for _ in range(m - 1)], s=z.copy())
    u = np.asarray(s_init, dtype=np.float64)
    T0 = lam0 * st.levels[0].tau
    if chain_field and len(st.levels) == 1:
        s = u.copy()
    else:
        s = st.S_chain.apply_fn(lambda e: e / (e + T0), u)
    return State(t=[u.copy() for _ in range(m)],
                 dd=[u.copy() for _ in range(m - 1)], s=s)


def sweep(st: Setup, x: State, lam: float,
          on_update: Optional[Callable[[str], None]] = None) -> State:
    """One pass of the messenger equations at cooling parameter lam, data side
    first.  ``on_update(name)`` is called after each single-field update."""
    lv = st.levels
    m = len(lv)
    T = [lam * l.tau for l in lv]
    for i in reversed(range(m)):
        left = x.dd[i - 1] if i > 0 else x.s
        right = x.dd[i] if i < m - 1 else st.d
        x.t[i] = lv[i].nbar.messenger_update(T[i], right, left)
        if on_update:
            on_update(f"t{i}")
        if i > 0:
            x.dd[i - 1] = lv[i - 1].nbar.messenger_update(T[i], x.t[i - 1], x.t[i])
            if on_update:
                on_update(f"d{i - 1}")
    T0 = T[0]
    x.s = st.S_chain.apply_fn(lambda e: e / (e + T0), x.t[0])
    if on_update:
        on_update("s")
    return x


@dataclass
class Diagnostics:
    rho: float         # |m (d_rec - d)| / |m d|: Section 2 residual, observed pixels
    rho_mask: float    # |(1 - m) nu S^-1 s| / |m d|: the masked-pixel part
    dd2: float         # sum over observed pixels of (d_rec - d)^2
    masked_x: float    # |(1 - m) S^-1 s|
    d2: float          # sum over observed pixels of d^2

    @property
    def rho_full(self) -> float:
        return float(np.hypot(self.rho, self.rho_mask))


def diagnostics(st: Setup, x: State, lam: float) -> Diagnostics:
    """Section 2: d_rec(s) = (I + N S^-1) s and Delta d = d_rec - d.  With
    x = S^-1 s = (S_chain + T_0)^-1 t_0 no division by the signal spectrum is
    needed, and s + N x = S_chain x + (sum of the chain's noise terms) x for
    every chain.

    On a masked pixel N is infinite and Delta d is undefined; there the
    Wiener solution has x = 0 instead.  ``rho`` is the observed part (the
    paper's monitor, and the stopping test); ``rho_mask`` measures nu x on
    masked pixels with nu the largest white-noise variance of any observed
    pixel, so that rho = rho_mask = 0 exactly at the Wiener solution.  The
    observed part alone can be tiny while the masked region is still far from
    converged."""
    T0 = lam * st.levels[0].tau
    return _diagnostics_of_x(st, rfft2u(x.t[0]) / (st.S_chain.eig + T0))


def diagnostics_of_field(st: Setup, u: np.ndarray) -> Diagnostics:
    """The same residual for a given signal-end field u = S_chain x (for
    instance a solver's output in field mode 1), with x = S_chain^-1 u formed
    mode by mode.  Well conditioned for the augmented chain, whose S_chain
    includes the Fourier-diagonal noise."""
    return _diagnostics_of_x(st, rfft2u(np.asarray(u, dtype=np.float64)) / st.S_chain.eig)


def _diagnostics_of_x(st: Setup, xk: np.ndarray) -> Diagnostics:
    """Residual of Section 2 from the modes of x = S^-1 s."""
    xs = irfft2u(xk, st.shape)
    # terms diagonal in the 2-D Fourier basis act on x's modes directly (a
    # round trip of x through pixel space would put rounding noise on every
    # mode, which a projected mode's 1e30 variance would then amplify)
    fsum = st.S_chain.eig.copy()
    rec = np.zeros(st.shape)
    for l in st.levels:
        if isinstance(l.n_true, PixelDiag):
            rec += np.where(st.observed, l.n_true.eig * xs, 0.0)
        elif isinstance(l.n_true, FourierDiag):
            fsum = fsum + l.n_true.eig
        else:
            rec += l.n_true.apply(xs)
    rec += irfft2u(fsum * xk, st.shape)
    obs = st.observed
    dd = np.where(obs, rec - st.d, 0.0)
    d2 = float(np.sum(st.d[obs] ** 2))
    dd2 = float(np.sum(dd * dd))
    xm = np.where(obs, 0.0, xs)
    nu = float(st.n_pix[obs].max())
    mx = float(np.sqrt(np.sum(xm ** 2)))
    return Diagnostics(rho=float(np.sqrt(dd2 / d2)), rho_mask=nu * mx / np.sqrt(d2),
                       dd2=dd2, masked_x=mx, d2=d2)


def joint_objective(st: Setup, x: State, lam: float) -> float:
    """-2 log P of the hierarchical model (eqn 2mess_prob, three levels) at
    T_i = lam tau_i: s^T S^-1 s + sum over the chain links of the quadratic
    form of the difference of neighbouring fields."""
    lv = st.levels
    m = len(lv)
    total = st.S_chain.inv_quad(x.s)
    for i in range(m):
        left = x.dd[i - 1] if i > 0 else x.s
        right = x.dd[i] if i < m - 1 else st.d
        dl = x.t[i] - left
        total += float(np.sum(dl * dl)) / (lam * lv[i].tau)
        total += lv[i].nbar.inv_quad(right - x.t[i])
    return total


# --------------------------------------------------------------------------
# schedules (Section 2 cooling; Section 3.3 adaptive recipe)
# --------------------------------------------------------------------------

@dataclass
class FixedSchedule:
    lams: Sequence[float]

    def first(self) -> float:
        return float(self.lams[0])

    def at(self, k: int) -> float:
        return float(self.lams[min(k, len(self.lams) - 1)])


@dataclass
class AdaptiveSchedule:
    """Start at lam0; when Delta d^T Delta d changes by less than ``plateau``
    per sweep, set lam <- lam^shrink; lam is set to 1 once lam - 1 < snap."""
    lam0: float = 1.0e4
    shrink: float = 0.7
    plateau: float = 1.0e-2
    snap: float = 1.0e-3

    def first(self) -> float:
        return float(self.lam0)


def next_lambda(schedule: AdaptiveSchedule, lam: float, prev: Optional[tuple], k: int,
                dd2: float) -> tuple:
    """One decision of the Section 3.3 recipe at a residual check after sweep
    k (0-based) with squared residual dd2 = Delta d^T Delta d.  ``prev`` is
    (k, dd2) of the previous check, or None at the first one.

    The paper waits until Delta d^T Delta d changes by less than 1e-2 per
    iteration and then lowers lam to lam^0.7.  With checks every few sweeps
    the per-iteration change is the change since the previous check divided
    by the sweeps between them, relative to dd2.  lam^0.7 only approaches 1,
    so lam is set to 1 once lam - 1 < snap.  Returns (new lam, new prev)."""
    if prev is not None and abs(dd2 - prev[1]) < schedule.plateau * (k - prev[0]) * dd2:
        lam = lam ** schedule.shrink
        if lam - 1.0 < schedule.snap:
            lam = 1.0
    return lam, (k, dd2)


def cooling_ramp(n_cool: int, n_total: int, lam0: float = 1.0e4) -> np.ndarray:
    """lam_k = lam0^(1 - k/n_cool) for k < n_cool, then 1 up to n_total."""
    k = np.arange(n_total, dtype=np.float64)
    lam = np.where(k < n_cool, lam0 ** (1.0 - k / n_cool), 1.0)
    return lam


@dataclass
class Result:
    s: np.ndarray
    sweeps: int
    converged: bool
    lam_used: List[float] = field(default_factory=list)
    trace: List[tuple] = field(default_factory=list)  # (sweep, lam, rho, dd2, rho_mask)
    state: Optional[State] = None


def solve(problem, schedule, *, settings: Settings = Settings(),
          s_init: Optional[np.ndarray] = None, max_sweeps: int = 1000,
          monitor_every: int = 1, rtol: float = 0.0,
          full_residual: bool = False, chain_field: bool = False,
          record_joint: bool = False) -> Result:
    """Iterate sweeps under a cooling schedule.

    Every ``monitor_every`` sweeps (and after the last sweep) the residual is
    evaluated; the solve stops when lam = 1 and rho <= rtol, or after
    ``max_sweeps`` (with ``full_residual`` the test uses hypot(rho, rho_mask)).
    With ``chain_field`` the warm start and the result are the chain's
    signal-end field u = S_chain x instead of s = S x (they differ only for
    the augmented chain, where u = s + N_F x).
    An adaptive schedule changes lam only at those points:
    if |dd2 - dd2_prev| < plateau * (sweeps since prev) * dd2, lam <- lam^shrink.
    With ``record_joint`` each trace record also holds the joint objective
    J_lam of the state (eqn 2mess_prob) as a sixth value.
    """
    st = setup(problem, settings)
    lam = schedule.first()
    x = init_state(st, lam, s_init, chain_field)
    res = Result(s=x.s, sweeps=0, converged=False)
    prev = None  # (k, dd2)
    adaptive = isinstance(schedule, AdaptiveSchedule)
    k = 0
    while k < max_sweeps:
        if not adaptive:
            lam = schedule.at(k)
        sweep(st, x, lam)
        res.lam_used.append(lam)
        k += 1
        if k % monitor_every == 0 or k == max_sweeps:
            dg = diagnostics(st, x, lam)
            rec = (k - 1, lam, dg.rho, dg.dd2, dg.rho_mask)
            if record_joint:
                rec = rec + (joint_objective(st, x, lam),)
            res.trace.append(rec)
            if not np.isfinite(dg.dd2):
                break
            if lam == 1.0 and (dg.rho_full if full_residual else dg.rho) <= rtol:
                res.converged = True
                break
            if adaptive:
                lam, prev = next_lambda(schedule, lam, prev, k - 1, dg.dd2)
    res.s = final_chain_field(st, x, lam) if chain_field else final_signal(st, x, lam)
    res.sweeps = k
    res.state = x
    return res


def final_signal(st: Setup, x: State, lam: float) -> np.ndarray:
    """s = S (S_chain + T_0)^-1 t_0: eqn 2mess_s for the three-level and
    merged chains, followed by s = S S'^-1 u for the augmented chain."""
    T0 = lam * st.levels[0].tau
    return st.S.apply(st.S_chain.apply_fn(lambda e: 1.0 / (e + T0), x.t[0]))


def final_chain_field(st: Setup, x: State, lam: float) -> np.ndarray:
    """u = S_chain (S_chain + T_0)^-1 t_0: the field at the signal end of the
    chain (equal to s except for the augmented chain)."""
    T0 = lam * st.levels[0].tau
    return st.S_chain.apply_fn(lambda e: e / (e + T0), x.t[0])


def rfft2_of(u):
    return rfft2u(u)


def irfft2_of(uk, shape):
    return irfft2u(uk, shape)


def inverse_noise_weight(problem, alpha: float, schedule, **kw) -> Result:
    """Section 4: N^-1 d ~= alpha^-1 [alpha I (alpha I + N)^-1 d].  Runs the
    messenger iteration with the flat signal covariance S = alpha I and
    returns the result divided by alpha in ``Result.s``."""
    import copy
    q = copy.copy(problem)
    q.s_k = np.full_like(np.asarray(problem.s_k, dtype=np.float64), float(alpha))
    res = solve(q, schedule, **kw)
    res.s = res.s / alpha
    return res
