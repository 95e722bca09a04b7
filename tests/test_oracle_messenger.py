"""Pins of the oracle's messenger iteration.

Each pin checks the oracle against something other than its own formulas:
the exact minimiser of a dense joint quadratic, a dense Cholesky solve, a
Fourier closed form, the chi^2 gradient, or an invariant of the method.
"""

import dataclasses
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import bases, direct, messenger
from oracle.messenger import State

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers: dense matrices built from the problem definition
# --------------------------------------------------------------------------

def _tiny_problem(mask=True, seed=5):
    p = synth.make_problem(8, 8, seed, pix_arcmin=20.0)
    if mask:
        m = np.ones((8, 8), np.uint8)
        m[2:4, 3:6] = 0
        m[6, 0] = 0
        p.mask = m
    return p


def _dense_chain(p, settings, lam):
    """Covariances along the chain, signal end first, as dense matrices:
    [S_chain, T_0, Nbar_0, T_1, Nbar_1, ...], built from the problem arrays
    with tau_i recomputed from eigenvalues of the dense noise terms."""
    ny, nx = p.d.shape
    n = ny * nx
    I = np.eye(n)
    obs = np.ones(n, bool) if p.mask is None else p.mask.ravel() != 0
    b0, b1, b2 = settings.beta
    S = direct.stationary_cov_dense(p.s_k, nx)
    Noof = direct.stationary_cov_dense(p.p_oof, nx)
    Nst = direct.stripe_cov_dense(p.p_stripe, nx)
    npix = p.n_pix.ravel()
    covs, nbar_pix = [], None
    if settings.chain == "three":
        phi = settings.floor_frac * npix[obs].min()
        N1 = Nst + phi * I
        tau0 = b0 * np.linalg.eigvalsh(Noof).min()
        tau1 = b1 * np.linalg.eigvalsh(N1).min()
        tau2 = b2 * (npix - phi)[obs].min()
        covs = [S, lam * tau0 * I, Noof - tau0 * I, lam * tau1 * I, N1 - tau1 * I,
                lam * tau2 * I]
        nbar_pix = npix - phi - tau2
    elif settings.chain == "merged":
        NF = Noof + Nst
        tau0 = b0 * np.linalg.eigvalsh(NF).min()
        tau2 = b2 * npix[obs].min()
        covs = [S, lam * tau0 * I, NF - tau0 * I, lam * tau2 * I]
        nbar_pix = npix - tau2
    else:
        tau2 = b2 * npix[obs].min()
        covs = [S + Noof + Nst, lam * tau2 * I]
        nbar_pix = npix - tau2
    return covs, nbar_pix, obs


def _joint_hessian(covs, nbar_pix, obs, d):
    """J = z^T H z - 2 b^T z + const for fields z = (s, t_0, d_0, ..., t_last)
    linked by the chain covariances, the last one tied to the data d."""
    n = d.size
    nf = len(covs)
    H = np.zeros((nf * n, nf * n))
    b = np.zeros(nf * n)

    def blk(i):
        return slice(i * n, (i + 1) * n)

    H[blk(0), blk(0)] += np.linalg.inv(covs[0])
    for i in range(1, nf):
        M = np.linalg.inv(covs[i])
        H[blk(i - 1), blk(i - 1)] += M
        H[blk(i), blk(i)] += M
        H[blk(i - 1), blk(i)] -= M
        H[blk(i), blk(i - 1)] -= M
    winv = np.where(obs, 1.0 / np.where(obs, nbar_pix, 1.0), 0.0)
    H[blk(nf - 1), blk(nf - 1)] += np.diag(winv)
    b[blk(nf - 1)] += winv * d.ravel()
    return H, b, blk


def _fields(x):
    out = [x.s]
    for i in range(len(x.t)):
        out.append(x.t[i])
        if i < len(x.dd):
            out.append(x.dd[i])
    return out


def _vec(x):
    return np.concatenate([f.ravel() for f in _fields(x)])


# --------------------------------------------------------------------------
# every single update is the exact conditional minimiser (eqn 2mess_prob)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("chain", ["three", "merged", "augmented"])
@pytest.mark.parametrize("lam", [1.0, 7.0])
def test_each_update_is_exact_conditional_minimiser(chain, lam):
    p = _tiny_problem()
    settings = oracle.Settings(beta=(0.8, 0.7, 0.9), floor_frac=0.5, chain=chain)
    st = oracle.setup(p, settings)
    covs, nbar_pix, obs = _dense_chain(p, settings, lam)
    H, b, blk = _joint_hessian(covs, nbar_pix, obs, p.d)
    m = len(st.levels)
    rng = np.random.default_rng(0)
    x = State(t=[30 * rng.standard_normal(p.d.shape) for _ in range(m)],
              dd=[30 * rng.standard_normal(p.d.shape) for _ in range(m - 1)],
              s=30 * rng.standard_normal(p.d.shape))
    # position of each named field in the chain vector
    pos = {"s": 0}
    for i in range(m):
        pos[f"t{i}"] = 2 * i + 1
        pos[f"d{i}"] = 2 * i + 2
    nf = len(covs)
    prev = [_vec(x)]
    seen = []

    def check(name):
        z0, z1 = prev[0], _vec(x)
        i = pos[name]
        rest = b[blk(i)] - sum(H[blk(i), blk(j)] @ z0[blk(j)] for j in range(nf) if j != i)
        expect = np.linalg.solve(H[blk(i), blk(i)], rest)
        got = z1[blk(i)]
        assert np.linalg.norm(got - expect) <= 1e-11 * np.linalg.norm(expect), name
        others = np.delete(z1 - z0, np.r_[blk(i)])
        assert np.all(others == 0.0), name
        seen.append(name)
        prev[0] = z1

    oracle.sweep(st, x, lam, on_update=check)
    expected_order = {"three": ["t2", "d1", "t1", "d0", "t0", "s"],
                      "merged": ["t1", "d0", "t0", "s"],
                      "augmented": ["t0", "s"]}[chain]
    assert seen == expected_order


# --------------------------------------------------------------------------
# the fixed point is the Wiener filter
# --------------------------------------------------------------------------

def _easy_three_term(seed=7, mask=False):
    p = synth.make_problem(32, 32, seed, pix_arcmin=4.0, stripe_rms=3.0,
                           white_contrast=0.2)
    if mask:
        m = np.ones((32, 32), np.uint8)
        yy, xx = np.mgrid[:32, :32]
        m[(yy - 10) ** 2 + (xx - 20) ** 2 <= 16] = 0
        p.mask = m
    return p


def test_three_level_chain_converges_to_dense_cholesky():
    """Unmasked: with a mask the three-level chain needs far more sweeps than a
    unit test affords (masked regions are the slowest, Section 3.2); the masked
    fixed point is pinned through the variant chains below."""
    p = _easy_three_term(mask=False)
    sd = direct.wiener_dense(p)
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     max_sweeps=30000, monitor_every=4, rtol=1e-11)
    assert r.converged
    assert np.linalg.norm(r.s - sd) / np.linalg.norm(sd) < 1e-9


@pytest.mark.parametrize("chain,mask", [("augmented", True), ("augmented", False),
                                        ("merged", False)])
def test_variant_chains_share_the_fixed_point(chain, mask):
    """Appendix A shortcuts keep the Wiener fixed point.  (The merged chain
    with a mask needs more sweeps than a unit test affords.)"""
    p = _easy_three_term(mask=mask)
    sd = direct.wiener_dense(p)
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     settings=oracle.Settings(chain=chain),
                     max_sweeps=40000, monitor_every=4, rtol=1e-12, full_residual=True)
    assert r.converged
    assert np.linalg.norm(r.s - sd) / np.linalg.norm(sd) < 1e-9


def test_c1_augmented_chain_matches_dense_cholesky():
    """The 64x64 three-term workload against the 4096x4096 Cholesky solve."""
    p = synth.named_config("c1")
    sd = direct.wiener_dense(p)
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e4, plateau=1e-2),
                     settings=oracle.Settings(chain="augmented"),
                     max_sweeps=5000, monitor_every=1, rtol=1e-12)
    assert r.converged
    assert np.linalg.norm(r.s - sd) / np.linalg.norm(sd) < 1e-10


def test_stationary_closed_form_three_levels():
    """No mask, uniform white noise: N is Fourier diagonal and the Wiener
    filter is a per-mode ratio; the stripe term sits on k_x = 0 there, while
    the iteration applies it through row means."""
    p = synth.make_stationary_problem(32, 32, 11, pix_arcmin=4.0, stripe_rms=3.0)
    sc = direct.wiener_stationary(p)
    np.testing.assert_allclose(sc, direct.wiener_dense(p), rtol=0, atol=1e-10 * np.abs(sc).max())
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     max_sweeps=30000, monitor_every=4, rtol=1e-12)
    assert r.converged
    assert np.linalg.norm(r.s - sc) / np.linalg.norm(sc) < 1e-10


def test_ew_limit_converges_in_one_sweep():
    """Section 3.1: with only uniform white noise and tau = sigma^2 the
    messenger takes all of the noise and one sweep gives the exact filter."""
    p = synth.make_stationary_problem(64, 64, 3, oof_level=None, stripe_rms=None)
    settings = oracle.Settings(beta=(0.9, 0.9, 1.0))
    st = oracle.setup(p, settings)
    x = oracle.init_state(st, 1.0)
    oracle.sweep(st, x, 1.0)
    sigma2 = p.n_pix[0, 0]
    dk = np.fft.rfft2(p.d)
    expect = np.fft.irfft2(p.s_k / (p.s_k + sigma2) * dk, s=p.d.shape)
    np.testing.assert_allclose(x.s, expect, rtol=0, atol=1e-13 * np.abs(expect).max())


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("chain", ["three", "merged"])
def test_joint_objective_never_increases(chain):
    """Appendix A: every update maximises P_2 along one field, so J_lambda
    cannot go up after any single-field update at fixed lambda."""
    p = _easy_three_term(mask=True)
    settings = oracle.Settings(beta=(0.9, 0.9, 0.95), chain=chain)
    st = oracle.setup(p, settings)
    x = oracle.init_state(st, 5.0)
    for lam in [50.0, 5.0, 1.0]:
        js = [oracle.joint_objective(st, x, lam)]

        def cb(_name):
            js.append(oracle.joint_objective(st, x, lam))
        for _ in range(5):
            oracle.sweep(st, x, lam, on_update=cb)
        steps = np.diff(js)
        assert np.all(steps <= 1e-12 * abs(js[0])), steps.max()


def test_residual_is_noise_times_half_chi2_gradient():
    """N grad(chi^2)/2 = (I + N S^-1) s - d = Delta d for any s (Sections 1
    and 2, no mask), checked with dense N at an arbitrary state."""
    p = _easy_three_term(mask=False)
    st = oracle.setup(p)
    x = oracle.init_state(st, 1.0)
    for _ in range(3):
        oracle.sweep(st, x, 3.0)
    lam = 3.0
    dg = oracle.diagnostics(st, x, lam)
    s = oracle.messenger.final_signal(st, x, lam)
    _, N = direct.dense_covariances(p)
    g = direct.grad_chi2_dense(p, s)
    dd = N @ (0.5 * g.ravel())
    assert np.sqrt(np.sum(dd ** 2)) == pytest.approx(np.sqrt(dg.dd2), rel=1e-9)
    assert dg.rho == pytest.approx(np.linalg.norm(dd) / np.linalg.norm(p.d), rel=1e-9)


def test_converged_solution_is_stationary_and_profile_identity_holds():
    """At convergence grad chi^2 = 0, and min over messengers of J_1 equals
    chi^2(s) (marginalising the messengers returns P(s, d), Appendix A)."""
    p = _easy_three_term(mask=False)
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     max_sweeps=30000, monitor_every=4, rtol=1e-12)
    assert r.converged
    g = direct.grad_chi2_dense(p, r.s)
    sk = np.fft.fft2(r.s, norm="ortho")
    prior_grad_scale = np.linalg.norm(
        np.fft.ifft2(sk / bases.full_from_half(p.s_k, 32), norm="ortho").real)
    assert np.linalg.norm(g) < 1e-8 * prior_grad_scale
    st = oracle.setup(p)
    J = oracle.joint_objective(st, r.state, 1.0)
    assert J == pytest.approx(direct.chi2_dense(p, r.s), rel=1e-9)


def test_unit_beta_on_inner_level_locks_modes():
    """tau_1 equal to the smallest stripe-level eigenvalue makes Nbar_1 zero
    off the row-constant modes: d_1 and t_1 then copy each other and those
    components never leave their start."""
    p = _easy_three_term()
    st = oracle.setup(p, oracle.Settings(beta=(0.9, 1.0, 1.0)))
    x = oracle.init_state(st, 1.0)
    for _ in range(20):
        oracle.sweep(st, x, 10.0)
    t1 = x.t[1]
    off_rows = t1 - t1.mean(axis=1, keepdims=True)
    assert np.max(np.abs(off_rows)) == 0.0
    assert np.max(np.abs(t1)) > 0.0  # the row-constant part did move


def test_cooling_beats_no_cooling():
    """Section 3.3: without cooling the iteration is much slower."""
    p = _easy_three_term(mask=True)
    kw = dict(settings=oracle.Settings(chain="augmented"), max_sweeps=3000,
              monitor_every=1, rtol=1e-6)
    cooled = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3), **kw)
    flat = oracle.solve(p, oracle.FixedSchedule([1.0]), **kw)
    assert cooled.converged
    assert (not flat.converged) or flat.sweeps > cooled.sweeps


def test_more_noise_in_fourier_level_converges_faster():
    """Section 3.1: uniform white noise split between a harmonic term and a
    pixel term converges faster the more of it sits in the harmonic term."""
    sweeps = {}
    for frac in (0.99, 0.5):
        p = synth.make_stationary_problem(32, 32, 4, oof_level=None, stripe_rms=None)
        sigma2 = p.n_pix[0, 0]
        p.p_oof = np.full_like(p.s_k, frac * sigma2)
        p.n_pix = np.full_like(p.n_pix, (1 - frac) * sigma2)
        r = oracle.solve(p, oracle.FixedSchedule([1.0]),
                         settings=oracle.Settings(beta=(0.5, 0.9, 0.5)),
                         max_sweeps=5000, monitor_every=1, rtol=1e-6)
        assert r.converged
        sweeps[frac] = r.sweeps
    assert sweeps[0.99] < sweeps[0.5]


def _chi2_uniform(p, s, sigma2):
    """chi^2(s) = |d - s|^2 / sigma^2 + s^T S^-1 s for uniform white noise,
    with the unitary transform's half-plane weights (nx even)."""
    nx = p.d.shape[1]
    sk = np.fft.rfft2(s, norm="ortho")
    w = np.ones_like(p.s_k)
    w[:, 1:nx // 2] = 2.0
    return float(np.sum((p.d - s) ** 2) / sigma2 + np.sum(w * np.abs(sk) ** 2 / p.s_k))


def test_section_3_1_iteration_counts_match_the_paper():
    """Section 3.1 prints how many iterations (no cooling) the method needs
    before chi^2 is within one part in 1e3 of its converged value, for
    uniform white noise with 99% or 50% of its power in the harmonic term
    N_0: 4 and 75.  The oracle (default tau fractions) on a 64^2 map with a
    red signal spectrum needs exactly 4 for the 99% split; the 50% count
    depends on the signal spectrum (the paper's is a beam-smoothed CMB
    spectrum on a HEALPix N_side = 64 sphere), so it is held to a factor
    of two of the printed value."""
    gold = json.load(open(os.path.join(GOLDEN, "sec3_1_uniform_noise.json")))
    n = 64
    p0 = synth.make_problem(n, n, 7, oof_level=None, stripe_rms=None, white_contrast=0.0,
                            mask_frac=0.0)
    sigma2 = float(p0.n_pix[0, 0])
    dk = np.fft.rfft2(p0.d, norm="ortho")
    s_star = np.fft.irfft2(p0.s_k / (p0.s_k + sigma2) * dk, s=(n, n), norm="ortho")
    c_star = _chi2_uniform(p0, s_star, sigma2)
    counts = []
    for frac in gold["fraction_in_N0"]:
        p = dataclasses.replace(p0, p_oof=np.full_like(p0.s_k, frac * sigma2),
                                n_pix=np.full_like(p0.n_pix, (1 - frac) * sigma2))
        st = oracle.setup(p)
        x = oracle.init_state(st, 1.0)
        k = 0
        while k < 1000:
            oracle.sweep(st, x, 1.0)
            k += 1
            s = messenger.final_signal(st, x, 1.0)
            if abs(_chi2_uniform(p, s, sigma2) - c_star) / c_star < 1e-3:
                break
        counts.append(k)
    k99, k50 = counts
    g99, g50 = gold["iterations"]
    assert k99 == g99
    assert g50 / 2 <= k50 <= 2 * g50


def test_convergence_is_exponential_at_unit_lambda():
    """Section 3.2: once the fast modes have died out the log residual falls
    linearly with the sweep count."""
    p = _easy_three_term(mask=True)
    r = oracle.solve(p, oracle.FixedSchedule([1.0]),
                     settings=oracle.Settings(chain="augmented"),
                     max_sweeps=2000, monitor_every=1)
    rho = np.array([np.hypot(t[2], t[4]) for t in r.trace])
    late = np.log(rho[1200:2000])
    k = np.arange(late.size)
    slope, icpt = np.polyfit(k, late, 1)
    assert slope < 0
    assert np.max(np.abs(late - (slope * k + icpt))) < 0.02 * abs(late[0] - late[-1])


# --------------------------------------------------------------------------
# error conditions (Section 3.1: an empty covariance makes the method fail)
# --------------------------------------------------------------------------

def test_empty_noise_term_is_not_positive_definite():
    p = _easy_three_term()
    p.p_oof = np.zeros_like(p.p_oof)
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.setup(p)


def test_stripe_level_without_floor_is_not_positive_definite():
    p = _easy_three_term()
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.setup(p, oracle.Settings(floor_frac=0.0))


def test_all_masked_is_invalid():
    p = _easy_three_term()
    p.mask = np.zeros_like(p.d, dtype=np.uint8)
    with pytest.raises(oracle.InvalidInput):
        oracle.setup(p)


def test_masked_pixels_are_ignored():
    p = _easy_three_term(mask=True)
    r1 = oracle.solve(p, oracle.FixedSchedule(oracle.cooling_ramp(20, 40, 1e3)), max_sweeps=40)
    q = _easy_three_term(mask=True)
    q.d = np.where(q.mask == 0, 1e6, q.d)
    q.n_pix = np.where(q.mask == 0, -5.0, q.n_pix)
    r2 = oracle.solve(q, oracle.FixedSchedule(oracle.cooling_ramp(20, 40, 1e3)), max_sweeps=40)
    np.testing.assert_array_equal(r1.s, r2.s)


def _chain_field_dense(p, chain):
    """u = S_chain x with x = S^-1 s from the dense Cholesky solve; S_chain is
    S + N_1/f + N_stripe for the augmented chain (built here from dense
    circulant and stripe matrices) and S otherwise."""
    ny, nx = p.d.shape
    x = direct.wiener_dense_x(p).ravel()
    Sc = direct.stationary_cov_dense(p.s_k, nx)
    if chain == "augmented":
        Sc = Sc + direct.stationary_cov_dense(p.p_oof, nx) + direct.stripe_cov_dense(p.p_stripe, nx)
    return (Sc @ x).reshape(ny, nx)


@pytest.mark.parametrize("mask", [False, True])
def test_chain_field_output_and_exact_warm_start(mask):
    """Augmented chain: the chain-field output of a converged solve is
    (S + N_F) x with x from the dense Cholesky solve, and starting from that
    field at lambda = 1 is already the fixed point (no sweep moves it)."""
    p = _easy_three_term(mask=mask)
    st = oracle.setup(p, oracle.Settings(chain="augmented"))
    if st.phi > 0:
        pytest.skip("stripe floor without a 1/f partner changes S_chain")
    ud = _chain_field_dense(p, "augmented")
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     settings=oracle.Settings(chain="augmented"), max_sweeps=40000,
                     monitor_every=4, rtol=1e-12, full_residual=True, chain_field=True)
    assert r.converged
    assert np.linalg.norm(r.s - ud) / np.linalg.norm(ud) < 1e-9
    # the residual of the dense field, evaluated from the field alone
    assert oracle.diagnostics_of_field(st, ud).rho < 1e-9
    w = oracle.solve(p, oracle.FixedSchedule([1.0]), settings=oracle.Settings(chain="augmented"),
                     s_init=ud, max_sweeps=5, monitor_every=1, chain_field=True)
    assert w.trace[0][2] < 1e-9
    assert np.linalg.norm(w.s - ud) / np.linalg.norm(ud) < 1e-9
    # the signal-mode warm start from the same field is not at the fixed point
    v = oracle.solve(p, oracle.FixedSchedule([1.0]), settings=oracle.Settings(chain="augmented"),
                     s_init=ud, max_sweeps=1, monitor_every=1)
    assert v.trace[0][2] > 1e-6


def test_chain_field_is_the_signal_for_chains_with_a_fourier_level():
    p = _easy_three_term(mask=True)
    lams = list(oracle.cooling_ramp(10, 20, 30.0))
    a = oracle.solve(p, oracle.FixedSchedule(lams), s_init=p.s_true, max_sweeps=20)
    b = oracle.solve(p, oracle.FixedSchedule(lams), s_init=p.s_true, max_sweeps=20, chain_field=True)
    # the same iterates; the two outputs differ only in rounding (S x formed
    # with one or two transforms)
    assert [t[2] for t in a.trace] == [t[2] for t in b.trace]
    assert np.linalg.norm(a.s - b.s) / np.linalg.norm(a.s) < 1e-13


def _projected(p, modes):
    """Copy of p with the 1/f variance of the given half-spectrum modes set
    to +inf (projected out)."""
    import dataclasses
    po = np.array(p.p_oof, dtype=np.float64)
    for ky, kx in modes:
        po[ky, kx] = np.inf
    return dataclasses.replace(p, p_oof=po)


LOW_MODES = [(0, 0), (1, 0), (31, 0), (0, 1), (1, 1), (31, 1)]


@pytest.mark.parametrize("chain,mask", [("augmented", True), ("augmented", False),
                                        ("three", False)])
def test_projected_modes_match_the_exact_limit(chain, mask):
    """Section 4: infinite covariance on chosen Fourier modes removes them
    from the data.  The converged iteration equals the exact limit computed
    on the subspace orthogonal to those modes (and to masked pixels).

    The three-level chain's residual is not usable here: its 1/f term
    multiplies x by 1e30 on the projected modes, where the pixel-space fields
    of this reference carry rounding noise; the fields themselves converge,
    so that chain runs a fixed number of sweeps instead."""
    p = _projected(_easy_three_term(mask=mask), LOW_MODES)
    sd = direct.wiener_projected_dense(p)
    if chain == "augmented":
        r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                         settings=oracle.Settings(chain=chain), max_sweeps=40000,
                         monitor_every=4, rtol=1e-12, full_residual=True)
        assert r.converged
    else:
        r = oracle.solve(p, oracle.FixedSchedule(list(oracle.cooling_ramp(2000, 12000, 1e3))),
                         settings=oracle.Settings(chain=chain), max_sweeps=12000,
                         monitor_every=1000)
    assert np.linalg.norm(r.s - sd) / np.linalg.norm(sd) < 1e-8
    # the projected modes carry no signal in the result when nothing couples
    # them to the rest (no mask): the estimate is orthogonal to them
    if not mask:
        sk = np.fft.rfft2(r.s)
        for ky, kx in LOW_MODES:
            assert abs(sk[ky, kx]) < 1e-8 * np.abs(sk).max()


def test_projected_modes_stationary_closed_form():
    """No mask, uniform white noise: s_k = S / (S + N) d_k with N = inf on the
    projected modes, i.e. those modes of the estimate are zero."""
    p = synth.make_stationary_problem(32, 32, 3)
    p = _projected(p, LOW_MODES)
    ref = direct.wiener_stationary(p)
    lams = [1.0]
    r = oracle.solve(p, oracle.FixedSchedule(lams), settings=oracle.Settings(chain="augmented",
                     beta=(0.9, 0.9, 1.0)), max_sweeps=1)
    assert np.linalg.norm(r.s - ref) / np.linalg.norm(ref) < 1e-12


def test_projected_mode_errors():
    p = _easy_three_term()
    import dataclasses
    with pytest.raises(oracle.InvalidInput):
        oracle.setup(dataclasses.replace(p, p_oof=np.full_like(p.p_oof, np.inf)))
    bad = np.array(p.p_oof)
    bad[2, 2] = -np.inf
    with pytest.raises(oracle.InvalidInput):
        oracle.setup(dataclasses.replace(p, p_oof=bad))


def test_projected_dense_limit_matches_closed_form():
    """The exact projected-mode limit (dense, on the orthogonal subspace)
    equals the Fourier closed form with zero gain on the projected modes when
    the noise is stationary (no mask, uniform white noise), and equals the
    plain dense Wiener filter when nothing is projected."""
    p = synth.make_stationary_problem(16, 16, 4, pix_arcmin=8.0)
    q = _projected(p, [(0, 0), (1, 0), (15, 0), (0, 1)])
    a = direct.wiener_projected_dense(q)
    b = direct.wiener_stationary(q)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-10
    r = _easy_three_term(mask=True)
    c = direct.wiener_projected_dense(r)
    d = direct.wiener_dense(r)
    assert np.linalg.norm(c - d) / np.linalg.norm(d) < 1e-10


# --------------------------------------------------------------------------
# the adaptive cooling rule of Section 3.3, on hand-built residual sequences
# --------------------------------------------------------------------------

def _replay(sched, ks, dd2s, lam0):
    """lambda in force after each residual check, by oracle.next_lambda."""
    lam, prev, out = lam0, None, []
    for k, v in zip(ks, dd2s):
        lam, prev = oracle.next_lambda(sched, lam, prev, k, v)
        out.append(lam)
    return out


def test_adaptive_rule_shrinks_exactly_on_a_one_percent_plateau():
    """Section 3.3: lambda starts large; whenever Delta d^T Delta d changes by
    less than 1e-2 per iteration, lambda is lowered to lambda^0.7.  Checks
    after every sweep; the expected values are written out by hand."""
    sched = oracle.AdaptiveSchedule(lam0=1e4, shrink=0.7, plateau=1e-2, snap=1e-3)
    dd2 = [100.0, 90.0, 89.5, 89.0, 88.0, 101.0, 100.0]
    got = _replay(sched, range(len(dd2)), dd2, 1e4)
    l1 = 10.0 ** 2.8           # (1e4)^0.7
    l2 = 10.0 ** (2.8 * 0.7)   # (1e4)^(0.7^2)
    expect = [1e4,             # first check: nothing to compare with
              1e4,             # 10 / 90 = 11 % per sweep
              l1,              # 0.5 / 89.5 = 0.56 % per sweep: plateau
              l2,              # 0.5 / 89 = 0.56 %: plateau again
              l2,              # 1 / 88 = 1.14 %: still moving
              l2,              # 13 / 101: moving
              l2]              # 1 / 100 is exactly 1 %: not below it
    np.testing.assert_allclose(got, expect, rtol=1e-14)


def test_adaptive_rule_counts_sweeps_between_checks():
    """With a check every 4 sweeps the change per iteration is the change
    since the last check over 4: 3 in 4 sweeps at dd2 = 97 is 0.77 % per
    sweep (plateau), 4 in 4 sweeps at 93 is 1.08 % (not)."""
    sched = oracle.AdaptiveSchedule(lam0=1e4, shrink=0.7, plateau=1e-2, snap=1e-3)
    got = _replay(sched, [3, 7, 11], [100.0, 97.0, 93.0], 1e4)
    np.testing.assert_allclose(got, [1e4, 10.0 ** 2.8, 10.0 ** 2.8], rtol=1e-14)


def test_adaptive_rule_snaps_to_one_and_needs_26_shrinks_from_1e4():
    """lambda^0.7 only approaches 1; the reading here sets lambda = 1 once
    lambda - 1 < 1e-3.  1.0015^0.7 = 1.00105 stays, its next power 1.00073
    snaps.  From 1e4, 0.7^n ln(1e4) < ln(1 + 1e-3) first holds at n = 26."""
    sched = oracle.AdaptiveSchedule(lam0=1.0015, shrink=0.7, plateau=1e-2, snap=1e-3)
    got = _replay(sched, [0, 1, 2], [5.0, 5.0, 5.0], 1.0015)
    assert got[0] == 1.0015
    assert got[1] == pytest.approx(1.0015 ** 0.7, rel=1e-15) and got[1] - 1.0 > 1e-3
    assert got[2] == 1.0
    sched = oracle.AdaptiveSchedule(lam0=1e4)
    lams = _replay(sched, range(40), [7.0] * 40, 1e4)
    n_shrinks = sum(1 for a, b in zip([1e4] + lams, lams) if b < a)
    assert n_shrinks == 26
    assert lams[26] == 1.0 and lams[25] > 1.0
    assert lams[-1] == 1.0


def test_solve_follows_the_adaptive_rule():
    """The lambdas an adaptive oracle solve ran match the rule replayed on
    the residuals of its own trace (the wiring of solve)."""
    p = _easy_three_term(mask=True)
    sched = oracle.AdaptiveSchedule(lam0=1e3, plateau=5e-2)
    K = 3
    r = oracle.solve(p, sched, settings=oracle.Settings(chain="augmented"), max_sweeps=300,
                     monitor_every=K)
    ks = [t[0] for t in r.trace]
    lam_after = _replay(sched, ks, [t[3] for t in r.trace], 1e3)
    # lambda of the sweeps after each check is the rule's output there
    for (k, lam_at, *_), nxt in zip(r.trace[1:], lam_after[:-1]):
        assert lam_at == nxt
    assert r.trace[0][1] == 1e3 and r.trace[-1][1] < 1e3


# --------------------------------------------------------------------------
# the start is not critical (Section 2): warm starts reach the same solution
# --------------------------------------------------------------------------

@pytest.mark.parametrize("chain,mask", [("three", False), ("augmented", True)])
@pytest.mark.parametrize("start", ["truth", "constant"])
def test_warm_start_converges_to_the_dense_solution(chain, mask, start):
    """Section 2 states that the initial values do not matter for the
    result.  From the true signal, and from a constant 50 uK field, the
    iteration reaches the dense Cholesky Wiener solution."""
    p = _easy_three_term(mask=mask)
    sd = direct.wiener_dense(p)
    s0 = p.s_true if start == "truth" else np.full(p.d.shape, 50.0)
    r = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     settings=oracle.Settings(chain=chain), s_init=s0, max_sweeps=40000,
                     monitor_every=4, rtol=1e-12, full_residual=True)
    assert r.converged
    assert np.linalg.norm(r.s - sd) / np.linalg.norm(sd) < 1e-9
    # the warm start did change the path: its first residual differs from
    # the zero start's
    z = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                     settings=oracle.Settings(chain=chain), max_sweeps=4, monitor_every=4)
    assert r.trace[0][2] != z.trace[0][2]
