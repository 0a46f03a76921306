"""Pins of the oracle's operators for profiles that do not factorise
(Section 4.2: TPMG^(full), TPMG^(partial) and TPMG^(x); Appendix A, eq.
hatFunctionsNonFac; Section 3.2.2, eq. RichardsonConvergenceRate):

  * full-profile assembly given factorising samples equals the (separately
    pinned) factorised assembly on every level, coarse grids included;
  * symmetry, definiteness, row sums and coarse-grid conservation for
    random non-factorising profiles;
  * the balanced flow of Section 5.2 factorises exactly at eps = 0 (then
    TPMG^(full) = TPMG^(x)) and not for eps > 0;
  * the perturbation bound of Section 3.2.2: with A = A^x + dA and
    Delta = ||(A^x)^-1 dA||, Richardson for A preconditioned by mu V-cycles
    of A^x contracts by at most Delta + (1 + Delta) rho_x^mu (norms of the
    A^x energy inner product, computed densely on a small grid).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import mesh, operator as opm, tpmg

H = synth.H10KM


def _full_from_factors(prof, n, nz):
    ar = (np.ones(n) if prof.alpha_r_h is None else prof.alpha_r_h)[:, None] * prof.alpha_r_v[None, :]
    as_ = (np.ones(n) if prof.alpha_s_h is None else prof.alpha_s_h)[:, None] * prof.alpha_s_v[None, :]
    b = (np.ones(n) if prof.beta_h is None else prof.beta_h)[:, None] * prof.beta_v[None, :]
    return opm.FullProfiles(ar, as_, b)


def _random_full(n, nz, seed):
    rng = np.random.default_rng(seed)
    return opm.FullProfiles(rng.uniform(0.5, 2.0, (n, nz + 1)), rng.uniform(0.5, 2.0, (n, nz)),
                            rng.uniform(0.5, 2.0, (n, nz)))


@pytest.mark.parametrize("terms", [tpmg.FULL_TERMS, ("alpha_r",), ("beta", "alpha_s")])
def test_full_assembly_of_factorising_samples_equals_factorised(terms):
    nz, ref = 7, 3
    r = synth.vertical_faces(nz, H, "quadratic")
    om2 = synth.omega_for(ref) ** 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=31, tie_beta_to_alpha_r=False)
    h0 = tpmg.build(ref, r, om2, profiles=prof)
    h1 = tpmg.build(ref, r, om2, profiles=prof, full=_full_from_factors(prof, synth.n_cells(ref), nz),
                    full_terms=terms)
    assert len(h0.ops) == len(h1.ops) == 4
    for a, b in zip(h0.ops, h1.ops):
        for name in ("beta", "alpha_s", "alpha_r"):
            x, y = getattr(a, name), getattr(b, name)
            assert np.allclose(x, y, rtol=1e-13, atol=0.0), name


def test_full_operator_structure():
    nz, ref = 5, 1
    r = synth.vertical_faces(nz, H, "quadratic")
    full = _random_full(synth.n_cells(ref), nz, 32)
    h = tpmg.build(ref, r, synth.omega_for(ref) ** 2, profiles=synth.profiles_unit(nz), full=full)
    a = opm.to_sparse(h.finest)
    assert abs(a - a.T).max() == 0.0
    assert np.linalg.eigvalsh(a.toarray()).min() > 0
    op = h.finest
    assert np.array_equal(opm.apply(op, np.ones((op.n, nz))), op.beta)
    # every coefficient really varies within a column and across columns
    for name in ("beta", "alpha_r"):
        v = getattr(op, name)[:, 1:-1] if name == "alpha_r" else getattr(op, name)
        ratio = v / v.mean(axis=0, keepdims=True)
        assert np.std(ratio / ratio.mean(axis=1, keepdims=True)) > 0.05


def test_full_coarse_coefficients_conserve_children():
    """Cell-integral coefficients (mass, vertical couplings) of a coarse cell
    equal the sums of its four children's, level by level (the coarse
    profile is the area-weighted mean of the children's)."""
    nz, ref = 4, 3
    r = synth.vertical_faces(nz, H, "quadratic")
    full = _random_full(synth.n_cells(ref), nz, 33)
    h = tpmg.build(ref, r, synth.omega_for(ref) ** 2, profiles=synth.profiles_unit(nz), full=full, n_levels=4)
    for lvl in range(1, len(h.ops)):
        fine, coarse = h.ops[lvl], h.ops[lvl - 1]
        for name in ("beta", "alpha_r"):
            child_sum = getattr(fine, name).reshape(coarse.n, 4, -1).sum(axis=1)
            assert np.allclose(getattr(coarse, name), child_sum, rtol=1e-13, atol=0.0), (lvl, name)


def test_balanced_flow_factorises_only_at_eps_zero():
    ref, nz = 3, 8
    m = mesh.hierarchy(ref)[-1]
    r = synth.vertical_faces(nz, H, "quadratic")
    om = synth.omega_for(ref)
    for eps, exact in ((0.0, True), (0.5, False), (1.23, False)):
        bf = synth.balanced_flow(eps, m.centre, r, om)
        h_full = tpmg.build(ref, r, om * om, profiles=bf.factorised, full=bf)
        h_fac = tpmg.build(ref, r, om * om, profiles=bf.factorised)
        d = 0.0
        for a, b in zip(h_full.ops, h_fac.ops):
            for k in ("beta", "alpha_s", "alpha_r"):
                x, y = getattr(a, k), getattr(b, k)
                nz_ = y != 0
                assert np.array_equal(x == 0, ~nz_)
                d = max(d, float(np.max(np.abs(x[nz_] / y[nz_] - 1))))
        if exact:
            assert d <= 1e-13
        else:
            assert d > 0.05


def _dense_vcycle(h):
    n = h.finest.n * h.finest.nz
    cols = [tpmg.vcycle(h, e.reshape(h.finest.n, h.finest.nz)).ravel() for e in np.eye(n)]
    return np.array(cols).T


@pytest.mark.parametrize("eps", [0.5, 1.23])
def test_perturbation_bound_richardson(eps):
    """Section 3.2.2: ||I - M_mu A||_{A^x} <= Delta + (1 + Delta) rho_x^mu
    with rho_x = ||I - M A^x||_{A^x}, Delta = ||(A^x)^-1 (A - A^x)||_{A^x},
    M_mu = mu Richardson steps of the V-cycle of A^x (as a linear map), on
    the balanced flow at refinement 1 x 4 levels (320 unknowns); and the
    Richardson rate the oracle measures for A preconditioned by TPMG^(x) is
    below the bound for mu = 1."""
    ref, nz = 1, 4
    m = mesh.hierarchy(ref)[-1]
    r = synth.vertical_faces(nz, H, "quadratic")
    om = synth.omega_for(3)
    bf = synth.balanced_flow(eps, m.centre, r, om)
    h_fac = tpmg.build(ref, r, om * om, profiles=bf.factorised)
    a = opm.to_sparse(tpmg.build(ref, r, om * om, profiles=bf.factorised, full=bf).finest).toarray()
    af = opm.to_sparse(h_fac.finest).toarray()
    lf = np.linalg.cholesky(af)                         # A^x = L L^T: ||X||_{A^x} = ||L^T X L^-T||_2

    def enorm(x):
        return float(np.linalg.norm(lf.T @ x @ np.linalg.inv(lf.T), 2))

    mv = _dense_vcycle(h_fac)
    n = a.shape[0]
    eye = np.eye(n)
    delta = enorm(np.linalg.solve(af, a - af))
    rho_x = enorm(eye - mv @ af)
    assert delta < 1.0 and rho_x < 1.0
    e_fac = eye - mv @ af
    for mu in (1, 2, 3):
        m_mu = (eye - np.linalg.matrix_power(e_fac, mu)) @ np.linalg.inv(af)
        lhs = enorm(eye - m_mu @ a)
        bound = delta + (1 + delta) * rho_x ** mu
        print(f"eps {eps} mu {mu}: ||I - M_mu A|| = {lhs:.4f} <= {bound:.4f} (Delta {delta:.4f}, rho_x {rho_x:.4f})")
        assert lhs <= bound * (1 + 1e-12)
    # the oracle's measured Richardson factor for A with TPMG^(x) (mu = 1)
    # over cycles 60..100 (late enough for the dominant pair of eigenvalues
    # to take over): the spectral radius of I - M A, at most its norm
    outer = tpmg.build(ref, r, om * om, profiles=bf.factorised, full=bf).finest
    rate = tpmg.richardson_rate(h_fac, seed=7, cycles=100, skip=60, outer=outer)
    srad = max(abs(np.linalg.eigvals(eye - mv @ a)))
    print(f"eps {eps}: measured Richardson factor {rate:.4f}, spectral radius {srad:.4f}")
    assert rate <= delta + (1 + delta) * rho_x + 1e-12
    assert abs(rate - srad) <= 1e-6 * srad
