"""Pins of the oracle's finite-volume operator (paper Appendix A, eqs.
hatFunctionsNonFac / hatFunctionsFac, eq. ColumnEquation): symmetry and
definiteness, matrix-free apply vs explicit matrix, closed-form coefficient
sums, the energy identity, and second-order convergence of manufactured
solutions."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import mesh, operator as opm, tpmg

H = synth.H10KM
OM2 = synth.omega_for(3) ** 2


def _hier(ref, nz, grading="uniform", profiles=None, levels=0, thickness=H, om2=OM2):
    return tpmg.build(ref, synth.vertical_faces(nz, thickness, grading), om2, profiles=profiles, n_levels=levels)


@pytest.mark.parametrize("grading", ["uniform", "quadratic"])
def test_symmetric_positive_definite(grading):
    prof = synth.profiles_random(6, 80, seed=1, tie_beta_to_alpha_r=False)
    h = _hier(1, 6, grading, prof)
    a = opm.to_sparse(h.finest)
    assert abs(a - a.T).max() == 0.0
    ev = np.linalg.eigvalsh(a.toarray())
    assert ev.min() > 0
    # Gershgorin with the margin: every row strictly diagonally dominant
    d = a.diagonal()
    off = np.asarray(abs(a).sum(axis=1)).ravel() - d
    assert np.all(d > off)


def test_apply_matches_sparse_and_row_sums():
    prof = synth.profiles_random(9, 320, seed=2)
    h = _hier(2, 9, "quadratic", prof)
    op = h.finest
    u = np.random.default_rng(3).standard_normal((op.n, op.nz))
    a = opm.to_sparse(op)
    y1 = opm.apply(op, u)
    y2 = (a @ u.ravel()).reshape(u.shape)
    assert np.allclose(y1, y2, rtol=1e-12, atol=1e-12 * np.abs(y2).max())
    ones = (a @ np.ones(op.n * op.nz)).reshape(op.n, op.nz)
    # the explicit row sum cancels the large diagonal; exact up to its rounding
    diag = a.diagonal().reshape(op.n, op.nz)
    assert np.all(np.abs(ones - op.beta) <= 1e-14 * diag)
    assert np.array_equal(opm.apply(op, np.ones((op.n, op.nz))), op.beta)


def test_energy_identity():
    """u.Au = sum beta u^2 + 1/2 sum_edges alphaS (du)^2 + sum_faces alphar (du)^2."""
    prof = synth.profiles_random(7, 320, seed=4)
    op = _hier(2, 7, "uniform", prof).finest
    u = np.random.default_rng(5).standard_normal((op.n, op.nz))
    lhs = float(np.sum(u * opm.apply(op, u)))
    e_mass = float(np.sum(op.beta * u * u))
    e_h = 0.5 * sum(float(np.sum(op.alpha_s[:, j, :] * (u - u[op.nbr[:, j]]) ** 2)) for j in range(3))
    e_v = float(np.sum(op.alpha_r[:, 1:-1] * (u[:, 1:] - u[:, :-1]) ** 2))
    assert math.isclose(lhs, e_mass + e_h + e_v, rel_tol=1e-12)


def test_closed_form_coefficient_sums():
    """Unit profiles: sum beta^ = shell volume; vertical couplings of a
    uniform grid are omega^2 |T| r_k^2 / dr; horizontal = omega^2 dr g."""
    nz, thick = 5, 0.01
    h = _hier(2, nz, "uniform", thickness=thick)
    op, m = h.finest, h.meshes[-1]
    vol = 4 * math.pi * ((1 + thick) ** 3 - 1) / 3
    assert math.isclose(op.beta.sum(), vol, rel_tol=1e-13)
    dr = thick / nz
    r = 1 + dr * np.arange(nz + 1)
    expect = OM2 * m.area[:, None] * (r[1:-1] ** 2 / dr)[None, :]
    assert np.allclose(op.alpha_r[:, 1:-1], expect, rtol=1e-10)
    assert np.all(op.alpha_r[:, 0] == 0) and np.all(op.alpha_r[:, -1] == 0)
    assert np.allclose(op.alpha_s, OM2 * dr * m.g[:, :, None], rtol=1e-10)


def _mms_error(kind, ref, nz, grading):
    h = _hier(ref, nz, grading, levels=min(ref + 1, 5))
    m = h.meshes[-1]
    man = synth.Manufactured(kind, H, OM2)
    r = h.vert.r
    f = man.cell_rhs(m.centre, m.area, r)
    res = tpmg.solve(h, f, rtol=1e-12, maxit=200)
    assert res.status == "converged"
    ue = man.u(m.centre, 0.5 * (r[1:] + r[:-1]))
    vol = m.area[:, None] * h.vert.vk[None, :]
    return math.sqrt(np.sum(vol * (res.x - ue) ** 2) / np.sum(vol * ue ** 2))


def _orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("grading", ["uniform", "quadratic"])
def test_manufactured_vertical_second_order(grading):
    errs = [_mms_error("vertical", 1, nz, grading) for nz in (8, 16, 32, 64)]
    assert min(_orders(errs)) >= 1.9, errs


def test_manufactured_horizontal_second_order():
    errs = [_mms_error("horizontal", ref, 2, "uniform") for ref in (2, 3, 4, 5)]
    assert min(_orders(errs)) >= 1.9, errs


@pytest.mark.slow
def test_manufactured_joint():
    smooth = [_mms_error("smooth", ref, nz, "uniform") for ref, nz in ((2, 8), (3, 16), (4, 32))]
    assert min(_orders(smooth)) >= 1.9, smooth
    # the config-1 field cos(lat) sin(2 lon) is only Lipschitz at the poles
    cfg = [_mms_error("config1", ref, nz, "uniform") for ref, nz in ((2, 8), (3, 16), (4, 32))]
    assert min(_orders(cfg)) >= 1.8, cfg


def test_solve_equals_direct():
    prof = synth.profiles_random(12, 1280, seed=6)
    h = _hier(3, 12, "quadratic", prof)
    f = synth.cell_integral(synth.uniform_noise(1280, 12, 8), h.meshes[-1].area, h.vert.vk)
    res = tpmg.solve(h, f, rtol=1e-13, maxit=200)
    ud = tpmg.direct_solve(h.finest, f)
    assert res.status == "converged"
    assert np.linalg.norm(res.x - ud) <= 1e-9 * np.linalg.norm(ud)


def test_coarse_coefficients_conserve_children():
    """Coarse grids (rediscretised with the horizontal profile factors of the
    four children combined): the children of a coarse cell tile it exactly
    (Section 4.1: each coarse triangle is four fine ones), so the coarse mass
    and vertical-coupling coefficients, which are cell integrals |T| x
    profile, must equal the sums of their four children's. An unweighted
    mean of the children's factors fails this on the icosahedral grid, whose
    children differ in area."""
    nz = 4
    prof = synth.profiles_random(nz, 1280, seed=21, tie_beta_to_alpha_r=False)
    h = _hier(3, nz, "quadratic", prof, levels=4)
    for lvl in range(1, len(h.ops)):
        fine, coarse = h.ops[lvl], h.ops[lvl - 1]
        for name in ("beta", "alpha_r"):
            child_sum = getattr(fine, name).reshape(coarse.n, 4, -1).sum(axis=1)
            parent = getattr(coarse, name)
            assert np.allclose(parent, child_sum, rtol=1e-13, atol=0.0), (lvl, name)
    # the children really differ in area, so the weighting matters
    a = h.meshes[-1].area.reshape(-1, 4)
    assert np.max(np.abs(a - a.mean(axis=1, keepdims=True))) > 1e-3 * a.mean()
    # and an unweighted mean is caught
    ar_h = prof.alpha_r_h.reshape(-1, 4)
    plain = ar_h.mean(axis=1) * h.meshes[-2].area
    weighted = (ar_h * h.meshes[-1].area.reshape(-1, 4)).sum(axis=1)
    assert not np.allclose(plain, weighted, rtol=1e-6)


def test_caller_samples_on_coarse_grids():
    """Horizontal factors sampled by the caller on a coarse grid (the
    coarse operator is rediscretised on each grid, Section 3.2.1): giving
    every grid exactly the area means of its children reproduces the default
    hierarchy bit for bit; a sample given on refinement 2 makes that grid's
    coefficients the cell integrals |T| x sample (mass: beta^S_T = |T|
    beta_T, as in Appendix A) and refinement 1 their children's sums (the
    conservation of the default hierarchy, now of the given samples), while
    the finest grid is unchanged."""
    nz = 4
    r = synth.vertical_faces(nz, H, "quadratic")
    prof = synth.profiles_random(nz, 1280, seed=23, tie_beta_to_alpha_r=False)
    h0 = tpmg.build(3, r, OM2, profiles=prof, n_levels=4)
    means = {3: (prof.alpha_r_h, prof.alpha_s_h, prof.beta_h)}
    for ref in (3, 2, 1):
        means[ref - 1] = tuple(opm.restrict_cell_factor(np.asarray(x), h0.meshes[ref].area) for x in means[ref])
    h1 = tpmg.build(3, r, OM2, profiles=prof, n_levels=4, level_factors=means)
    for a, b in zip(h0.ops, h1.ops):
        for name in ("beta", "alpha_r", "alpha_s"):
            assert np.array_equal(getattr(a, name), getattr(b, name)), name
    rng = np.random.default_rng(24)
    sample = rng.uniform(0.5, 2.0, 320)
    h2 = tpmg.build(3, r, OM2, profiles=prof, n_levels=4, level_factors={2: (None, None, sample)})
    m2 = h2.meshes[2]
    assert np.allclose(h2.ops[2].beta, m2.area[:, None] * h2.vert.vk[None, :] * sample[:, None] *
                       np.asarray(prof.beta_v)[None, :], rtol=1e-14, atol=0)
    child_sum = h2.ops[2].beta.reshape(80, 4, nz).sum(axis=1)
    assert np.allclose(h2.ops[1].beta, child_sum, rtol=1e-13, atol=0)
    assert np.array_equal(h2.ops[3].beta, h0.ops[3].beta)
    assert np.array_equal(h2.ops[2].alpha_r, h0.ops[2].alpha_r)
    assert not np.allclose(h2.ops[2].beta, h0.ops[2].beta)
