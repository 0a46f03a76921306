"""Pins of the oracle's vertical advection (the xi_r term of the operator,
Section 2.1 eq. HelmholtzVector; Appendix A "Vertical advection") and of the
paper's two outer solvers (Section 5.2: preconditioned Richardson and
BiCGStab):

  * xi_r = 0 gives the operator without advection; the flux form keeps
    A 1 = beta^; the skew part of A is the advection alone;
  * the advection stencil applied to u = r is the cell integral of
    r^2 xi d_r r to second order in the layer thickness;
  * the non-symmetric column solve (margin form with different couplings
    below and above) equals a banded LU solve;
  * BiCGStab and Richardson: one iteration with the exact preconditioner,
    the direct solution with the identity preconditioner (BiCGStab), and
    TPMG-preconditioned convergence on the advective balanced flow.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import mesh, operator as opm, tpmg

H = synth.H10KM


def _bf(eps=0.5, ref=2, nz=8, om_ref=None):
    r = synth.vertical_faces(nz, H, "quadratic")
    om = synth.omega_for(om_ref or ref)
    m = mesh.hierarchy(ref)[-1]
    return r, om, synth.balanced_flow(eps, m.centre, r, om)


def test_zero_advection_and_row_sums():
    r, om, bf = _bf()
    zero = opm.FullProfiles(bf.alpha_r, bf.alpha_s, bf.beta, np.zeros_like(bf.xi_r))
    a0 = tpmg.build(2, r, om * om, profiles=bf.factorised, full=bf).finest
    az = tpmg.build(2, r, om * om, profiles=bf.factorised, full=zero, full_terms=tpmg.FULL_TERMS_ADV).finest
    u = np.random.default_rng(71).standard_normal((a0.n, a0.nz))
    assert np.array_equal(opm.apply(a0, u), opm.apply(az, u))
    aa = tpmg.build(2, r, om * om, profiles=bf.factorised, full=bf, full_terms=tpmg.FULL_TERMS_ADV).finest
    assert np.allclose(opm.apply(aa, np.ones((aa.n, aa.nz))), aa.beta, rtol=1e-13, atol=0)
    A = opm.to_sparse(aa).toarray()
    S = opm.to_sparse(a0).toarray()
    skew = A - A.T
    assert np.max(np.abs(skew)) > 0
    # the skew part is the advection's: (A - A^T) = (A - S) - (A - S)^T
    D = A - S
    assert np.allclose(skew, D - D.T, rtol=0, atol=1e-15 * np.max(np.abs(A)))
    # advection is small next to the vertical diffusion (an M-matrix still)
    l, m, e = opm.column_bands(aa)
    assert np.all(l[:, 1:] > 0) and np.all(m[:, :-1] > 0)


def test_advection_stencil_second_order():
    """u = r at the cell centres, xi = 1, no diffusion or mass: the stencil
    gives -omega^2 times |T| (r_{k+1}-r_k)(r_k^2 + r_{k+1}^2)/2 on interior
    cells, the cell integral |T| v_k of r^2 d_r r up to O(dr^2)."""
    errs = []
    for nz in (8, 16, 32, 64):
        r = synth.vertical_faces(nz, 0.05, "uniform")
        vert = opm.vertical(r)
        m = mesh.hierarchy(1)[-1]
        z = np.zeros((m.n, nz))
        op = opm.assemble_full(m, vert, 1.0, np.zeros((m.n, nz + 1)), z, z, np.ones((m.n, nz + 1)))
        rc = 0.5 * (r[:-1] + r[1:])
        y = opm.apply(op, np.tile(rc, (m.n, 1)))
        exact = -m.area[:, None] * vert.vk[None, :]
        inner = slice(1, nz - 1)
        errs.append(np.max(np.abs(y[:, inner] / exact[:, inner] - 1)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders) > 1.9, (errs, orders)


def test_nonsymmetric_thomas_vs_banded():
    rng = np.random.default_rng(72)
    n, nz = 50, 17
    l = rng.uniform(0.1, 5.0, (n, nz))
    m = rng.uniform(0.1, 5.0, (n, nz))
    l[:, 0] = 0
    m[:, -1] = 0
    e = rng.uniform(0.01, 1.0, (n, nz))
    b = rng.standard_normal((n, nz))
    x = tpmg.thomas_margin(l, m, e, b)
    for t in range(n):
        ab = np.zeros((3, nz))
        ab[0, 1:] = -m[t, :-1]
        ab[1] = e[t] + l[t] + m[t]
        ab[2, :-1] = -l[t, 1:]
        xr = sla.solve_banded((1, 1), ab, b[t])
        assert np.allclose(x[t], xr, rtol=1e-12, atol=1e-14 * np.max(np.abs(xr)))


def test_outer_solvers_exact_and_identity_preconditioners():
    r, om, bf = _bf(eps=1.0, ref=1, nz=6, om_ref=3)
    op = tpmg.build(1, r, om * om, profiles=bf.factorised, full=bf, full_terms=tpmg.FULL_TERMS_ADV).finest
    A = opm.to_sparse(op).tocsc()
    f = synth.cell_integral(synth.uniform_noise(op.n, op.nz, 73), mesh.hierarchy(1)[-1].area, opm.vertical(r).vk)
    xd = spla.spsolve(A, f.ravel()).reshape(f.shape)
    app = lambda v: opm.apply(op, v)
    exact = lambda v: spla.spsolve(A, v.ravel()).reshape(v.shape)
    for solver in (tpmg.bicgstab, tpmg.richardson):
        res = solver(app, exact, f, rtol=1e-10, maxit=5)
        assert res.status == "converged" and res.iters == 1
        assert np.linalg.norm(res.x - xd) <= 1e-10 * np.linalg.norm(xd)
    res = tpmg.bicgstab(app, lambda v: v, f, rtol=1e-12, maxit=2000)
    assert res.status == "converged"
    assert np.linalg.norm(res.x - xd) <= 1e-6 * np.linalg.norm(xd)
    # scipy's BiCGStab reaches the same solution
    xs, info = spla.bicgstab(A, f.ravel(), rtol=1e-12, maxiter=2000)
    assert info == 0 and np.linalg.norm(xs.reshape(f.shape) - xd) <= 1e-6 * np.linalg.norm(xd)


@pytest.mark.parametrize("eps", [0.0, 1.23])
def test_tpmg_outer_solvers_on_advective_balanced_flow(eps):
    """TPMG^(full) with advection preconditions Richardson and BiCGStab to
    1e-8 on the balanced flow (refinement 3 x 16 levels); BiCGStab takes at
    most about half Richardson's iterations (two V-cycles per iteration),
    both solutions equal the direct solve to the tolerance."""
    r, om, bf = _bf(eps=eps, ref=3, nz=16)
    h = tpmg.build(3, r, om * om, profiles=bf.factorised, full=bf, full_terms=tpmg.FULL_TERMS_ADV)
    f = synth.cell_integral(synth.uniform_noise(h.finest.n, 16, 74), h.meshes[-1].area, h.vert.vk)
    xd = tpmg.direct_solve(h.finest, f)
    rr = tpmg.solve(h, f, rtol=1e-8, maxit=200, method="richardson")
    rb = tpmg.solve(h, f, rtol=1e-8, maxit=200, method="bicgstab")
    print(f"eps {eps}: Richardson {rr.iters}, BiCGStab {rb.iters} iterations")
    assert rr.status == "converged" and rb.status == "converged"
    assert rb.iters <= rr.iters // 2 + 1
    for res in (rr, rb):
        assert np.linalg.norm(res.x - xd) <= 1e-5 * np.linalg.norm(xd)
