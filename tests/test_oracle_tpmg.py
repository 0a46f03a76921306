"""Pins of the oracle's TPMG pieces (paper Section 3, Algorithm 1; Section
4.1, eq. BlockJacobi; Section 5): the Thomas solve against exact and dense
solves, the smoother against dense block inverses, the transfers, the
tensor-product decoupling of the V-cycle (eq. EigenvalueEquation), the
V-cycle rate, and flexible CG against scipy's CG / PCG."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import mesh, operator as opm, tpmg

H = synth.H10KM


def _bands(rng, n, nz, scale_off, scale_e):
    l = rng.uniform(0.0, 1.0, (n, nz)) * scale_off
    m = rng.uniform(0.0, 1.0, (n, nz)) * scale_off
    # a column is one chain: couplings l_k and m_{k-1} are the same face
    l[:, 1:] = m[:, :-1]
    l[:, 0] = 0.0
    m[:, -1] = 0.0
    e = rng.uniform(0.1, 1.0, (n, nz)) * scale_e
    return l, m, e


def _dense(l, m, e):
    nz = len(e)
    a = np.diag(e + l + m)
    a -= np.diag(l[1:], -1)
    a -= np.diag(m[:-1], 1)
    return a


def test_thomas_vs_banded_lu():
    rng = np.random.default_rng(0)
    l, m, e = _bands(rng, 40, 17, 10.0, 1.0)
    b = rng.standard_normal((40, 17))
    x = tpmg.thomas_margin(l, m, e, b)
    for i in range(40):
        ab = np.zeros((3, 17))
        ab[0, 1:] = -m[i, :-1]
        ab[1] = e[i] + l[i] + m[i]
        ab[2, :-1] = -l[i, 1:]
        ref = sla.solve_banded((1, 1), ab, b[i])
        assert np.allclose(x[i], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def _exact_solve(l, m, e, b):
    """Gaussian elimination in exact rational arithmetic."""
    nz = len(b)
    F = [Fraction(float(v)) for v in e]
    L = [Fraction(float(v)) for v in l]
    M = [Fraction(float(v)) for v in m]
    B = [Fraction(float(v)) for v in b]
    diag = [F[k] + L[k] + M[k] for k in range(nz)]
    for k in range(1, nz):
        f = -L[k] / diag[k - 1]          # row_k -= f * row_{k-1}
        diag[k] -= f * (-M[k - 1])
        B[k] -= f * B[k - 1]
    x = [Fraction(0)] * nz
    x[-1] = B[-1] / diag[-1]
    for k in range(nz - 2, -1, -1):
        x[k] = (B[k] + M[k] * x[k + 1]) / diag[k]
    return np.array([float(v) for v in x])


@pytest.mark.parametrize("ratio", [1e2, 1e8, 1e14])
def test_thomas_extreme_anisotropy_exact(ratio):
    """Couplings up to 1e14 times the excess: the margin form stays accurate
    to a few ulps (checked against exact rational elimination)."""
    rng = np.random.default_rng(1)
    l, m, e = _bands(rng, 3, 8, ratio, 1.0)
    b = rng.standard_normal((3, 8))
    x = tpmg.thomas_margin(l, m, e, b)
    for i in range(3):
        ref = _exact_solve(l[i], m[i], e[i], b[i])
        assert np.max(np.abs(x[i] - ref)) <= 64 * np.finfo(float).eps * np.max(np.abs(ref))
    x32 = tpmg.thomas_margin(*(a.astype(np.float32) for a in (l, m, e, b)))
    for i in range(3):
        ref = _exact_solve(*(a[i].astype(np.float32).astype(np.float64) for a in (l, m, e, b)))
        assert np.max(np.abs(x32[i] - ref)) <= 4 * 8 * np.finfo(np.float32).eps * np.max(np.abs(ref))


def test_smoother_vs_dense_block_inverse():
    prof = synth.profiles_random(5, 80, seed=3)
    h = tpmg.build(1, synth.vertical_faces(5, H, "quadratic"), synth.omega_for(1) ** 2, profiles=prof)
    op = h.finest
    rng = np.random.default_rng(4)
    u = rng.standard_normal((op.n, op.nz))
    f = rng.standard_normal((op.n, op.nz))
    a = opm.to_sparse(op).toarray()
    nz = op.nz
    r = f.ravel() - a @ u.ravel()
    expect = u.ravel().copy()
    for t in range(op.n):
        sl = slice(t * nz, (t + 1) * nz)
        expect[sl] += h.omega * np.linalg.solve(a[sl, sl], r[sl])
    got = tpmg.smooth(op, f, u, h.omega)
    assert np.allclose(got.ravel(), expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())


def test_restriction_conserves():
    rng = np.random.default_rng(5)
    r = rng.standard_normal((320, 7))
    c = tpmg.restrict(r)
    assert c.shape == (80, 7)
    assert np.allclose(c.sum(axis=0), r.sum(axis=0), rtol=1e-14, atol=1e-13)
    assert np.array_equal(c[3], r[12] + r[13] + r[14] + r[15]) or np.allclose(c[3], r[12:16].sum(axis=0), rtol=1e-15)


def test_prolongation_linear_fields():
    ms = mesh.hierarchy(6)
    errs = []
    c = np.array([0.3, -0.7, 0.5])
    for ref in (3, 4, 5, 6):
        coarse, fine = ms[ref - 1], ms[ref]
        w = tpmg.prolongation_weights(coarse, fine)
        ec = (coarse.centre @ c)[:, None]
        ef = tpmg.prolong(ec, coarse.nbr, w)[:, 0]
        errs.append(np.max(np.abs(ef - fine.centre @ c)))
        # constants are reproduced exactly
        assert np.array_equal(tpmg.prolong(np.full((coarse.n, 2), 3.5), coarse.nbr, w), np.full((fine.n, 2), 3.5))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders) > 1.8, (errs, orders)


def test_prolongation_weights_vs_lstsq():
    ms = mesh.hierarchy(3)
    coarse, fine = ms[2], ms[3]
    w = tpmg.prolongation_weights(coarse, fine)
    for P in (0, 17, 123, 319):
        rp = coarse.centre[P]
        proj = np.eye(3) - np.outer(rp, rp)
        D = np.array([proj @ (coarse.centre[coarse.nbr[P, j]] - rp) for j in range(3)])
        # minimum-norm least squares in 3-D: solution lies in the tangent plane
        for i in range(4):
            delta = proj @ (fine.centre[4 * P + i] - rp)
            for j in range(3):
                rhs = np.zeros(3)
                rhs[j] = 1.0
                G = np.linalg.lstsq(D, rhs, rcond=None)[0]
                assert abs(G @ delta - w[4 * P + i, j]) < 1e-12


def _vcycle_matrix(h):
    op = h.finest
    n = op.n * op.nz
    a = opm.to_sparse(op)
    B = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        B[:, i] = tpmg.vcycle(h, e.reshape(op.n, op.nz)).ravel()
    return np.eye(n) - B @ a.toarray()


def test_tensor_decoupling_of_vcycle_spectrum():
    """Section 3.2.1: with factorising profiles and beta^S = alpha_r^S the
    3-D V-cycle error operator is similar to the direct sum over the radial
    eigenpairs (omega^2 A^r + B^r) e = lambda M^r e of 2-D V-cycles for
    omega^2 A^S + lambda M^S with point smoothing. Traces of its powers and
    its spectral radius must agree."""
    nz, ref = 5, 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=11, tie_beta_to_alpha_r=True)
    r = synth.vertical_faces(nz, H, "quadratic")
    om2 = synth.omega_for(ref) ** 2
    h3 = tpmg.build(ref, r, om2, profiles=prof)
    E3 = _vcycle_matrix(h3)
    v = opm.vertical(r)
    # radial matrices: A^r (stiffness from the face couplings), B^r, M^r
    ff = v.face_factor * prof.alpha_r_v
    Ar = np.zeros((nz, nz))
    for k in range(1, nz):
        Ar[k, k] += ff[k]; Ar[k - 1, k - 1] += ff[k]; Ar[k, k - 1] -= ff[k]; Ar[k - 1, k] -= ff[k]
    Br = np.diag(v.vk * prof.beta_v)
    Mr = np.diag(v.dr * prof.alpha_s_v)
    lam = sla.eigh(om2 * Ar + Br, Mr, eigvals_only=True)
    blocks = []
    for lj in lam:
        v2 = opm.Vertical(np.array([1.0, 2.0]), np.array([lj]), np.array([1.0]), np.zeros(2))
        prof2 = synth.Profiles(np.ones(2), np.ones(1), np.ones(1), prof.alpha_r_h, prof.alpha_s_h, prof.beta_h)
        h2 = tpmg.build(ref, None, om2, profiles=prof2, vert=v2)
        blocks.append(_vcycle_matrix(h2))
    for p in (1, 2, 3):
        t3 = np.trace(np.linalg.matrix_power(E3, p))
        t2 = sum(np.trace(np.linalg.matrix_power(b, p)) for b in blocks)
        assert math.isclose(t3, t2, rel_tol=1e-9, abs_tol=1e-9), (p, t3, t2)
    rho3 = np.max(np.abs(np.linalg.eigvals(E3)))
    rho2 = max(np.max(np.abs(np.linalg.eigvals(b))) for b in blocks)
    assert math.isclose(rho3, rho2, rel_tol=1e-7)


def test_vcycle_rate_bounded_in_h():
    rates = []
    for ref in (3, 4, 5):
        h = tpmg.build(ref, synth.vertical_faces(16, H, "quadratic"), synth.omega_for(ref) ** 2)
        rates.append(tpmg.richardson_rate(h))
    assert max(rates) < 0.4, rates
    assert rates[-1] - rates[-2] < 0.1, rates


def test_vcycle_rate_bounded_in_anisotropy():
    rates = []
    for ratio in (1e-1, 1e-2, 1e-3, 1e-4):
        th = ratio * synth.nominal_spacing(4)
        h = tpmg.build(4, synth.vertical_faces(32, th, "quadratic"), synth.omega_for(4) ** 2)
        rates.append(tpmg.richardson_rate(h))
    assert max(rates) < 0.35, rates


def _small_problem(seed=0):
    prof = synth.profiles_random(6, 320, seed=seed)
    h = tpmg.build(2, synth.vertical_faces(6, H, "quadratic"), synth.omega_for(2) ** 2, profiles=prof)
    f = synth.cell_integral(synth.uniform_noise(320, 6, seed + 1), h.meshes[-1].area, h.vert.vk)
    return h, f


def test_fcg_identity_preconditioner_is_cg():
    h, f = _small_problem(1)
    op = h.finest
    a = opm.to_sparse(op)
    ours = tpmg.fcg(lambda v: opm.apply(op, v), lambda r: r.copy(), f, rtol=1e-30, maxit=12)
    xs = []
    spla.cg(a, f.ravel(), x0=np.zeros(f.size), rtol=1e-30, atol=0.0, maxiter=12, callback=lambda xk: xs.append(xk.copy()))
    ref_hist = [np.linalg.norm(f.ravel() - a @ x) / np.linalg.norm(f) for x in xs]
    # the recursive residual of FCG follows CG's true residual
    for k in range(6):
        assert math.isclose(ours.history[k + 1], ref_hist[k], rel_tol=1e-6), (k, ours.history[k + 1], ref_hist[k])


def test_fcg_exact_preconditioner_one_step():
    h, f = _small_problem(2)
    op = h.finest
    lu = spla.splu(opm.to_sparse(op).tocsc())
    res = tpmg.fcg(lambda v: opm.apply(op, v), lambda r: lu.solve(r.ravel()).reshape(r.shape), f, rtol=1e-8)
    assert res.iters == 1 and res.status == "converged"


def test_fcg_symmetric_preconditioner_is_pcg():
    h, f = _small_problem(3)
    op = h.finest
    a = opm.to_sparse(op)
    d = a.diagonal()
    ours = tpmg.fcg(lambda v: opm.apply(op, v), lambda r: r / d.reshape(r.shape), f, rtol=1e-30, maxit=10)
    xs = []
    m = spla.LinearOperator(a.shape, matvec=lambda v: v / d)
    spla.cg(a, f.ravel(), x0=np.zeros(f.size), rtol=1e-30, atol=0.0, maxiter=10, M=m, callback=lambda xk: xs.append(xk.copy()))
    ref_hist = [np.linalg.norm(f.ravel() - a @ x) / np.linalg.norm(f) for x in xs]
    for k in range(6):
        assert math.isclose(ours.history[k + 1], ref_hist[k], rel_tol=1e-6)


def test_fcg_zero_rhs_and_breakdown():
    h, f = _small_problem(4)
    op = h.finest
    z = tpmg.solve(h, np.zeros_like(f))
    assert z.iters == 0 and z.status == "converged" and not np.any(z.x)
    bad = f.copy()
    bad[0, 0] = np.nan
    assert tpmg.solve(h, bad).status == "breakdown"


def test_mixed_precision_converges():
    h, f = _small_problem(5)
    x64 = tpmg.solve(h, f, rtol=1e-12)
    x32 = tpmg.solve(h, f, rtol=1e-8, precision="fp32")
    assert x32.status == "converged"
    assert np.linalg.norm(x32.x - x64.x) <= 1e-6 * np.linalg.norm(x64.x)


def _dense_vcycle(h, level):
    """The V-cycle of Algorithm 1 as a dense matrix B (z = B f), composed from
    explicit matrices and not from tpmg.vcycle. With W = omega D^-1 (D the
    block diagonal of the column matrices A_T, eq. BlockJacobi) one sweep is
    u <- S u + W f with S = I - W A, so nu sweeps from zero give
    G_nu = sum_{i<nu} S^i W. On the coarsest level B = G_nu_coarse; above it,
    pre-smoothing from zero, restriction R (sum over the four children) of
    the residual, the coarse V-cycle B_c from zero, prolongation P from the
    interpolation weights, then post-smoothing:
        B = S^nu_post (G_nu_pre + P B_c R (I - A G_nu_pre)) + G_nu_post."""
    op = h.ops[level]
    n, nz = op.n, op.nz
    N = n * nz
    a = opm.to_sparse(op).toarray()
    d = np.zeros_like(a)
    for t in range(n):
        sl = slice(t * nz, (t + 1) * nz)
        d[sl, sl] = a[sl, sl]
    W = h.omega * np.linalg.inv(d)
    S = np.eye(N) - W @ a

    def G(nu):
        out, Si = np.zeros((N, N)), np.eye(N)
        for _ in range(nu):
            out += Si @ W
            Si = S @ Si
        return out

    if level == 0:
        return G(h.nu_coarse)
    cop = h.ops[level - 1]
    nc = cop.n
    R = np.zeros((nc * nz, N))
    P = np.zeros((N, nc * nz))
    w = h.weights[level]
    for c in range(n):
        p = c // 4
        for k in range(nz):
            R[p * nz + k, c * nz + k] = 1.0
            P[c * nz + k, p * nz + k] += 1.0 - w[c].sum()
            for j in range(3):
                P[c * nz + k, cop.nbr[p, j] * nz + k] += w[c, j]
    bc = _dense_vcycle(h, level - 1)
    gpre = G(h.nu_pre)
    return np.linalg.matrix_power(S, h.nu_post) @ (gpre + P @ bc @ R @ (np.eye(N) - a @ gpre)) + G(h.nu_post)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_vcycle_schedule_dense_identity(levels):
    """Algorithm 1 with nu_pre = nu_post = 2 and one coarsest sweep from zero
    (Section 5), checked column by column against the composition of dense
    operators: a dropped or extra sweep, a non-zero coarse guess or a
    transposed transfer changes the matrix. A thick shell keeps the column
    matrices well conditioned, so the dense inverses are accurate to a few
    ulps."""
    nz, ref = 3, 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=31, tie_beta_to_alpha_r=False)
    h = tpmg.build(ref, synth.vertical_faces(nz, 0.3, "uniform"), synth.omega_for(ref) ** 2, profiles=prof,
                   n_levels=levels)
    op = h.finest
    n = op.n * op.nz
    want = _dense_vcycle(h, len(h.ops) - 1)
    got = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        got[:, i] = tpmg.vcycle(h, e.reshape(op.n, op.nz)).ravel()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_fp32_vcycle_is_a_float32_rounding_of_the_fp64_one():
    """make_preconditioner("fp32") is the V-cycle of Algorithm 1 (pinned in
    FP64 by test_vcycle_schedule_dense_identity) evaluated in float32: every
    coefficient array of its hierarchy is float32, and one V-cycle differs
    from the FP64 one by a float32 rounding: more than 1e3 FP64 epsilons
    (so float32 arithmetic is really used) and less than 100 float32
    epsilons. Changing the algorithm moves it by orders of magnitude more
    (one post-smoothing sweep fewer: 7e-2; damping 0.7 instead of 2/3:
    3e-2), so the bar separates rounding from a different computation."""
    import dataclasses

    h, f = _small_problem(5)
    h32 = h.astype(np.float32)
    for op in h32.ops:
        assert op.beta.dtype == np.float32 and op.alpha_r.dtype == np.float32 and op.alpha_s.dtype == np.float32
    z64 = tpmg.vcycle(h, f)
    z32 = tpmg.make_preconditioner(h, "fp32")(f)
    d = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e3 * np.finfo(np.float64).eps < d < 100 * np.finfo(np.float32).eps
    for changed in (dataclasses.replace(h, nu_post=1), dataclasses.replace(h, omega=0.7)):
        dc = np.linalg.norm(tpmg.vcycle(changed, f) - z64) / np.linalg.norm(z64)
        assert dc > 1e3 * 100 * np.finfo(np.float32).eps
