"""Pins of the oracle's multicolour block-SOR smoother (the paper's
implementation smoother, Section 5: block-SOR, here taken colour by colour
so that cells of one colour relax together; eq. BlockJacobi per cell):

  * the greedy colouring is proper and uses at most four colours (three on
    every icosahedral grid but refinement 1);
  * one sweep equals the dense block Gauss-Seidel / SOR formula in colour
    order, u + omega (D + omega L)^-1 (f - A u), D the column blocks and L
    the couplings to cells of earlier colours (later colours for the
    reverse sweep);
  * the V-cycle built on it equals the composition of dense operators of
    Algorithm 1 (SOR ascending before the coarse-grid correction,
    descending after, one ascending sweep from zero on the coarsest grid);
  * as a smoother it converges alone, and its V-cycle contracts (by 0.35
    at most on the cases below; faster than block-Jacobi on graded
    refinement-4 and -5 columns, slower on the uniform refinement-3 one).
"""
import numpy as np
import pytest

import synth
from oracle import mesh, operator as opm, tpmg


@pytest.mark.parametrize("ref", [0, 1, 2, 3, 4, 5])
def test_colouring_proper(ref):
    m = mesh.hierarchy(ref)[-1]
    col = tpmg.greedy_colouring(m.nbr)
    assert np.all(col[:, None] != col[m.nbr])
    assert col.max() + 1 == (4 if ref == 1 else 3)


def _sor_dense(op, colours, omega, reverse):
    a = opm.to_sparse(op).toarray()
    n, nz = op.n, op.nz
    cell = np.repeat(np.arange(n), nz)
    ci, cj = colours[cell][:, None], colours[cell][None, :]
    same = cell[:, None] == cell[None, :]
    earlier = (cj > ci) if reverse else (cj < ci)
    d = np.where(same, a, 0.0)
    low = np.where(earlier, a, 0.0)
    return a, d, low


@pytest.mark.parametrize("omega,reverse", [(1.0, False), (1.0, True), (1.3, False)])
def test_sor_sweep_equals_dense_formula(omega, reverse):
    nz, ref = 4, 1
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=51, tie_beta_to_alpha_r=False)
    h = tpmg.build(ref, synth.vertical_faces(nz, synth.H10KM, "quadratic"), synth.omega_for(ref) ** 2,
                   profiles=prof)
    op = h.finest
    col = tpmg.greedy_colouring(op.nbr)
    rng = np.random.default_rng(52)
    u = rng.standard_normal((op.n, nz))
    f = rng.standard_normal((op.n, nz))
    got = tpmg.smooth_sor(op, f, u, omega, col, reverse=reverse)
    a, d, low = _sor_dense(op, col, omega, reverse)
    want = u.ravel() + omega * np.linalg.solve(d + omega * low, f.ravel() - a @ u.ravel())
    assert np.max(np.abs(got.ravel() - want)) <= 1e-10 * np.max(np.abs(want))


def _dense_sor_vcycle(h, level):
    op = h.ops[level]
    n, nz = op.n, op.nz
    N = n * nz
    col = h.colours[level]
    a, d, low = _sor_dense(op, col, h.omega, False)
    _, _, up = _sor_dense(op, col, h.omega, True)
    Wf = h.omega * np.linalg.inv(d + h.omega * low)     # ascending sweep: u <- u + Wf (f - A u)
    Wb = h.omega * np.linalg.inv(d + h.omega * up)      # descending
    Sf, Sb = np.eye(N) - Wf @ a, np.eye(N) - Wb @ a

    def G(W, S, nu):
        out, Si = np.zeros((N, N)), np.eye(N)
        for _ in range(nu):
            out += Si @ W
            Si = S @ Si
        return out

    if level == 0:
        return G(Wf, Sf, h.nu_coarse)
    cop = h.ops[level - 1]
    R = np.zeros((cop.n * nz, N))
    P = np.zeros((N, cop.n * nz))
    w = h.weights[level]
    for c in range(n):
        p = c // 4
        for k in range(nz):
            R[p * nz + k, c * nz + k] = 1.0
            P[c * nz + k, p * nz + k] += 1.0 - w[c].sum()
            for j in range(3):
                P[c * nz + k, cop.nbr[p, j] * nz + k] += w[c, j]
    bc = _dense_sor_vcycle(h, level - 1)
    gpre = G(Wf, Sf, h.nu_pre)
    return np.linalg.matrix_power(Sb, h.nu_post) @ (gpre + P @ bc @ R @ (np.eye(N) - a @ gpre)) + G(Wb, Sb, h.nu_post)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_sor_vcycle_dense_identity(levels):
    nz, ref = 3, 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=53, tie_beta_to_alpha_r=False)
    h = tpmg.build(ref, synth.vertical_faces(nz, 0.3, "uniform"), synth.omega_for(ref) ** 2, profiles=prof,
                   n_levels=levels).with_sor()
    op = h.finest
    n = op.n * op.nz
    want = _dense_sor_vcycle(h, len(h.ops) - 1)
    got = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        got[:, i] = tpmg.vcycle(h, e.reshape(op.n, op.nz)).ravel()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("ref,nz,grading", [(3, 16, "uniform"), (4, 32, "quadratic")])
def test_sor_smoother_and_vcycle_rates(ref, nz, grading):
    r = synth.vertical_faces(nz, synth.H10KM, grading)
    h = tpmg.build(ref, r, synth.omega_for(ref) ** 2)
    hs = h.with_sor()
    rj = tpmg.richardson_rate(h, seed=7)
    rs = tpmg.richardson_rate(hs, seed=7)
    print(f"ref {ref} nz {nz}: V-cycle factor block-Jacobi {rj:.4f}, multicolour block-SOR {rs:.4f}")
    assert rs < 0.36 and rj < 0.3
    # the smoother alone reduces the residual (diagonally dominant blocks)
    op = h.finest
    u = np.random.default_rng(54).uniform(-1, 1, (op.n, nz))
    f = np.zeros_like(u)
    r0 = np.linalg.norm(opm.apply(op, u))
    for _ in range(3):
        u = tpmg.smooth_sor(op, f, u, 1.0, hs.colours[-1])
    assert np.linalg.norm(opm.apply(op, u)) < r0
