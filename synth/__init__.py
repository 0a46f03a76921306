"""Seeded synthetic inputs for the TPMG pressure-correction solve.

This module only draws random numbers and evaluates closed-form continuous
fields; it holds no step of the discretisation or of the solver. Both the CPU
oracle's tests and the GPU benchmark take their inputs from here, so the two
sides always see the same numbers.

Conventions (shared with the C ABI):
  * lengths are non-dimensionalised by the Earth radius, so the shell is
    r in [1, 1 + H/R] (Section 2.1 of the paper);
  * fields are stored cell-major, value (T, k) at T * nz + k, the column
    layout the paper describes for its finite-volume vectors (Section 4.1,
    Appendix A);
  * right-hand sides are cell integrals, as in Section 5 of the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

R_EARTH_M = 6371.0e3

# ---------------------------------------------------------------------------
# grid recipes
# ---------------------------------------------------------------------------


def n_cells(refinement: int) -> int:
    """Number of triangles of the icosahedral grid refined `refinement` times."""
    return 20 * 4 ** refinement


def nominal_spacing(refinement: int) -> float:
    """Nominal horizontal spacing h of a refined icosahedral grid (unit sphere).

    Centre-to-centre distance of an equilateral triangle whose area is the
    mean cell area 4*pi/n_T. Used to fix omega (Courant-number scaling of
    Section 2.1) and the anisotropy sweep without reading any mesh geometry.
    """
    a = 4.0 * math.pi / n_cells(refinement)
    return math.sqrt(4.0 * a / (3.0 * math.sqrt(3.0)))


def omega_for(refinement: int, courant: float = 8.0) -> float:
    """omega = C * h on the finest grid: horizontal acoustic Courant number C."""
    return courant * nominal_spacing(refinement)


def vertical_faces(nz: int, thickness: float, grading: str = "uniform") -> np.ndarray:
    """Radial faces 1 = r_0 < ... < r_nz = 1 + thickness (Appendix A).

    grading "uniform": zeta_k = k/nz; "quadratic": zeta_k = (k/nz)^2, finest
    at the surface.
    """
    k = np.arange(nz + 1, dtype=np.float64)
    if grading == "uniform":
        zeta = k / nz
    elif grading == "quadratic":
        zeta = (k / nz) ** 2
    else:
        raise ValueError(f"unknown grading {grading!r}")
    r = 1.0 + thickness * zeta
    r[0] = 1.0
    r[-1] = 1.0 + thickness
    return r


# ---------------------------------------------------------------------------
# profiles (factorised: alpha_r = a_r^r(r) a_r^S(x), ...)
# ---------------------------------------------------------------------------


@dataclass
class Profiles:
    """Factorised profile samples (eq. alphaxrfac in Section 3, Appendix A).

    Vertical factors: alpha_r_v at the nz+1 radial faces, alpha_s_v and beta_v
    at the nz layer midpoints. Horizontal factors: one value per finest-grid
    cell (alpha_r_h, alpha_s_h, beta_h); None means identically one.
    """

    alpha_r_v: np.ndarray
    alpha_s_v: np.ndarray
    beta_v: np.ndarray
    alpha_r_h: np.ndarray | None = None
    alpha_s_h: np.ndarray | None = None
    beta_h: np.ndarray | None = None


def profiles_unit(nz: int) -> Profiles:
    """alpha_r = alpha_S = beta = 1: exactly factorising, beta^S = alpha_r^S."""
    return Profiles(np.ones(nz + 1), np.ones(nz), np.ones(nz))


def profiles_random(nz: int, n_fine: int, seed: int, tie_beta_to_alpha_r: bool = True) -> Profiles:
    """Seeded positive factorised profiles, every factor drawn from U[0.5, 2].

    With tie_beta_to_alpha_r the horizontal factor of beta equals that of
    alpha_r (the assumption beta^S = alpha_r^S of Section 3.2.1).
    """
    rng = np.random.default_rng(seed)
    ar_v = rng.uniform(0.5, 2.0, nz + 1)
    as_v = rng.uniform(0.5, 2.0, nz)
    b_v = rng.uniform(0.5, 2.0, nz)
    ar_h = rng.uniform(0.5, 2.0, n_fine)
    as_h = rng.uniform(0.5, 2.0, n_fine)
    b_h = ar_h.copy() if tie_beta_to_alpha_r else rng.uniform(0.5, 2.0, n_fine)
    return Profiles(ar_v, as_v, b_v, ar_h, as_h, b_h)


# ---------------------------------------------------------------------------
# balanced zonal flow (Section 5.2): profiles that do not factorise
# ---------------------------------------------------------------------------

# physical constants of the balanced-flow profiles (SI units); g, c_p and R_d
# are not printed in the paper and take their usual values
GRAVITY = 9.81
C_P = 1005.0
R_DRY = 287.0
T_0 = 273.0
P_0 = 1.0e4
OMEGA_EARTH = 2.0 * np.pi / (24.0 * 3600.0)
JET_U0, JET_LAT, JET_SIGMA = 100.0, np.pi / 4.0, 0.1


def buoyancy_reference() -> float:
    """N* = g / sqrt(c_p T_0), the buoyancy frequency at which the balanced
    flow's profiles factorise exactly (0.01873 1/s)."""
    return GRAVITY / np.sqrt(C_P * T_0)


def jet_function(lat: np.ndarray) -> np.ndarray:
    """F(lat) with dF/dlat = 2 R Omega u(lat) sin(lat) + u(lat)^2 tan(lat),
    F(0) = 0, for the two-jet zonal wind u(lat) = u0 cos(lat)/cos(lat_M)
    exp(-(cos(lat) - cos(lat_M))^2 / (2 sigma^2)); integrated on a fine grid
    (composite Simpson, 20,001 points on [0, pi/2]) and interpolated. F is
    even in lat."""
    grid = np.linspace(0.0, np.pi / 2, 20001)
    c, sn = np.cos(grid), np.sin(grid)
    u = JET_U0 * c / np.cos(JET_LAT) * np.exp(-((c - np.cos(JET_LAT)) ** 2) / (2 * JET_SIGMA ** 2))
    # u^2 tan = u * (u / cos) * sin, finite at the pole (u ~ cos)
    u_over_c = JET_U0 / np.cos(JET_LAT) * np.exp(-((c - np.cos(JET_LAT)) ** 2) / (2 * JET_SIGMA ** 2))
    dF = 2.0 * R_EARTH_M * OMEGA_EARTH * u * sn + u * u_over_c * sn
    h = grid[1] - grid[0]
    F = np.zeros_like(grid)
    # Simpson on pairs of intervals, trapezoid for the odd point in between
    F[2::2] = np.cumsum(h / 3.0 * (dF[0:-2:2] + 4 * dF[1:-1:2] + dF[2::2]))
    F[1::2] = F[0:-1:2] + 0.5 * h * (dF[0:-1:2] + dF[1::2])
    return np.interp(np.abs(lat), grid, F)


@dataclass
class BalancedFlow:
    """Profiles of the balanced zonal flow with constant buoyancy frequency N
    (Section 5.2, eqs. BalancedFlow, JetFunction, VelocityField) and their
    approximate factorisation pi ~ pi^r(r) pi^S(lat) (eq. FacApproxBalancedFlow),
    sampled at the points the discretisation uses (Appendix A): alpha_r at the
    radial faces (r_k, centre), alpha_S and beta at the layer midpoints
    (r_{k+1/2}, centre). Background fields are scaled by T_0 and p_0/(R_d T_0):
    theta = 1/(E_h E_v), rho = pi^gamma E_h E_v, with E_h = exp(-N^2 F/g^2),
    E_v = exp(-N^2 R (r-1)/g), pi = (eps + E_h E_v)/(1 + eps),
    eps = (N/N*)^2 - 1; profiles (eq. profiles) alpha_S = rho theta,
    alpha_r = r^2 Lambda rho theta, beta = gamma rho/pi, xi_r = Lambda rho d_r theta
    (d_r in the radial unit, Earth radii), Lambda = 1/(1 + dt^2 N^2) with
    dt = omega R / c_h, c_h = sqrt(c_p T_0), gamma = (1 - kappa)/kappa,
    kappa = R_d/c_p."""

    alpha_r: np.ndarray        # [n, nz+1]
    alpha_s: np.ndarray        # [n, nz]
    beta: np.ndarray           # [n, nz]
    xi_r: np.ndarray           # [n, nz+1] (vertical advection, at the faces)
    factorised: Profiles       # the approximate factorisation's factors
    eps: float
    lam: float


def balanced_flow(eps: float, centres: np.ndarray, r_faces: np.ndarray, omega: float) -> BalancedFlow:
    r = np.asarray(r_faces, dtype=np.float64)
    rm = 0.5 * (r[:-1] + r[1:])
    lat, _ = _latlon(centres)
    n_star = buoyancy_reference()
    nb = n_star * np.sqrt(1.0 + eps)
    kappa = R_DRY / C_P
    gam = (1.0 - kappa) / kappa
    dt = omega * R_EARTH_M / np.sqrt(C_P * T_0)
    lam = 1.0 / (1.0 + (dt * nb) ** 2)
    e_h = np.exp(-(nb ** 2) / GRAVITY ** 2 * jet_function(lat))          # [n]

    def fields(rr):
        e_v = np.exp(-(nb ** 2) * R_EARTH_M / GRAVITY * (rr - 1.0))      # [m]
        eh, ev = e_h[:, None], e_v[None, :]
        pi = (eps + eh * ev) / (1.0 + eps)
        rho = pi ** gam * eh * ev
        theta = 1.0 / (eh * ev)
        # d_r theta = theta N^2 R / g (E_v' / E_v = -N^2 R / g)
        dtheta = theta * (nb ** 2) * R_EARTH_M / GRAVITY
        return pi, rho, theta, dtheta, e_v

    pi_m, rho_m, th_m, _, ev_m = fields(rm)
    pi_f, rho_f, th_f, dth_f, ev_f = fields(r)
    alpha_s = rho_m * th_m
    beta = gam * rho_m / pi_m
    alpha_r = (r ** 2)[None, :] * lam * rho_f * th_f
    xi_r = lam * rho_f * dth_f
    # factorisation: pi^x = pi^r(r) pi^S(lat), pi^r = (eps + E_v)/(1 + eps),
    # pi^S = E_h; the profiles of pi^x split into radial and horizontal factors
    pr_m = (eps + ev_m) / (1.0 + eps)
    pr_f = (eps + ev_f) / (1.0 + eps)
    fac = Profiles(alpha_r_v=r ** 2 * lam * pr_f ** gam, alpha_s_v=pr_m ** gam,
                   beta_v=gam * pr_m ** (gam - 1.0) * ev_m,
                   alpha_r_h=e_h ** gam, alpha_s_h=e_h ** gam, beta_h=e_h ** gam)
    return BalancedFlow(alpha_r, alpha_s, beta, xi_r, fac, eps, lam)


# ---------------------------------------------------------------------------
# right-hand sides
# ---------------------------------------------------------------------------


def uniform_noise(n: int, nz: int, seed: int) -> np.ndarray:
    """Seeded i.i.d. U[-1, 1] values, cell-major [n, nz]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, nz))


def cell_integral(point_values: np.ndarray, areas: np.ndarray, vk: np.ndarray) -> np.ndarray:
    """Cell integral |T| v_k * value (midpoint rule), cell-major [n, nz]."""
    return point_values * areas[:, None] * vk[None, :]


def _latlon(xyz: np.ndarray):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    lat = np.arctan2(z, np.hypot(x, y))
    lon = np.arctan2(y, x)
    return lat, lon


@dataclass
class Manufactured:
    """Closed-form u(r, x) = u_S(x) u_r(r) of the unit-profile operator
    L u = -omega^2 [ r^-2 d_r(r^2 d_r u) + r^-2 Lap_S u ] + u  (Appendix A).

    kind "config1": u = cos(lat) sin(2 lon) sin(pi (r-1)/H)  (not Neumann;
    cell_rhs carries its boundary fluxes);
    kind "smooth": u = 2xy cos(pi (r-1)/H)  (Neumann, degree-2 harmonic);
    kind "vertical": u = cos(pi (r-1)/H); kind "horizontal": u = 2xy.
    """

    kind: str
    thickness: float
    omega2: float

    # -- separable factors -------------------------------------------------
    def _us(self, xyz):
        x, y = xyz[:, 0], xyz[:, 1]
        if self.kind == "config1":
            lat, lon = _latlon(xyz)
            return np.cos(lat) * np.sin(2 * lon)
        if self.kind in ("smooth", "horizontal"):
            return 2.0 * x * y
        return np.ones(len(xyz))

    def _lap_us(self, xyz):
        if self.kind == "config1":
            lat, lon = _latlon(xyz)
            return -2.0 * np.cos(lat) * np.sin(2 * lon) - 3.0 * np.sin(2 * lon) / np.cos(lat)
        if self.kind in ("smooth", "horizontal"):
            return -6.0 * 2.0 * xyz[:, 0] * xyz[:, 1]
        return np.zeros(len(xyz))

    def _ur(self, r):
        s = math.pi / self.thickness
        if self.kind == "config1":
            return np.sin(s * (r - 1.0))
        if self.kind in ("smooth", "vertical"):
            return np.cos(s * (r - 1.0))
        return np.ones_like(r)

    def _dur(self, r):
        s = math.pi / self.thickness
        if self.kind == "config1":
            return s * np.cos(s * (r - 1.0))
        if self.kind in ("smooth", "vertical"):
            return -s * np.sin(s * (r - 1.0))
        return np.zeros_like(r)

    def _d2ur(self, r):
        s = math.pi / self.thickness
        return -s * s * self._ur(r) if self.kind != "horizontal" else np.zeros_like(r)

    # -- public ------------------------------------------------------------
    def u(self, xyz: np.ndarray, r: np.ndarray) -> np.ndarray:
        return self._us(xyz)[:, None] * self._ur(r)[None, :]

    def f(self, xyz: np.ndarray, r: np.ndarray) -> np.ndarray:
        us, lap = self._us(xyz)[:, None], self._lap_us(xyz)[:, None]
        ur, dur, d2ur = self._ur(r)[None, :], self._dur(r)[None, :], self._d2ur(r)[None, :]
        rr = r[None, :]
        radial = us * (d2ur + 2.0 * dur / rr)
        horiz = ur * lap / (rr * rr)
        return -self.omega2 * (radial + horiz) + us * ur

    def cell_rhs(self, xyz: np.ndarray, areas: np.ndarray, r_faces: np.ndarray) -> np.ndarray:
        """Cell integrals of L u over E = (T, k), as the discrete equations need them.

        Radial diffusion: the flux omega^2 |T| r^2 d_r u is taken exactly on
        every interior face and omitted on r_0 and r_nz, where the discrete
        operator imposes zero flux (a u that is not Neumann there moves its
        boundary flux onto the right-hand side this way). The remaining radial
        integrals use 3-point Gauss-Legendre; the horizontal integral is
        |T| times the value at the cell centre.
        """
        r = np.asarray(r_faces, dtype=np.float64)
        us, lap = self._us(xyz)[:, None], self._lap_us(xyz)[:, None]
        flux = r * r * self._dur(r)
        flux[0] = 0.0
        flux[-1] = 0.0
        radial = -self.omega2 * us * (flux[1:] - flux[:-1])[None, :]
        gx, gw = np.polynomial.legendre.leggauss(3)
        lo, hi = r[:-1], r[1:]
        half = 0.5 * (hi - lo)
        int_u = np.zeros_like(lo)        # integral of u_r dr
        int_r2u = np.zeros_like(lo)      # integral of r^2 u_r dr
        for x, wgt in zip(gx, gw):
            rr = 0.5 * (hi + lo) + half * x
            ur = self._ur(rr)
            int_u += wgt * half * ur
            int_r2u += wgt * half * rr * rr * ur
        horiz = -self.omega2 * lap * int_u[None, :]
        mass = us * int_r2u[None, :]
        return areas[:, None] * (radial + horiz + mass)


def smooth_random_field(xyz: np.ndarray, r: np.ndarray, thickness: float, seed: int, n_modes: int = 16) -> np.ndarray:
    """Sum of n_modes seeded low-order lat/lon/vertical Fourier modes,
    a_i cos(n_i lat + phi_i) cos(m_i lon + psi_i) cos(p_i pi (r-1)/H),
    with n, m, p in {0..3}, a ~ U[-1, 1] and phases ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    lat, lon = _latlon(xyz)
    out = np.zeros((len(xyz), len(r)))
    for _ in range(n_modes):
        a = rng.uniform(-1.0, 1.0)
        nn, mm, pp = rng.integers(0, 4, size=3)
        ph, ps = rng.uniform(0.0, 2 * math.pi, size=2)
        out += a * (np.cos(nn * lat + ph) * np.cos(mm * lon + ps))[:, None] * np.cos(
            pp * math.pi * (r - 1.0) / thickness
        )[None, :]
    return out


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    refinement: int
    nz: int
    grading: str
    thickness: float          # H / R
    omega2: float
    rhs: str                  # "config1", "manufactured_noise", "uniform", "smooth_sequence"
    seed: int = 0
    n_levels: int = 0         # 0: min(6, refinement + 1)
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return n_cells(self.refinement)

    @property
    def unknowns(self) -> int:
        return self.n * self.nz

    def levels(self) -> int:
        return self.n_levels or min(6, self.refinement + 1)

    def r_faces(self) -> np.ndarray:
        return vertical_faces(self.nz, self.thickness, self.grading)


H10KM = 10.0e3 / R_EARTH_M


def workload(name: str) -> Workload:
    """The solve configurations used by the tests and the benchmark."""
    if name == "ico3_nz16":      # 20,480 unknowns, manufactured solution
        return Workload(name, 3, 16, "uniform", H10KM, omega_for(3) ** 2, "config1", 0)
    if name == "ico6_nz128":     # 10,485,760 unknowns, manufactured + 10% noise
        return Workload(name, 6, 128, "quadratic", H10KM, omega_for(6) ** 2, "manufactured_noise", 2)
    if name.startswith("ico7_nz128_ar"):   # anisotropy sweep, H = ratio * h_7
        ratio = float(name.split("_ar")[1])
        return Workload(name, 7, 128, "quadratic", ratio * nominal_spacing(7), omega_for(7) ** 2, "uniform", 3)
    if name == "ico6_nz64_seq":  # learned-guess sequence
        return Workload(name, 6, 64, "quadratic", H10KM, omega_for(6) ** 2, "smooth_sequence", 50)
    m = name.split("_")
    if m[0] == "seq":            # seq_<ref>_<nz>: a smaller smooth sequence (seeds 50 and 51)
        ref, nz = int(m[1]), int(m[2])
        return Workload(name, ref, nz, "quadratic", H10KM, omega_for(ref) ** 2, "smooth_sequence", 50)
    if m[0] == "test":           # test_<ref>_<nz>_<grading>_<seed>
        ref, nz, grading, seed = int(m[1]), int(m[2]), m[3], int(m[4])
        return Workload(name, ref, nz, grading, H10KM, omega_for(ref) ** 2, "uniform", seed)
    raise KeyError(name)


def batch_list():
    """Sixteen solves of uneven size: (refinement, nz) = (4 + i mod 3, [32, 64, 128][(i div 3) mod 3])."""
    out = []
    for i in range(16):
        ref = 4 + i % 3
        nz = [32, 64, 128][(i // 3) % 3]
        out.append(Workload(f"batch{i}", ref, nz, "quadratic", H10KM, omega_for(ref) ** 2, "uniform", 40 + i))
    return out


def sequence_rhs(w: Workload, centres: np.ndarray, areas: np.ndarray, vk: np.ndarray, t) -> np.ndarray:
    """Right-hand side number t of a smooth sequence: the cell integral of
    f_0 + 0.05 t g, with f_0 and g smooth seeded fields (seeds w.seed and
    w.seed + 1) sampled at the cell centres and layer midpoints. t may be a
    scalar or a sequence (then the result is [len(t), n, nz])."""
    r = w.r_faces()
    r_mid = 0.5 * (r[:-1] + r[1:])
    f0 = smooth_random_field(centres, r_mid, w.thickness, w.seed)
    g = smooth_random_field(centres, r_mid, w.thickness, w.seed + 1)
    ts = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.stack([cell_integral(f0 + 0.05 * tt * g, areas, vk) for tt in ts])
    return out if np.ndim(t) else out[0]


def make_rhs(w: Workload, centres: np.ndarray, areas: np.ndarray, vk: np.ndarray) -> np.ndarray:
    """Cell-integral right-hand side [n, nz] for workload w.

    centres, areas: the finest-grid cell centres and areas; vk: the radial
    cell volume factors v_k. These come from whichever side builds the mesh.
    """
    r_faces = w.r_faces()
    if w.rhs == "config1":
        return Manufactured("config1", w.thickness, w.omega2).cell_rhs(centres, areas, r_faces)
    if w.rhs == "manufactured_noise":
        fm = Manufactured("config1", w.thickness, w.omega2).cell_rhs(centres, areas, r_faces)
        vol = areas[:, None] * vk[None, :]
        rms = float(np.sqrt(np.mean((fm / vol) ** 2)))
        return fm + 0.1 * rms * uniform_noise(len(areas), w.nz, w.seed) * vol
    if w.rhs == "uniform":
        return cell_integral(uniform_noise(len(areas), w.nz, w.seed), areas, vk)
    if w.rhs == "smooth_sequence":
        return sequence_rhs(w, centres, areas, vk, 1)
    raise ValueError(w.rhs)
