"""Oracle: the HEVI split-explicit large step of the THOR dynamical core.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The step follows Sec. 3 (flux-form deep non-hydrostatic Euler equations,
Eqs. mass / mom / entropy, equation of state Eq. pressure, 3D operator split
with Eqs. proj_h / proj_r, Wicker-Skamarock RK3 for the slow terms,
forward-backward acoustic substeps in perturbation form, Eqs. dens2 / mom2 /
momr2 / pt2 / theta_to_p, HEVI vertical momentum solved per column with the
Thomas algorithm and a rigid lid), Sec. 4 (fourth-order hyperdiffusion
Eqs. diff_rho ... diff_p, 3D divergence damping every short step, Eqs. kd /
tau_d) and Sec. 5 (backward-Euler Newtonian relaxation, Eq. im_eq_t).

Readings taken where the paper is silent or garbled (also in the design
notes):
  * the three "large time steps" of the inner-loop schedule are the three
    RK stages: (1 substep of dt/3), (n/2 of dt/n), (n of dt/n);
  * every stage restarts the small-step state from Phi[t]; deviations are
    taken from Phi[t]; advection, Coriolis and the linearisation
    coefficients (theta, gamma p / rho theta) use the previous stage state;
    hyperdiffusion, grad p[t] and the [t] vertical imbalance use Phi[t];
  * the vertical-momentum equation is the tridiagonal that follows from
    inserting the discrete density and rho-theta updates (linearised
    pressure, p = EOS(rho theta)) into the discrete vertical momentum
    equation; this is the content of the printed Eq. vr22 in theta form;
  * hyperdiffusion of momentum acts on velocity, F_q = -lap(rho Kd lap v_q);
    the pressure diffusion F_p becomes a rho-theta tendency through
    d(rho theta)/dp = rho theta / (gamma p);
  * divergence damping: DD = -Kd lap(grad D) per Cartesian component, with
    D the 3D momentum divergence of the current small-step state;
  * levels equally spaced in height, linear (k = 1) Lagrange interpolation
    between centres and interfaces; W = 0 at the bottom and the lid;
  * anelastic switch: the mass flux of the continuity equation becomes
    rho_r v with v = momentum / rho[t] and rho_r the isothermal hydrostatic
    column of the initial state; the factors rho_r / rho[t] (centres, and
    interpolated ratio at interior interfaces) are frozen over the large
    step and scale the horizontal mass divergence, the vertical mass flux
    of the density update and, so that both stay consistent, the buoyancy
    the density change adds to the vertical momentum equation; the
    divergence-damping D, rho theta, the momenta and the equation of state
    are unchanged.

State arrays: rho[n, L], M[n, L, 3] (horizontal momentum, Cartesian),
rth[n, L] (rho theta), W[n, L+1] (rho v_r at interfaces).
"""
from dataclasses import dataclass, field

import numpy as np

from . import grid as grid_mod
from . import operators as op
from . import rng


@dataclass
class Planet:
    radius: float
    omega: float
    gravity: float
    Rd: float
    Cp: float
    p_ref: float = 1.0e5


@dataclass
class Vertical:
    n_lev: int
    z_top: float


@dataclass
class Numerics:
    dt: float
    diff_D: float
    div_damp: bool = True
    energy_fixer: bool = False   # Sec. 3: globally uniform internal-energy fixer
    hydrostatic: bool = False    # Sec. 3: hydrostatic approximation
    shallow: bool = False        # Sec. 3: shallow atmosphere, traditional approximation
    lagrange_order: int = 1      # Sec. 2.1: order k of the vertical interpolation
    anelastic: bool = False      # Sec. 3: anelastic approximation (reading: mass flux rho_r v)


@dataclass
class Forcing:
    kind: int = 0            # 0 none, 1 Newtonian relaxation, 2 hot-Jupiter benchmark
    tau: float = 1.0e5
    T_mean: float = 1300.0   # kind 2: T_surf of T_vert
    dT_daynight: float = 500.0   # kind 2: equator-to-pole difference Delta T_E-P
    lon_substellar: float = 0.0
    lapse: float = 2.0e-4        # kind 2: Gamma_trop (K/m)
    z_strat: float = 2.0e6       # kind 2: z_stra (m)
    dT_strat: float = 10.0       # kind 2: Delta T_stra (K)
    sigma_strat: float = 0.12    # kind 2: sigma_stra
    # kind 3, Held-Suarez (Eqs. im_eq_v, im_eq_fv, Sec. 7.1 T_eq and K_T)
    k_f: float = 1.0 / 86400.0
    k_a: float = 1.0 / (40.0 * 86400.0)
    k_s: float = 1.0 / (4.0 * 86400.0)
    sigma_b: float = 0.7
    dT_y: float = 60.0
    dtheta_z: float = 10.0       # not printed in the paper (reading)
    p_star: float = 1.0e5        # not printed in the paper (reading)
    T_top: float = 315.0
    T_min: float = 200.0


@dataclass
class Init:
    T0: float
    p_surf: float
    noise_amp: float = 0.0
    seed: int = 0


def lon_lat(P):
    """Longitude and latitude of unit vectors.  At a pole the longitude is
    undefined; there it is taken as 0 (east = +y, north = -sign(z) x)."""
    horiz = np.sqrt(P[:, 0] ** 2 + P[:, 1] ** 2)
    lam = np.where(horiz < 1e-12, 0.0, np.arctan2(P[:, 1], P[:, 0]))
    phi = np.arcsin(np.clip(P[:, 2], -1.0, 1.0))
    return lam, phi


@dataclass
class Model:
    """Everything fixed for a run: grid, planet, levels and derived constants."""
    G: object
    planet: Planet
    vert: Vertical
    num: Numerics
    forcing: Forcing = field(default_factory=Forcing)

    def __post_init__(self):
        pl, v = self.planet, self.vert
        self.Cv = pl.Cp - pl.Rd
        self.gamma = pl.Cp / self.Cv
        L = v.n_lev
        k = self.num.lagrange_order
        if k not in (1, 3) or (k == 3 and L < 4):
            raise ValueError("Lagrange order 1, or 3 with at least 4 levels")
        self.dz = v.z_top / L
        self.zI = np.arange(L + 1) * self.dz
        self.zC = (np.arange(L) + 0.5) * self.dz
        self.rI = pl.radius + self.zI
        self.rC = pl.radius + self.zC
        if self.num.shallow:
            # shallow atmosphere: every distance from the centre is the
            # planet radius (horizontal operators, vertical flux
            # divergence, volumes)
            self.rI = np.full(L + 1, pl.radius)
            self.rC = np.full(L, pl.radius)
        # Eq. kd with dbar of Eq. grid_qts
        dbar = grid_mod.mean_spacing(self.G.g, pl.radius)
        self.Kd = self.num.diff_D * dbar ** 4 / self.num.dt
        self.rhat = self.G.P
        # anelastic reference column (model_from_workload sets it to the
        # initial state's isothermal column)
        self.rho_ref = None
        # Newtonian relaxation target (day/night contrast, height independent)
        lam, phi = lon_lat(self.rhat)
        f = self.forcing
        teq = f.T_mean + 0.5 * f.dT_daynight * np.cos(phi) * np.cos(lam - f.lon_substellar)
        self.Teq = np.repeat(teq[:, None], L, axis=1)

    # Eq. pressure and its inverse
    def eos(self, rth):
        pr, Rd = self.planet.p_ref, self.planet.Rd
        return pr * (Rd * rth / pr) ** self.gamma

    def rth_from_p(self, p):
        pr, Rd = self.planet.p_ref, self.planet.Rd
        return (pr / Rd) * (p / pr) ** (1.0 / self.gamma)


@dataclass
class State:
    rho: np.ndarray
    M: np.ndarray
    rth: np.ndarray
    W: np.ndarray

    def copy(self):
        return State(self.rho.copy(), self.M.copy(), self.rth.copy(), self.W.copy())


# ---------------------------------------------------------------------------
# Initial state: isothermal, in discrete hydrostatic balance, plus noise
# ---------------------------------------------------------------------------
def isothermal_column(model, init):
    """Density of the isothermal column at T0 in discrete hydrostatic
    balance with the W equation, p at the first centre p_s exp(-g dz / 2 Rd T0)."""
    pl = model.planet
    L = model.vert.n_lev
    RT = pl.Rd * init.T0
    half = 0.5 * pl.gravity * model.dz
    rho_col = np.empty(L)
    rho_col[0] = init.p_surf * np.exp(-half / RT) / RT
    for k in range(1, L):
        # p_k - p_{k-1} = -g dz (rho_{k-1} + rho_k) / 2 with p = rho Rd T0
        rho_col[k] = rho_col[k - 1] * (RT - half) / (RT + half)
    return rho_col


def init_state(model, init, planet_index=0):
    pl = model.planet
    L, n = model.vert.n_lev, model.G.n
    RT = pl.Rd * init.T0
    rho_col = isothermal_column(model, init)
    p_col = rho_col * RT
    eps = rng.column_noise(init.seed, n, L, init.noise_amp, planet_index)
    T = init.T0 + eps
    p = np.repeat(p_col[None, :], n, axis=0)
    rho = p / (pl.Rd * T)
    rth = model.rth_from_p(p)
    return State(rho, np.zeros((n, L, 3)), rth, np.zeros((n, L + 1)))


# ---------------------------------------------------------------------------
# Vertical helpers (Lagrange interpolation, flux divergence in r)
# ---------------------------------------------------------------------------
def to_interfaces(x):
    """Interior interface values (j = 1..L-1) of a centre field [n, L, ...]."""
    return 0.5 * (x[:, :-1] + x[:, 1:])


def to_centres(W):
    """Centre values of an interface field [n, L+1]."""
    return 0.5 * (W[:, :-1] + W[:, 1:])


def lagrange_weights(nodes, target):
    """Weights L_j(target) of the Lagrange polynomial through `nodes`
    (Sec. 2.1): prod over i != j of (target - z_i) / (z_j - z_i)."""
    w = np.ones(len(nodes))
    for j, zj in enumerate(nodes):
        for i, zi in enumerate(nodes):
            if i != j:
                w[j] *= (target - zi) / (zj - zi)
    return w


def centre_to_interface_matrix(L, k):
    """[L-1, L]: interior interfaces j = 1..L-1 (height j dz) from the k + 1
    centres (heights (i + 1/2) dz) nearest to them: the stencil starts at
    j - (k + 1) // 2, shifted to stay inside the column."""
    A = np.zeros((L - 1, L))
    for j in range(1, L):
        s = min(max(j - (k + 1) // 2, 0), L - 1 - k)
        A[j - 1, s:s + k + 1] = lagrange_weights(np.arange(s, s + k + 1) + 0.5, float(j))
    return A


def interface_to_centre_matrix(L, k):
    """[L, L+1]: centres (height (c + 1/2) dz) from the k + 1 interfaces
    (heights i dz, ground and lid included) nearest to them: the stencil
    starts at c - (k - 1) // 2, shifted to stay inside the column."""
    A = np.zeros((L, L + 1))
    for c in range(L):
        s = min(max(c - (k - 1) // 2, 0), L - k)
        A[c, s:s + k + 1] = lagrange_weights(np.arange(s, s + k + 1, dtype=float), c + 0.5)
    return A


def interp_c2i(model, x):
    """Interior interface values of a centre field with the model's
    Lagrange order (order 1: the mean of the two neighbours)."""
    k = model.num.lagrange_order
    if k == 1:
        return to_interfaces(x)
    return np.einsum("jl,nl...->nj...", centre_to_interface_matrix(x.shape[1], k), x)


def interp_i2c(model, W):
    """Centre values of an interface field with the model's Lagrange
    order."""
    k = model.num.lagrange_order
    if k == 1:
        return to_centres(W)
    return np.einsum("cl,nl->nc", interface_to_centre_matrix(W.shape[1] - 1, k), W)


def vertical_div(model, F):
    """(1 / r_C^2) d(r^2 F)/dr for interface fluxes F[n, L+1, ...]."""
    rI2 = model.rI ** 2
    rC2 = model.rC ** 2
    sh = (1, -1) + (1,) * (F.ndim - 2)
    flux = F * rI2.reshape((1, -1) + (1,) * (F.ndim - 2))
    return (flux[:, 1:] - flux[:, :-1]) / (rC2.reshape(sh) * model.dz)


# ---------------------------------------------------------------------------
# Thomas algorithm (Sec. 3, rigid lid)
# ---------------------------------------------------------------------------
def thomas(a, b, c, d):
    """Solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j, j = 0..m-1.

    Arrays are [n, m]; a[:, 0] and c[:, -1] are ignored (the boundary values
    are zero).  Forward elimination, then back substitution.
    """
    n, m = d.shape
    cp = np.zeros((n, m))
    dp = np.zeros((n, m))
    cp[:, 0] = c[:, 0] / b[:, 0]
    dp[:, 0] = d[:, 0] / b[:, 0]
    for j in range(1, m):
        den = b[:, j] - a[:, j] * cp[:, j - 1]
        cp[:, j] = c[:, j] / den
        dp[:, j] = (d[:, j] - a[:, j] * dp[:, j - 1]) / den
    x = np.zeros((n, m))
    x[:, -1] = dp[:, -1]
    for j in range(m - 2, -1, -1):
        x[:, j] = dp[:, j] - cp[:, j] * x[:, j + 1]
    return x


# ---------------------------------------------------------------------------
# Split-explicit schedule (Wicker-Skamarock RK3 + inner loop)
# ---------------------------------------------------------------------------
def stage_schedule(dt, n):
    """(substeps, dtau) of the three RK stages: (1, dt/3), (n/2, dt/n), (n, dt/n)."""
    if n < 2 or n % 2:
        raise ValueError("n_acoustic must be even and >= 2")
    return [(1, dt / 3.0), (n // 2, dt / n), (n, dt / n)]


def split_explicit(phi_t, slow, substep, dt, n):
    """One large step: for each stage evaluate the slow forcing at the
    previous stage state, restart from phi[t] and take the stage's substeps.

    slow(phi_prev) -> forcing;  substep(phi, forcing, dtau) -> phi.
    With only slow terms this is exactly the WS-RK3 predictor-corrector.
    """
    prev = phi_t
    for ns, dtau in stage_schedule(dt, n):
        forcing = slow(prev)
        phi = phi_t
        for _ in range(ns):
            phi = substep(phi, forcing, dtau)
        prev = phi
    return prev


# ---------------------------------------------------------------------------
# Hyperdiffusion (Sec. 4), once per large step at Phi[t]
# ---------------------------------------------------------------------------
def hyperdiffusion(model, st, p):
    G, Kd, rC = model.G, model.Kd, model.rC
    Rd = model.planet.Rd
    H_rho = -Kd * op.lap(G, op.lap(G, st.rho, rC), rC)
    v = st.M / st.rho[..., None]
    H_M = np.zeros_like(st.M)
    for q in range(3):
        H_M[..., q] = -op.lap(G, st.rho * Kd * op.lap(G, v[..., q], rC), rC)
    H_M = op.proj_h(H_M, model.rhat)
    L = model.vert.n_lev
    H_W = np.zeros((G.n, L + 1))
    if L > 1:
        rhoI = interp_c2i(model, st.rho)
        w = st.W[:, 1:L] / rhoI
        rI = model.rI[1:L]
        H_W[:, 1:L] = -op.lap(G, rhoI * Kd * op.lap(G, w, rI), rI)
    T = p / (st.rho * Rd)
    F_p = -Rd * op.lap(G, st.rho * Kd * op.lap(G, T, rC), rC)
    H_rth = st.rth / (model.gamma * p) * F_p
    return H_rho, H_M, H_W, H_rth


# ---------------------------------------------------------------------------
# Slow terms of one RK stage: advection, Coriolis, projections
# ---------------------------------------------------------------------------
def slow_forcing(model, prev, large):
    """Forcings S_M, S_W, S_rho, S_rth and linearisation at the stage state."""
    G, rC, rhat = model.G, model.rC, model.rhat
    L = model.vert.n_lev
    rh = rhat[:, None, :]
    Om = model.planet.omega
    if model.num.shallow:
        # shallow atmosphere with the traditional approximation: the
        # horizontal momentum is carried by the horizontal velocity M / rho
        # (no metric terms in w), the vertical momentum as the scalar
        # w = rho v_r / rho (no curvature term from the horizontal motion),
        # and the Coriolis force keeps only the local vertical component of
        # Omega acting on the horizontal motion
        v = prev.M / prev.rho[..., None]
        A = np.zeros_like(prev.M)
        for q in range(3):
            A[..., q] = op.div(G, v[..., q, None] * prev.M, rC)
        vI = np.zeros((G.n, L + 1, 3))
        vI[:, 1:L] = interp_c2i(model, v)
        A += vertical_div(model, prev.W[..., None] * vI)
        C = 2.0 * Om * rhat[:, None, 2:3] * np.cross(np.broadcast_to(rh, prev.M.shape), prev.M)
        AC = A + C
        S_M = op.proj_h(-large["G_t"] - AC, rhat) + large["H_M"]
        w = interp_i2c(model, prev.W) / prev.rho
        Ar = op.div(G, w[..., None] * prev.M, rC)
        wI = np.zeros((G.n, L + 1))
        wI[:, 1:L] = interp_c2i(model, w)
        Ar = Ar + vertical_div(model, prev.W * wI)
        S_W = np.zeros((G.n, L + 1))
        S_W[:, 1:L] = large["I"][:, 1:L] - interp_c2i(model, Ar) + large["H_W"][:, 1:L]
    else:
        # full Cartesian momentum m = M + Wbar rhat and velocity m / rho
        m = prev.M + interp_i2c(model, prev.W)[..., None] * rh
        v = m / prev.rho[..., None]
        # advection A_q = div(v_q M) + (1/r^2) d(r^2 W v_q)/dr
        A = np.zeros_like(m)
        for q in range(3):
            A[..., q] = op.div(G, v[..., q, None] * prev.M, rC)
        vI = np.zeros((G.n, L + 1, 3))
        vI[:, 1:L] = interp_c2i(model, v)
        A += vertical_div(model, prev.W[..., None] * vI)
        # Coriolis 2 Omega zhat x m
        C = np.zeros_like(m)
        C[..., 0] = -2.0 * Om * m[..., 1]
        C[..., 1] = 2.0 * Om * m[..., 0]
        AC = A + C
        S_M = op.proj_h(-large["G_t"] - AC, rhat) + large["H_M"]
        S_W = np.zeros((G.n, L + 1))
        ACr = op.proj_r(AC, rhat)
        S_W[:, 1:L] = large["I"][:, 1:L] - interp_c2i(model, ACr) + large["H_W"][:, 1:L]
    thetaC = prev.rth / prev.rho
    thetaI = np.empty((G.n, L + 1))
    thetaI[:, 1:L] = interp_c2i(model, thetaC)
    thetaI[:, 0] = thetaC[:, 0]
    thetaI[:, L] = thetaC[:, L - 1]
    Gam = model.gamma * model.eos(prev.rth) / prev.rth
    return dict(S_M=S_M, S_W=S_W, S_rho=large["H_rho"], S_rth=large["H_rth"],
                thetaC=thetaC, thetaI=thetaI, Gam=Gam)


# ---------------------------------------------------------------------------
# One acoustic substep (Eqs. mom2, momr2, dens2, pt2, theta_to_p)
# ---------------------------------------------------------------------------
def momentum_divergence(model, M, W):
    """3D divergence of the momentum: div_h M + (1/r^2) d(r^2 W)/dr."""
    return op.div(model.G, M, model.rC) + vertical_div(model, W)


def acoustic_substep(model, st, f, dtau, large):
    G, rC, rhat = model.G, model.rC, model.rhat
    g = model.planet.gravity
    dz = model.dz
    L = model.vert.n_lev
    p_t, rho_t = large["p_t"], large["rho_t"]
    p = model.eos(st.rth)
    # divergence damping on the current small-step state
    DD = 0.0
    if model.num.div_damp:
        D = momentum_divergence(model, st.M, st.W)
        GD = op.grad(G, D, rC)
        DD = np.zeros_like(st.M)
        for q in range(3):
            DD[..., q] = -model.Kd * op.lap(G, GD[..., q], rC)
    # (H) explicit horizontal momentum with the deviation pressure gradient
    M = st.M + dtau * (-op.grad(G, p - p_t, rC) + f["S_M"] + DD)
    M = op.proj_h(M, rhat)
    # (Div) horizontal mass and theta fluxes of the new momentum (anelastic:
    # the mass flux is rho_r / rho[t] times the momentum)
    ane = model.num.anelastic
    D_rho = op.div(G, large["fC"][..., None] * M, rC) if ane else op.div(G, M, rC)
    D_th = op.div(G, f["thetaC"][..., None] * M, rC)
    # (Pred) explicit parts of density and pressure
    rho_hat = st.rho + dtau * (-D_rho + f["S_rho"])
    p_hat = p + dtau * f["Gam"] * (-D_th + f["S_rth"])
    rho_hs = rho_hat - rho_t
    p_hs = p_hat - p_t
    # (Tri) HEVI vertical momentum at interfaces 1..L-1
    rI2, rC2 = model.rI ** 2, model.rC ** 2
    ap = dtau * rI2[1:] / (rC2 * dz)        # alpha+_k, k = 0..L-1
    am = dtau * rI2[:-1] / (rC2 * dz)       # alpha-_k
    Gam, th = f["Gam"], f["thetaI"]
    W = st.W.copy()
    if L > 1:
        j = np.arange(1, L)
        c1 = dtau / dz
        c2 = 0.5 * g * dtau
        # the density change of the vertical mass flux enters through the
        # buoyancy: anelastic, that flux is rho_r / rho[t] times W
        fI = large["fI"] if ane else np.ones((G.n, L + 1))
        a = -c1 * Gam[:, j - 1] * am[j - 1] * th[:, j - 1] + c2 * am[j - 1] * fI[:, j - 1]
        c = -c1 * Gam[:, j] * ap[j] * th[:, j + 1] - c2 * ap[j] * fI[:, j + 1]
        if model.num.hydrostatic:
            # no vertical acceleration (no time derivative, advection or
            # other slow terms of rho v_r): the new W is the one that leaves
            # the end of the substep in hydrostatic balance, the [t]
            # imbalance I plus the deviation pressure gradient and buoyancy
            # summing to zero
            b = (c1 * th[:, j] * (Gam[:, j] * am[j] + Gam[:, j - 1] * ap[j - 1])
                 + c2 * (am[j] - ap[j - 1]) * fI[:, j])
            d = (dtau * large["I"][:, j] - c1 * (p_hs[:, j] - p_hs[:, j - 1])
                 - c2 * (rho_hs[:, j - 1] + rho_hs[:, j]))
        else:
            b = (1.0 + c1 * th[:, j] * (Gam[:, j] * am[j] + Gam[:, j - 1] * ap[j - 1])
                 + c2 * (am[j] - ap[j - 1]) * fI[:, j])
            d = (st.W[:, j] + dtau * f["S_W"][:, j] - c1 * (p_hs[:, j] - p_hs[:, j - 1])
                 - c2 * (rho_hs[:, j - 1] + rho_hs[:, j]))
        W[:, 1:L] = thomas(a, b, c, d)
    W[:, 0] = 0.0
    W[:, L] = 0.0
    # (Upd) density (Eq. dens2) and rho theta (Eq. pt2) with the new W
    if ane:
        fI = large["fI"]
        rho = rho_hat - ap * fI[:, 1:] * W[:, 1:] + am * fI[:, :-1] * W[:, :-1]
    else:
        rho = rho_hat - ap * W[:, 1:] + am * W[:, :-1]
    rth = (st.rth + dtau * (-D_th + f["S_rth"])
           - ap * th[:, 1:] * W[:, 1:] + am * th[:, :-1] * W[:, :-1])
    return State(rho, M, rth, W)


# ---------------------------------------------------------------------------
# Large step, physics, diagnostics
# ---------------------------------------------------------------------------
def large_step_terms(model, st):
    """Quantities frozen over a large step at Phi[t]."""
    G, rC = model.G, model.rC
    g = model.planet.gravity
    L = model.vert.n_lev
    p_t = model.eos(st.rth)
    H_rho, H_M, H_W, H_rth = hyperdiffusion(model, st, p_t)
    G_t = op.proj_h(op.grad(G, p_t, rC), model.rhat)
    I = np.zeros((G.n, L + 1))
    if L > 1:
        I[:, 1:L] = (-(p_t[:, 1:] - p_t[:, :-1]) / model.dz
                     - 0.5 * g * (st.rho[:, :-1] + st.rho[:, 1:]))
    out = dict(p_t=p_t, rho_t=st.rho.copy(), H_rho=H_rho, H_M=H_M, H_W=H_W,
               H_rth=H_rth, G_t=G_t, I=I)
    if model.num.anelastic:
        # Sec. 3 anelastic approximation: the mass flux rho v of the
        # continuity equation becomes rho_r v, with rho_r the reference
        # column and v the momentum over the density of Phi[t]; the factors
        # rho_r / rho[t] at the centres and interior interfaces are frozen
        # over the large step (boundary interfaces only meet W = 0)
        rr = np.repeat(model.rho_ref[None, :], G.n, axis=0)
        fI = np.ones((G.n, L + 1))
        if L > 1:
            fI[:, 1:L] = interp_c2i(model, rr) / interp_c2i(model, st.rho)
        out.update(fC=rr / st.rho, fI=fI)
    return out


def t_vert(f, z):
    """Eq. tvert: the hot-Jupiter vertical temperature profile at heights z."""
    zs, lap = f.z_strat, f.lapse
    trop = f.T_mean - lap * (zs + (z - zs) / 2.0) + np.sqrt((lap * (z - zs) / 2.0) ** 2 + f.dT_strat ** 2)
    return np.where(z <= zs, trop, f.T_mean - lap * zs + f.dT_strat)


def surface_pressure(model, p, T):
    """Sec. 5: surface pressure of each column, the lowest cell's pressure
    carried hydrostatically down to z = 0 at that cell's temperature."""
    pl = model.planet
    return p[:, 0] * np.exp(pl.gravity * model.zC[0] / (pl.Rd * T[:, 0]))


def hot_jupiter_teq(model, p, T):
    """Eqs. teq-hj and btrop: T_eq = T_vert + beta_trop Delta T_E-P cos(lambda
    - lambda_ss) cos(phi), with sigma = p / p_s of the dynamics output."""
    f = model.forcing
    z = model.zC[None, :]
    sigma = p / surface_pressure(model, p, T)[:, None]
    beta = np.where(z <= f.z_strat,
                    np.sin(np.pi * (sigma - f.sigma_strat) / (2.0 * (1.0 - f.sigma_strat))), 0.0)
    lam, phi = lon_lat(model.rhat)
    h = np.cos(lam - f.lon_substellar) * np.cos(phi)
    return t_vert(f, z) + beta * f.dT_daynight * h[:, None]


def held_suarez_rates(model, p, T):
    """Sec. 7.1, Earth benchmark: boundary-layer friction rate K_v(sigma)
    (Eq. im_eq_fv), the relaxation rate K_T(sigma, lat) and T_eq(p, lat), with
    sigma = p / p_s of the dynamics output (p_s as for the hot Jupiter)."""
    f, pl = model.forcing, model.planet
    sigma = p / surface_pressure(model, p, T)[:, None]
    _, phi = lon_lat(model.rhat)
    s2, c2 = np.sin(phi)[:, None] ** 2, np.cos(phi)[:, None] ** 2
    ramp = np.maximum(0.0, (sigma - f.sigma_b) / (1.0 - f.sigma_b))
    Kv = f.k_f * ramp
    KT = f.k_a + (f.k_s - f.k_a) * ramp * c2 * c2
    kappa = pl.Rd / pl.Cp
    x = p / f.p_star
    Teq = np.maximum(f.T_min, (f.T_top - f.dT_y * s2 - f.dtheta_z * np.log(x) * c2) * x ** kappa)
    return Kv, KT, Teq


def newtonian(model, st):
    """Sec. 5 physics after the dynamics, backward Euler (Eqs. im_eq_t and
    im_eq_v) at fixed density: kind 1 relaxes T with K_T = 1/tau toward the
    day/night T_eq, kind 2 toward the hot-Jupiter T_eq, kind 3 is the
    Held-Suarez forcing (relaxation and boundary-layer friction)."""
    f, pl = model.forcing, model.planet
    if f.kind not in (1, 2, 3):
        return st
    dt = model.num.dt
    p = model.eos(st.rth)
    T = p / (st.rho * pl.Rd)
    M = st.M
    if f.kind == 3:
        Kv, KT, Teq = held_suarez_rates(model, p, T)
        kt = dt * KT
        M = st.M / (1.0 + Kv * dt)[..., None]
    else:
        kt = dt / f.tau
        Teq = model.Teq if f.kind == 1 else hot_jupiter_teq(model, p, T)
    Tn = (T + kt * Teq) / (1.0 + kt)
    rth = model.rth_from_p(st.rho * pl.Rd * Tn)
    return State(st.rho, M, rth, st.W)


def large_step(model, st, n):
    large = large_step_terms(model, st)
    out = split_explicit(
        st,
        lambda prev: slow_forcing(model, prev, large),
        lambda phi, f, dtau: acoustic_substep(model, phi, f, dtau, large),
        model.num.dt, n)
    if model.num.energy_fixer:
        out = fix_energy(model, out, total_energy(model, st))
    return newtonian(model, out)


def run(model, st, n_large, n):
    for _ in range(n_large):
        st = large_step(model, st, n)
    return st


def mass(model, st):
    """sum_i sum_k rho A_c r_k^2 dz (A_c on the unit sphere)."""
    return float(np.sum(st.rho * model.G.Ac[:, None] * model.rC[None, :] ** 2) * model.dz)


def total_energy(model, st):
    """Total energy of the state: internal rho Cv T = Cv p / Rd, kinetic
    (|rho v_h|^2 + (rho v_r)^2) / (2 rho) with rho v_r at the layer centre,
    and potential rho g z (constant radial gravity, z above the ground),
    summed over the cells with the volumes of ``mass``."""
    pl = model.planet
    p = model.eos(st.rth)
    Wc = to_centres(st.W)
    e = (model.Cv / pl.Rd) * p \
        + 0.5 * (np.sum(st.M ** 2, axis=-1) + Wc ** 2) / st.rho \
        + st.rho * pl.gravity * model.zC[None, :]
    return float(np.sum(e * model.G.Ac[:, None] * model.rC[None, :] ** 2) * model.dz)


def axial_angular_momentum(model, st):
    """Absolute angular momentum about the rotation axis: per cell the
    relative part (R x rho v)_z with R = r_C rhat (the radial momentum adds
    nothing about the axis) plus the planetary part rho Omega r_C^2 cos^2(lat),
    summed over the cells with the volumes of ``mass``."""
    P = model.rhat
    rC = model.rC[None, :]
    rel = rC * (P[:, None, 0] * st.M[..., 1] - P[:, None, 1] * st.M[..., 0])
    plan = st.rho * model.planet.omega * rC ** 2 * (P[:, None, 0] ** 2 + P[:, None, 1] ** 2)
    return float(np.sum((rel + plan) * model.G.Ac[:, None] * model.rC[None, :] ** 2) * model.dz)


def fix_energy(model, st, E_target):
    """Energy fixer in the manner of Williamson (2009), which the paper
    implements (Sec. 3, discussion of the thermodynamic equation): one
    temperature increment, the same at every cell, at fixed density, that
    brings the total energy back to E_target.  The internal energy is linear
    in T at fixed rho, so the increment is (E_target - E) / (Cv * mass)."""
    pl = model.planet
    dT = (E_target - total_energy(model, st)) / (model.Cv * mass(model, st))
    T = model.eos(st.rth) / (st.rho * pl.Rd) + dT
    return State(st.rho, st.M, model.rth_from_p(st.rho * pl.Rd * T), st.W)


def fields(model, st):
    """Diagnostic fields T, u, v, w, p (canonical [col][lev])."""
    pl = model.planet
    p = model.eos(st.rth)
    T = p / (st.rho * pl.Rd)
    P = model.rhat
    lam, phi = lon_lat(P)
    east = np.stack([-np.sin(lam), np.cos(lam), np.zeros_like(lam)], axis=-1)
    north = np.stack([-np.sin(phi) * np.cos(lam), -np.sin(phi) * np.sin(lam),
                      np.cos(phi)], axis=-1)
    vel = st.M / st.rho[..., None]
    u = np.sum(vel * east[:, None, :], axis=-1)
    v = np.sum(vel * north[:, None, :], axis=-1)
    w = to_centres(st.W) / st.rho
    return dict(T=T, u=u, v=v, w=w, p=p, rho=st.rho, rhotheta=st.rth,
                Mx=st.M[..., 0], My=st.M[..., 1], Mz=st.M[..., 2], W=st.W)


def model_from_workload(w, G):
    """Oracle model and initial state for a workload recipe (``workloads``)."""
    planet = Planet(w.radius, w.omega, w.gravity, w.Rd, w.Cp, w.p_ref)
    vert = Vertical(w.n_lev, w.z_top)
    num = Numerics(w.dt, w.diff_D, w.div_damp, w.energy_fixer, w.hydrostatic, w.shallow,
                   w.lagrange_order, getattr(w, "anelastic", False))
    forcing = Forcing(w.forcing_kind, w.tau, w.T_mean, w.dT_daynight, w.lon_substellar,
                      w.lapse, w.z_strat, w.dT_strat, w.sigma_strat, w.k_f, w.k_a, w.k_s, w.sigma_b,
                      w.dT_y, w.dtheta_z, w.p_star, w.T_top, w.T_min)
    model = Model(G, planet, vert, num, forcing)
    init = Init(w.T0, w.p_surf, w.noise_amp, w.seed)
    model.rho_ref = isothermal_column(model, init)
    st = init_state(model, init)
    return model, st
