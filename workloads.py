"""Seeded synthetic workloads of the THOR HEVI step.

This module holds input recipes only (planet constants, level counts, time
steps, seeds); it contains none of the method's arithmetic and is the one
piece shared by the tests, the benchmark, the oracle runs and the library
runs.

Constants: Table 1 of the paper (Earth: radius 6.371e6 m, rotation
7.292e-5 1/s, gravity 9.8; hot Jupiter: radius 1e8 m, rotation 2.1e-5 1/s,
cp 13226.5, Rd 3779) as amended by the workload definitions below.  The
nondimensional diffusion number D follows from Eqs. kd and tau_d:
tau_d = dbar^4 / (32 Kd) and Kd = D dbar^4 / dt give D = dt / (32 tau_d),
evaluated with the paper's benchmark time steps and damping times
(Earth: 1000 s, 6.46e3 s; hot Jupiter: 600 s, 941.2 s).
"""
import math
from dataclasses import dataclass, field

D_EARTH = 1000.0 / (32.0 * 6460.0)     # 4.837e-3
D_HOT_JUPITER = 600.0 / (32.0 * 941.2)  # 1.992e-2


@dataclass
class Workload:
    name: str
    glevel: int
    n_lev: int
    z_top: float
    radius: float
    omega: float
    gravity: float
    Rd: float
    Cp: float
    p_ref: float
    dt: float
    n_acoustic: int
    n_large: int
    diff_D: float
    div_damp: bool
    T0: float
    p_surf: float
    noise_amp: float
    seed: int
    forcing_kind: int = 0
    tau: float = 1.0e5
    T_mean: float = 0.0
    dT_daynight: float = 0.0
    lon_substellar: float = 0.0
    lapse: float = 2.0e-4
    z_strat: float = 2.0e6
    dT_strat: float = 10.0
    sigma_strat: float = 0.12
    k_f: float = 1.0 / 86400.0
    k_a: float = 1.0 / (40.0 * 86400.0)
    k_s: float = 1.0 / (4.0 * 86400.0)
    sigma_b: float = 0.7
    dT_y: float = 60.0
    dtheta_z: float = 10.0
    p_star: float = 1.0e5
    T_top: float = 315.0
    T_min: float = 200.0
    energy_fixer: bool = False
    hydrostatic: bool = False
    shallow: bool = False
    lagrange_order: int = 1
    anelastic: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def n_col(self):
        return 10 * 4 ** self.glevel + 2

    @property
    def cells(self):
        return self.n_col * self.n_lev

    @property
    def substeps_per_large(self):
        return 1 + 3 * self.n_acoustic // 2


def substellar_longitude(seed):
    """Substellar longitude 2 pi U, U from the top 53 bits of a SplitMix64
    output step applied to the seed (reproducible, no library state)."""
    z = (seed + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    z ^= z >> 31
    return 2.0 * math.pi * ((z >> 11) * 2.0 ** -53)


def earth_c1():
    """g4 (2562 columns) x 20 levels to 36 km, Earth air, isothermal 300 K
    rest state with +/-0.1 K noise; 10 large steps of 600 s, 6 substeps."""
    return Workload("g4L20-earth", 4, 20, 36.0e3, 6.371e6, 7.292e-5, 9.8, 287.0,
                    1005.0, 1.0e5, 600.0, 6, 10, D_EARTH, True, 300.0, 1.0e5,
                    0.1, 1)


def gas_giant(glevel, n_lev, seed, n_large, dt=300.0, n_acoustic=8):
    """Gas-giant-like planet with Newtonian relaxation (timescale 1e5 s)
    toward a day/night equilibrium temperature of 500 K contrast."""
    T0, g, Rd = 1300.0, 9.42, 3779.0
    z_top = Rd * T0 / g * math.log(2.2e7 / 1.0e3)   # p_top ~ 1e3 Pa
    return Workload(f"g{glevel}L{n_lev}-gasgiant", glevel, n_lev, z_top, 1.0e8,
                    2.1e-5, g, Rd, 13226.0, 1.0e5, dt, n_acoustic, n_large,
                    D_HOT_JUPITER, True, T0, 2.2e7, 0.1, seed, forcing_kind=1,
                    tau=1.0e5, T_mean=1300.0, dT_daynight=500.0,
                    lon_substellar=substellar_longitude(seed))


def gas_giant_c2():
    """g6 (40962 columns) x 32 levels, 300 s large steps with 8 substeps."""
    return gas_giant(6, 32, 2, 1000)


def gas_giant_c3():
    """g7 (163842 columns) x 48 levels; one Earth day = 288 steps of 300 s."""
    return gas_giant(7, 48, 3, 288)


def small_gas_giant(glevel=3, n_lev=12, seed=7, n_large=3):
    """Small gas-giant case for fast parity tests of the forcing path."""
    return gas_giant(glevel, n_lev, seed, n_large, dt=300.0 * 2 ** (6 - glevel), n_acoustic=8)


def ensemble(n=64, seed=4, glevels=(4, 5, 6), levels=(20, 32, 48), n_acoustic=8):
    """Ensemble of planets: grid level and layer count drawn uniformly from the
    given sets, radius log-uniform in [3e6, 1e8] m, rotation log-uniform in
    [1e-6, 1e-4] 1/s, isothermal 200-1500 K with +/-0.1 K noise; Earth air
    (Rd 287, cp 1005), gravity 9.8, surface pressure 1e5 Pa, lid at
    ln(100) scale heights.  Time step per planet:
    min(n floor(0.1 dbar / c_s), 0.25 / Omega, 1800 s), i.e. an acoustic
    Courant number <= 0.1 per substep and 2 Omega dt <= 0.5."""
    import numpy as np
    rs = np.random.default_rng(seed)
    out = []
    Rd, Cp, g = 287.0, 1005.0, 9.8
    gamma = Cp / (Cp - Rd)
    for i in range(n):
        gl = int(rs.choice(glevels))
        L = int(rs.choice(levels))
        A = float(np.exp(rs.uniform(np.log(3e6), np.log(1e8))))
        om = float(np.exp(rs.uniform(np.log(1e-6), np.log(1e-4))))
        T0 = float(rs.uniform(200.0, 1500.0))
        dbar = math.sqrt(2 * math.pi / 5) * A / 2 ** gl
        cs = math.sqrt(gamma * Rd * T0)
        dt = min(n_acoustic * math.floor(0.1 * dbar / cs), 0.25 / om, 1800.0)
        z_top = Rd * T0 / g * math.log(100.0)
        out.append(Workload(f"member{i}-g{gl}L{L}", gl, L, z_top, A, om, g, Rd, Cp, 1.0e5,
                            dt, n_acoustic, 1, D_EARTH, True, T0, 1.0e5, 0.1,
                            seed * 1000 + i))
    return out


def hot_jupiter(glevel=5, n_lev=37, n_large=1, dt=600.0, n_acoustic=8, noise_amp=0.0, seed=5):
    """The hot-Jupiter benchmark of Sec. 7.2 (Eqs. teq-hj, btrop, tvert): Table 1
    planet (radius 1e8 m, rotation 2.1e-5 1/s, gravity 8, cp 13226.5,
    Rd 3779), 37 layers to 4875 km, isothermal 1600 K at rest, Newtonian
    relaxation with timescale 1.5e5 s toward T_vert + beta_trop 300 K
    cos(lon) cos(lat) (T_surf 1600 K, lapse 2e-4 K/m, z_stra 2000 km,
    Delta T_stra 10 K, sigma_stra 0.12), no boundary-layer friction, large
    step 600 s, diffusion timescale 941.2 s.  Surface pressure 2.2e7 Pa
    (not given for this test; the gas-giant recipes' value)."""
    return Workload(f"g{glevel}L{n_lev}-hotjupiter", glevel, n_lev, 4.875e6, 1.0e8, 2.1e-5, 8.0,
                    3779.0, 13226.5, 1.0e5, dt, n_acoustic, n_large, D_HOT_JUPITER, True, 1600.0,
                    2.2e7, noise_amp, seed, forcing_kind=2, tau=1.5e5, T_mean=1600.0,
                    dT_daynight=300.0, lon_substellar=0.0)


def held_suarez(glevel=5, n_lev=37, n_large=1, dt=1000.0, n_acoustic=8, noise_amp=0.1, seed=6, T0=300.0):
    """The Earth benchmark of Sec. 7.1 (Held-Suarez forcing): Table 1 Earth
    (radius 6.371e6 m, rotation 7.292e-5 1/s, gravity 9.8, cp 1004.6,
    Rd 287.04), 37 layers to 32 km, large step 1000 s, diffusion timescale
    6.46e3 s; friction k_f = 1/day above sigma_b = 0.7, relaxation k_a =
    1/40 days, k_s = 1/4 days, (Delta T)_y = 60 K.  (Delta theta)_z = 10 K
    and p* = 1e5 Pa are not printed in the paper (readings).  The start is
    isothermal with small noise instead of the equatorial T_eq profile."""
    return Workload(f"g{glevel}L{n_lev}-heldsuarez", glevel, n_lev, 3.2e4, 6.371e6, 7.292e-5, 9.8,
                    287.04, 1004.6, 1.0e5, dt, n_acoustic, n_large, D_EARTH, True, T0, 1.0e5,
                    noise_amp, seed, forcing_kind=3)


def corrector_pair(fine_glevel=7, coarse_glevel=5, n_lev=32, dt_coarse=600.0, ratio=4, base_seed=1000):
    """Coarse and fine gas-giant runs for the learned corrector: same planet,
    levels, forcing (substellar longitude from base_seed) and noise recipe;
    the fine step is dt_coarse / ratio.  Seeds of individual trajectories are
    set by the caller."""
    from copy import copy
    fine = gas_giant(fine_glevel, n_lev, base_seed, 1, dt=dt_coarse / ratio)
    coarse = copy(fine)
    coarse.glevel, coarse.dt = coarse_glevel, dt_coarse
    coarse.name = f"g{coarse_glevel}L{n_lev}-gasgiant"
    return fine, coarse
