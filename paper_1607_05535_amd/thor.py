"""ctypes binding of libthor (include/thor.h): argument marshalling only.

Every computation happens inside libthor.so; PyTorch supplies the device
buffer and the HIP stream.  Importing torch before loading the library makes
libthor bind to the HIP runtime torch already loaded.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libthor.so")

THOR_OK, THOR_EINVAL, THOR_ENOMEM, THOR_EHIP, THOR_ENONFINITE, THOR_ENOTCONV = 0, -1, -2, -3, -4, -5
THOR_ENOTSMOOTH = -6
THOR_FP64, THOR_MIXED = 0, 1
THOR_FORCING_NONE, THOR_FORCING_NEWTONIAN, THOR_FORCING_HOT_JUPITER, THOR_FORCING_HELD_SUAREZ = 0, 1, 2, 3
THOR_DIAG_MASS, THOR_DIAG_FIELD, THOR_DIAG_STATE_EXPORT, THOR_DIAG_SCALARS, THOR_DIAG_ENERGY = 1, 2, 3, 4, 5
THOR_DIAG_ANGULAR_MOMENTUM = 6
FIELDS = {"T": 0, "u": 1, "v": 2, "w": 3, "p": 4, "rho": 5, "rhotheta": 6,
          "Mx": 7, "My": 8, "Mz": 9, "W": 10}

EXPORTED = ["thor_last_error", "thor_grid_params_default", "thor_grid_build", "thor_grid_info",
            "thor_grid_export", "thor_grid_coefficients", "thor_grid_damping_coefficients", "thor_grid_free", "thor_state_bytes",
            "thor_state_init", "thor_step", "thor_diag", "thor_state_blob_bytes",
            "thor_state_import", "thor_set_timing", "thor_kernel_time", "thor_state_free",
            "thor_set_vert_levels_per_lane",
            "thor_autotune", "thor_batch_bytes", "thor_batch_init", "thor_batch_step",
            "thor_batch_member", "thor_batch_autotune", "thor_batch_free",
            "thor_mlp_bytes", "thor_mlp_init", "thor_mlp_param_count", "thor_mlp_set_params",
            "thor_mlp_get_params", "thor_mlp_forward", "thor_mlp_loss_grad", "thor_mlp_train_step",
            "thor_mlp_free", "thor_restriction_bytes", "thor_restriction_build",
            "thor_restriction_export", "thor_restriction_free", "thor_restrict", "thor_state_fields32",
            "thor_field_stats", "thor_corrector_bytes", "thor_corrector_init", "thor_corrector_batch",
            "thor_corrector_apply", "thor_corrector_free", "thor_zonal_bytes", "thor_zonal_init",
            "thor_zonal_accumulate", "thor_zonal_result", "thor_zonal_imprint", "thor_zonal_reset",
            "thor_zonal_free", "thor_stream_mix", "thor_field_stats_noalloc", "thor_mlp_set_fused"]
ZM_FIELDS = ("u", "v", "T", "theta", "upvp", "vpTp", "weight", "psi", "snapshots")


class ThorError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libthor error {code}: {msg}")
        self.code = code


class GridParams(ctypes.Structure):
    _fields_ = [("glevel", ctypes.c_int), ("smooth", ctypes.c_int), ("k", ctypes.c_double),
                ("beta", ctypes.c_double), ("alpha", ctypes.c_double), ("dt", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int)]


class Planet(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("radius", "omega", "gravity", "Rd", "Cp", "p_ref")]


class Vertical(ctypes.Structure):
    _fields_ = [("n_lev", ctypes.c_int), ("z_top", ctypes.c_double)]


class Numerics(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("diff_D", ctypes.c_double), ("div_damp", ctypes.c_int),
                ("precision", ctypes.c_int), ("energy_fixer", ctypes.c_int), ("hydrostatic", ctypes.c_int),
                ("shallow", ctypes.c_int), ("lagrange_order", ctypes.c_int), ("anelastic", ctypes.c_int)]


class Forcing(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tau", ctypes.c_double), ("T_mean", ctypes.c_double),
                ("dT_daynight", ctypes.c_double), ("lon_substellar", ctypes.c_double),
                ("lapse", ctypes.c_double), ("z_strat", ctypes.c_double), ("dT_strat", ctypes.c_double),
                ("sigma_strat", ctypes.c_double), ("k_f", ctypes.c_double), ("k_a", ctypes.c_double),
                ("k_s", ctypes.c_double), ("sigma_b", ctypes.c_double), ("dT_y", ctypes.c_double),
                ("dtheta_z", ctypes.c_double), ("p_star", ctypes.c_double), ("T_top", ctypes.c_double),
                ("T_min", ctypes.c_double)]


class Init(ctypes.Structure):
    _fields_ = [("T0", ctypes.c_double), ("p_surf", ctypes.c_double), ("noise_amp", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("planet_index", ctypes.c_int)]


class Scalars(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("mass", "max_speed", "max_w", "min_T", "max_T")]


_lib = None


def lib():
    """Load libthor.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libthor.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int), \
        ctypes.POINTER(ctypes.c_double)
    L.thor_last_error.restype = ctypes.c_char_p
    L.thor_grid_params_default.argtypes = [ctypes.c_int, ctypes.POINTER(GridParams)]
    L.thor_grid_params_default.restype = None
    L.thor_grid_build.argtypes = [ctypes.POINTER(GridParams), ctypes.POINTER(vp)]
    L.thor_grid_info.argtypes = [vp, i64p, ip, ip]
    L.thor_grid_export.argtypes = [vp, vp, vp, vp]
    L.thor_grid_coefficients.argtypes = [vp, vp, vp]
    L.thor_grid_damping_coefficients.argtypes = [vp, vp, vp]
    L.thor_grid_free.argtypes = [vp]
    L.thor_grid_free.restype = None
    L.thor_state_bytes.argtypes = [vp, ctypes.POINTER(Vertical), ctypes.POINTER(Numerics),
                                   ctypes.POINTER(ctypes.c_size_t)]
    L.thor_state_init.argtypes = [vp, ctypes.POINTER(Planet), ctypes.POINTER(Vertical),
                                  ctypes.POINTER(Numerics), ctypes.POINTER(Forcing), ctypes.POINTER(Init),
                                  vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.thor_step.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.thor_diag.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t]
    L.thor_state_blob_bytes.argtypes = [vp]
    L.thor_state_blob_bytes.restype = ctypes.c_size_t
    L.thor_state_import.argtypes = [vp, vp, ctypes.c_size_t]
    L.thor_set_timing.argtypes = [vp, ctypes.c_int]
    L.thor_set_vert_levels_per_lane.argtypes = [vp, ctypes.c_int]
    L.thor_kernel_time.argtypes = [vp, ctypes.c_char_p, dp, ip]
    L.thor_autotune.argtypes = [vp, ctypes.c_int, ip]
    L.thor_state_free.argtypes = [vp]
    L.thor_state_free.restype = None
    L.thor_batch_bytes.argtypes = [ctypes.c_int, vp, ctypes.POINTER(Vertical), ctypes.POINTER(Numerics),
                                   ctypes.POINTER(ctypes.c_size_t)]
    L.thor_batch_init.argtypes = [ctypes.c_int, vp, ctypes.POINTER(Planet), ctypes.POINTER(Vertical),
                                  ctypes.POINTER(Numerics), ctypes.POINTER(Forcing), ctypes.POINTER(Init),
                                  vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.thor_batch_step.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.thor_batch_member.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp)]
    L.thor_batch_autotune.argtypes = [vp, ctypes.c_int, ip]
    L.thor_batch_free.argtypes = [vp]
    L.thor_batch_free.restype = None
    L.thor_mlp_bytes.argtypes = [ctypes.c_int, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.thor_mlp_init.argtypes = [ctypes.c_int, vp, ctypes.c_int, ctypes.c_uint64, vp, ctypes.c_size_t, vp,
                                ctypes.POINTER(vp)]
    L.thor_mlp_param_count.argtypes = [vp]
    L.thor_mlp_param_count.restype = ctypes.c_size_t
    L.thor_mlp_set_params.argtypes = [vp, vp]
    L.thor_mlp_get_params.argtypes = [vp, vp]
    L.thor_mlp_forward.argtypes = [vp, vp, ctypes.c_int, vp]
    L.thor_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int, dp, vp]
    L.thor_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_float]
    L.thor_mlp_free.argtypes = [vp]
    L.thor_mlp_free.restype = None
    szp = ctypes.POINTER(ctypes.c_size_t)
    L.thor_restriction_bytes.argtypes = [vp, vp, szp]
    L.thor_restriction_build.argtypes = [vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.thor_restriction_export.argtypes = [vp, vp]
    L.thor_restriction_free.argtypes = [vp]
    L.thor_restriction_free.restype = None
    L.thor_restrict.argtypes = [vp, vp, vp]
    L.thor_state_fields32.argtypes = [vp, vp]
    L.thor_field_stats.argtypes = [vp, vp, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, vp,
                                   ctypes.c_size_t, vp, dp]
    L.thor_corrector_bytes.argtypes = [vp, szp]
    L.thor_corrector_init.argtypes = [vp, vp, vp, ctypes.c_float, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.thor_corrector_batch.argtypes = [vp, vp, vp, ctypes.c_size_t, vp, vp, ctypes.c_int, vp, vp]
    L.thor_corrector_apply.argtypes = [vp, ip]
    L.thor_corrector_free.argtypes = [vp]
    L.thor_corrector_free.restype = None
    _lib = L
    L.thor_zonal_bytes.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.thor_zonal_init.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, ctypes.c_int,
                                  vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.thor_zonal_accumulate.argtypes = [vp]
    L.thor_zonal_result.argtypes = [vp, vp, ip]
    L.thor_zonal_imprint.argtypes = [vp, vp, ip]
    L.thor_zonal_reset.argtypes = [vp]
    L.thor_zonal_free.argtypes = [vp]
    L.thor_zonal_free.restype = None
    L.thor_stream_mix.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int64, vp]
    L.thor_mlp_set_fused.argtypes = [vp, ctypes.c_int]
    L.thor_field_stats_noalloc.argtypes = [vp, vp, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, vp,
                                           ctypes.POINTER(ctypes.c_double)]
    return L


def _check(rc, allow=()):
    if rc != THOR_OK and rc not in allow:
        raise ThorError(rc, lib().thor_last_error().decode())
    return rc


# ---------------------------------------------------------------------------
# One Python function per C entry point
# ---------------------------------------------------------------------------
def thor_grid_params_default(glevel):
    p = GridParams()
    lib().thor_grid_params_default(glevel, ctypes.byref(p))
    return p


def thor_grid_build(params):
    """Returns (handle, rc); rc is THOR_OK, THOR_ENOTCONV or THOR_ENOTSMOOTH
    (a usable grid either way)."""
    h = ctypes.c_void_p()
    rc = _check(lib().thor_grid_build(ctypes.byref(params), ctypes.byref(h)), allow=(THOR_ENOTCONV, THOR_ENOTSMOOTH))
    return h, rc


def thor_grid_info(h):
    n, npent, it = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
    _check(lib().thor_grid_info(h, ctypes.byref(n), ctypes.byref(npent), ctypes.byref(it)))
    return n.value, npent.value, it.value


def thor_grid_export(h, n):
    nbr = np.empty((n, 6), dtype=np.int32)
    xyz = np.empty((n, 3))
    area = np.empty(n)
    _check(lib().thor_grid_export(h, nbr.ctypes.data, xyz.ctypes.data, area.ctypes.data))
    return nbr, xyz, area


def thor_grid_coefficients(h, n):
    dc = np.empty((n, 7, 3))
    lc = np.empty((n, 6))
    _check(lib().thor_grid_coefficients(h, dc.ctypes.data, lc.ctypes.data))
    return dc, lc


def thor_grid_free(h):
    lib().thor_grid_free(h)


def thor_state_bytes(gh, vert, num):
    out = ctypes.c_size_t()
    _check(lib().thor_state_bytes(gh, ctypes.byref(vert), ctypes.byref(num), ctypes.byref(out)))
    return out.value


def thor_state_init(gh, planet, vert, num, forcing, init, dev_ptr, dev_bytes, stream_ptr):
    h = ctypes.c_void_p()
    _check(lib().thor_state_init(gh, ctypes.byref(planet), ctypes.byref(vert), ctypes.byref(num),
                                 ctypes.byref(forcing), ctypes.byref(init), ctypes.c_void_p(dev_ptr),
                                 dev_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(h)))
    return h


def thor_step(sh, n_large, n_acoustic):
    _check(lib().thor_step(sh, n_large, n_acoustic))


def thor_diag(sh, kind, field, out):
    """out: a writable numpy array (host).  Returns the rc (ENONFINITE kept)."""
    return _check(lib().thor_diag(sh, kind, field, out.ctypes.data, out.nbytes),
                  allow=(THOR_ENONFINITE,))


def thor_state_blob_bytes(sh):
    return lib().thor_state_blob_bytes(sh)


def thor_state_import(sh, blob):
    _check(lib().thor_state_import(sh, blob.ctypes.data, blob.nbytes))


def thor_set_timing(sh, on):
    _check(lib().thor_set_timing(sh, int(on)))


def thor_set_vert_levels_per_lane(sh, nl):
    _check(lib().thor_set_vert_levels_per_lane(sh, int(nl)))


def thor_kernel_time(sh, name):
    ms, cnt = ctypes.c_double(), ctypes.c_int()
    _check(lib().thor_kernel_time(sh, name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def thor_autotune(sh, n_acoustic):
    """Returns the chosen wavefronts per workgroup per kernel family."""
    out = (ctypes.c_int * 4)()
    _check(lib().thor_autotune(sh, n_acoustic, out))
    return dict(zip(("large", "slow", "hmom", "vert"), list(out)))


def thor_state_free(sh):
    lib().thor_state_free(sh)


def _arrays(structs_per_member):
    cols = list(zip(*structs_per_member))
    out = []
    for col in cols:
        T = type(col[0]) * len(col)
        out.append(T(*col))
    return out


def thor_batch_bytes(grid_handles, verts, nums):
    n = len(grid_handles)
    gh = (ctypes.c_void_p * n)(*[g.value for g in grid_handles])
    V = (Vertical * n)(*verts)
    N = (Numerics * n)(*nums)
    out = ctypes.c_size_t()
    _check(lib().thor_batch_bytes(n, gh, V, N, ctypes.byref(out)))
    return out.value


def thor_batch_init(grid_handles, members, dev_ptr, dev_bytes, stream_ptr):
    """members: list of (planet, vert, num, forcing, init) structs."""
    n = len(grid_handles)
    gh = (ctypes.c_void_p * n)(*[g.value for g in grid_handles])
    P, V, N, F, I = _arrays(members)
    h = ctypes.c_void_p()
    _check(lib().thor_batch_init(n, gh, P, V, N, F, I, ctypes.c_void_p(dev_ptr), dev_bytes,
                                 ctypes.c_void_p(stream_ptr), ctypes.byref(h)))
    return h


def thor_batch_step(bh, n_large, n_acoustic):
    _check(lib().thor_batch_step(bh, n_large, n_acoustic))


def thor_batch_member(bh, i):
    h = ctypes.c_void_p()
    _check(lib().thor_batch_member(bh, i, ctypes.byref(h)))
    return h


def thor_batch_autotune(bh, n_acoustic):
    out = (ctypes.c_int * 4)()
    _check(lib().thor_batch_autotune(bh, n_acoustic, out))
    return dict(zip(("large", "slow", "hmom", "vert"), list(out)))


def thor_batch_free(bh):
    lib().thor_batch_free(bh)


# ---------------------------------------------------------------------------
# Small owning wrappers
# ---------------------------------------------------------------------------
class Grid:
    def __init__(self, glevel, smooth=True, **kw):
        p = thor_grid_params_default(glevel)
        p.smooth = int(smooth)
        for k, v in kw.items():
            setattr(p, k, v)
        self.params = p
        self.handle, self.rc = thor_grid_build(p)
        self.n, self.n_pent, self.spring_iters = thor_grid_info(self.handle)

    def export(self):
        return thor_grid_export(self.handle, self.n)

    def coefficients(self):
        return thor_grid_coefficients(self.handle, self.n)

    def damping_coefficients(self):
        idx = np.empty((self.n, 18), dtype=np.int32)
        w = np.empty((self.n, 18, 3))
        _check(lib().thor_grid_damping_coefficients(self.handle, idx.ctypes.data, w.ctypes.data))
        return idx, w

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                thor_grid_free(self.handle)
                self.handle = None
        except Exception:
            pass


def structs_from_workload(w, precision=THOR_FP64):
    planet = Planet(w.radius, w.omega, w.gravity, w.Rd, w.Cp, w.p_ref)
    vert = Vertical(w.n_lev, w.z_top)
    num = Numerics(w.dt, w.diff_D, int(w.div_damp), precision, int(w.energy_fixer), int(w.hydrostatic),
                   int(w.shallow), int(w.lagrange_order), int(getattr(w, "anelastic", False)))
    forcing = Forcing(w.forcing_kind, w.tau, w.T_mean, w.dT_daynight, w.lon_substellar,
                      w.lapse, w.z_strat, w.dT_strat, w.sigma_strat, w.k_f, w.k_a, w.k_s, w.sigma_b,
                      w.dT_y, w.dtheta_z, w.p_star, w.T_top, w.T_min)
    init = Init(w.T0, w.p_surf, w.noise_amp, w.seed, 0)
    return planet, vert, num, forcing, init


class State:
    """A state in a torch-owned device buffer on ``device``."""

    def __init__(self, grid, planet, vert, num, forcing, init, device="cuda:0", stream=None):
        self.grid = grid
        self.n_col, self.n_lev = grid.n, vert.n_lev
        nbytes = thor_state_bytes(grid.handle, vert, num)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.handle = thor_state_init(grid.handle, planet, vert, num, forcing, init,
                                      self.buf.data_ptr(), nbytes, self.stream.cuda_stream)

    def step(self, n_large, n_acoustic):
        thor_step(self.handle, n_large, n_acoustic)

    def field(self, name):
        out = np.empty((self.n_col, self.n_lev))
        rc = thor_diag(self.handle, THOR_DIAG_FIELD, FIELDS[name], out)
        return out, rc

    def mass(self):
        out = np.empty(1)
        rc = thor_diag(self.handle, THOR_DIAG_MASS, 0, out)
        return float(out[0]), rc

    def energy(self):
        out = np.empty(1)
        rc = thor_diag(self.handle, THOR_DIAG_ENERGY, 0, out)
        return float(out[0]), rc

    def angular_momentum(self):
        out = np.empty(1)
        rc = thor_diag(self.handle, THOR_DIAG_ANGULAR_MOMENTUM, 0, out)
        return float(out[0]), rc

    def scalars(self):
        s = Scalars()
        arr = np.frombuffer(s, dtype=np.float64)
        out = np.empty(5)
        rc = thor_diag(self.handle, THOR_DIAG_SCALARS, 0, out)
        del arr
        return dict(zip(("mass", "max_speed", "max_w", "min_T", "max_T"), out)), rc

    def export(self):
        blob = np.empty(thor_state_blob_bytes(self.handle) // 8)
        rc = thor_diag(self.handle, THOR_DIAG_STATE_EXPORT, 0, blob)
        return blob, rc

    def load(self, blob):
        thor_state_import(self.handle, blob)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                thor_state_free(self.handle)
                self.handle = None
        except Exception:
            pass


class Member:
    """A member of an ensemble seen as a state (diagnostics only)."""

    def __init__(self, batch, i, n_col, n_lev):
        self.batch, self.handle, self.n_col, self.n_lev = batch, thor_batch_member(batch.handle, i), n_col, n_lev

    field = State.field
    mass = State.mass
    energy = State.energy
    angular_momentum = State.angular_momentum
    scalars = State.scalars
    export = State.export

    def __del__(self):
        pass


class Batch:
    """An ensemble of planets in one torch-owned device buffer."""

    def __init__(self, grids, members, device="cuda:0", stream=None):
        self.grids = grids
        verts = [m[1] for m in members]
        nums = [m[2] for m in members]
        nbytes = thor_batch_bytes([g.handle for g in grids], verts, nums)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.handle = thor_batch_init([g.handle for g in grids], members, self.buf.data_ptr(), nbytes,
                                      self.stream.cuda_stream)
        self.members = [Member(self, i, g.n, v.n_lev) for i, (g, v) in enumerate(zip(grids, verts))]

    def step(self, n_large, n_acoustic):
        thor_batch_step(self.handle, n_large, n_acoustic)

    def autotune(self, n_acoustic):
        return thor_batch_autotune(self.handle, n_acoustic)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                thor_batch_free(self.handle)
                self.handle = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Corrector network
# ---------------------------------------------------------------------------
def thor_mlp_bytes(widths, max_batch):
    w = (ctypes.c_int * len(widths))(*widths)
    out = ctypes.c_size_t()
    _check(lib().thor_mlp_bytes(len(widths) - 1, w, max_batch, ctypes.byref(out)))
    return out.value


def thor_mlp_init(widths, max_batch, seed, dev_ptr, dev_bytes, stream_ptr):
    w = (ctypes.c_int * len(widths))(*widths)
    h = ctypes.c_void_p()
    _check(lib().thor_mlp_init(len(widths) - 1, w, max_batch, seed, ctypes.c_void_p(dev_ptr), dev_bytes,
                               ctypes.c_void_p(stream_ptr), ctypes.byref(h)))
    return h


class MLP:
    """Corrector network in a torch-owned device buffer.  Inputs are bf16
    device tensors [B, in]; targets and outputs fp32 device tensors."""

    def __init__(self, widths, max_batch, seed=0, device="cuda:0"):
        self.widths = list(widths)
        nbytes = thor_mlp_bytes(self.widths, max_batch)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.buf.device)
        self.handle = thor_mlp_init(self.widths, max_batch, seed, self.buf.data_ptr(), nbytes,
                                    self.stream.cuda_stream)
        self.n_params = lib().thor_mlp_param_count(self.handle)

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().thor_mlp_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, host):
        host = np.ascontiguousarray(host, dtype=np.float32)
        assert host.size == self.n_params
        _check(lib().thor_mlp_set_params(self.handle, host.ctypes.data))

    def unpack(self, flat):
        """Packed parameters -> [(W[out, in], b[out])]."""
        out, off = [], 0
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            W = flat[off:off + i * o].reshape(o, i)
            off += i * o
            b = flat[off:off + o]
            off += o
            out.append((W, b))
        return out

    def forward(self, x, y):
        _check(lib().thor_mlp_forward(self.handle, x.data_ptr(), x.shape[0], y.data_ptr()))

    def set_fused(self, on):
        _check(lib().thor_mlp_set_fused(self.handle, int(bool(on))))

    def loss_grad(self, x, t, want_grad=True):
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        _check(lib().thor_mlp_loss_grad(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0], ctypes.byref(loss),
                                        g.ctypes.data if want_grad else None))
        return loss.value, g

    def train_step(self, x, t, lr):
        _check(lib().thor_mlp_train_step(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0], lr))

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().thor_mlp_free(self.handle)
                self.handle = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Restriction and corrector
# ---------------------------------------------------------------------------
class Restriction:
    """device=None builds a host-only map (for inspection)."""

    def __init__(self, fine_grid, coarse_grid, device="cuda:0"):
        nbytes = ctypes.c_size_t()
        _check(lib().thor_restriction_bytes(fine_grid.handle, coarse_grid.handle, ctypes.byref(nbytes)))
        self.n_fine = fine_grid.n
        h = ctypes.c_void_p()
        if device is None:
            self.buf = None
            _check(lib().thor_restriction_build(fine_grid.handle, coarse_grid.handle, None, 0, None, ctypes.byref(h)))
        else:
            self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
            _check(lib().thor_restriction_build(fine_grid.handle, coarse_grid.handle, self.buf.data_ptr(),
                                                nbytes.value, torch.cuda.current_stream(self.buf.device).cuda_stream,
                                                ctypes.byref(h)))
        self.handle = h

    def coarse_of_fine(self):
        out = np.empty(self.n_fine, dtype=np.int32)
        _check(lib().thor_restriction_export(self.handle, out.ctypes.data))
        return out

    def __call__(self, fine_state, coarse_state):
        _check(lib().thor_restrict(fine_state.handle, coarse_state.handle, self.handle))

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().thor_restriction_free(self.handle)
                self.handle = None
        except Exception:
            pass


def thor_state_fields32(state, out):
    """(T, u, v, w, p) FP32 [5, n_col, n_lev] into the device tensor out."""
    _check(lib().thor_state_fields32(state.handle, out.data_ptr()))


def thor_field_stats(C, Fn, n_arrays, stride, n_col, n_lev):
    """Means and spreads per (field, level): array [2, 5, n_lev]."""
    scratch = torch.empty(n_arrays * 320 * n_lev, dtype=torch.float64, device=C.device)
    out = np.empty(10 * n_lev)
    _check(lib().thor_field_stats(C.data_ptr(), Fn.data_ptr() if Fn is not None else None, n_arrays, stride,
                                  n_col, n_lev, scratch.data_ptr(), scratch.numel() * 8,
                                  torch.cuda.current_stream(C.device).cuda_stream,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(2, 5, n_lev)


def thor_field_stats_noalloc(C, Fn, n_arrays, stride, n_col, n_lev):
    """thor_field_stats without caller scratch: array [2, 5, n_lev]."""
    out = np.empty(10 * n_lev)
    _check(lib().thor_field_stats_noalloc(C.data_ptr(), Fn.data_ptr() if Fn is not None else None, n_arrays,
                                          stride, n_col, n_lev, torch.cuda.current_stream(C.device).cuda_stream,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(2, 5, n_lev)


class Corrector:
    def __init__(self, state, net, norm, bound=5.0):
        nbytes = ctypes.c_size_t()
        _check(lib().thor_corrector_bytes(state.handle, ctypes.byref(nbytes)))
        self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=state.buf.device)
        self.state, self.net = state, net
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        assert norm.size == 20 * state.n_lev
        h = ctypes.c_void_p()
        _check(lib().thor_corrector_init(state.handle, net.handle, norm.ctypes.data, bound, self.buf.data_ptr(),
                                         nbytes.value, ctypes.byref(h)))
        self.handle = h

    def batch(self, C, F, pair_stride, pairs, cols, x, t):
        _check(lib().thor_corrector_batch(self.handle, C.data_ptr(), F.data_ptr(), pair_stride, pairs.data_ptr(),
                                          cols.data_ptr(), pairs.numel(), x.data_ptr(), t.data_ptr()))

    def apply(self, count=True):
        n = ctypes.c_int()
        _check(lib().thor_corrector_apply(self.handle, ctypes.byref(n) if count else None))
        return n.value if count else None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().thor_corrector_free(self.handle)
                self.handle = None
        except Exception:
            pass


class Zonal:
    """Zonal and time means on pressure levels of a state (see thor.h):
    accumulate() adds the state as it stands; result() returns a dict of
    [n_bands, n_plev] arrays (u, v, T, theta, upvp, vpTp, weight, psi,
    snapshots) and the number of accumulated snapshots; imprint() the
    first-layer grid-imprinting map [w*]."""

    def __init__(self, state, grid, radius, gravity, n_bands, plev):
        plev = np.ascontiguousarray(plev, dtype=np.float64)
        nbytes = ctypes.c_size_t()
        _check(lib().thor_zonal_bytes(state.handle, n_bands, plev.ctypes.data, len(plev), ctypes.byref(nbytes)))
        self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=state.buf.device)
        self.state, self.nb, self.np = state, n_bands, len(plev)
        h = ctypes.c_void_p()
        _check(lib().thor_zonal_init(state.handle, grid.handle, radius, gravity, n_bands, plev.ctypes.data,
                                     len(plev), self.buf.data_ptr(), nbytes.value, ctypes.byref(h)))
        self.handle = h

    def accumulate(self):
        _check(lib().thor_zonal_accumulate(self.handle))

    def reset(self):
        _check(lib().thor_zonal_reset(self.handle))

    def result(self):
        out = np.empty((self.nb, self.np, len(ZM_FIELDS)))
        n = ctypes.c_int()
        _check(lib().thor_zonal_result(self.handle, out.ctypes.data, ctypes.byref(n)))
        return {k: out[:, :, i] for i, k in enumerate(ZM_FIELDS)}, n.value

    def imprint(self):
        """[w*] per column (canonical ids) and the number of snapshots."""
        out = np.empty(self.state.n_col)
        n = ctypes.c_int()
        _check(lib().thor_zonal_imprint(self.handle, out.ctypes.data, ctypes.byref(n)))
        return out, n.value

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().thor_zonal_free(self.handle)
                self.handle = None
        except Exception:
            pass


def stream_mix(srcs, dsts, stream=None):
    """thor_stream_mix over torch float64 CUDA tensors of equal length
    (measurement aid: the read/write mix of a kernel without its work)."""
    import torch
    n = srcs[0].numel()
    if any(t.numel() != n or t.dtype != torch.float64 or not t.is_cuda for t in list(srcs) + list(dsts)):
        raise ValueError("stream_mix: float64 CUDA tensors of one length")
    sp = (ctypes.c_void_p * len(srcs))(*[t.data_ptr() for t in srcs])
    dp = (ctypes.c_void_p * len(dsts))(*[t.data_ptr() for t in dsts])
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().thor_stream_mix(sp, len(srcs), dp, len(dsts), n, ctypes.c_void_p(s)))
