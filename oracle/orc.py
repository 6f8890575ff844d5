"""ctypes binding of the FP64 CPU oracle (``liborc.so``).

TEST INFRASTRUCTURE ONLY (see ``orc.h``).  Arrays are NumPy float64, C-contiguous,
laid out ``[var][elem][node]``.  The library is built on first use if missing.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

__all__ = ["Oracle", "OracleError", "NonPhysicalState", "lgl", "legendre_vinv", "ln_mean",
           "flux_phys", "flux_ec", "flux_central", "flux_llf", "flux_hll", "entropy",
           "entropy_vars", "lsrk_coeffs", "num_threads", "set_num_threads", "VOLUME", "SURFACE", "lib",
           "CurvOracle", "curv_map", "curv_mms", "MhdOracle", "mhd_flux", "mhd_surface_flux",
           "mhd_fast_speed", "mhd_alfven", "mhd_ec_flux", "mhd_entropy", "mhd_entropy_vars"]

VOLUME = {"ec": 0, "central": 1, "shockcap_hg": 2, "weak": 3, "none": 4}
SURFACE = {"llf": 0, "hll": 1, "ec": 2, "none": 3}


class OracleError(RuntimeError):
    pass


class NonPhysicalState(OracleError):
    pass


class _Cfg(C.Structure):
    _fields_ = [("dim", C.c_int32), ("polydeg", C.c_int32), ("cells", C.c_int32 * 3),
                ("xmin", C.c_double * 3), ("xmax", C.c_double * 3), ("gamma", C.c_double),
                ("volume", C.c_int32), ("surface", C.c_int32), ("fv_flux", C.c_int32),
                ("alpha_max", C.c_double), ("alpha_min", C.c_double),
                ("alpha_smooth", C.c_int32)]


class _CurvCfg(C.Structure):
    _fields_ = [("polydeg", C.c_int32), ("cells", C.c_int32), ("warp", C.c_double),
                ("gamma", C.c_double), ("volume", C.c_int32), ("surface", C.c_int32),
                ("source", C.c_int32)]


class _MhdCfg(C.Structure):
    _fields_ = [("polydeg", C.c_int32), ("cells", C.c_int32), ("gamma", C.c_double),
                ("surface", C.c_int32), ("volume", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER(C.c_double)
        CP = C.POINTER(_Cfg)
        for name, args, res in [
            ("orc_lgl", [C.c_int, P, P, P], C.c_int),
            ("orc_legendre_vinv", [C.c_int, P], C.c_int),
            ("orc_ln_mean", [C.c_double, C.c_double], C.c_double),
            ("orc_flux_phys", [P, C.c_int, C.c_int, C.c_double, P], C.c_int),
            ("orc_flux_ec", [P, P, C.c_int, C.c_int, C.c_double, P], C.c_int),
            ("orc_flux_central", [P, P, C.c_int, C.c_int, C.c_double, P], C.c_int),
            ("orc_flux_llf", [P, P, C.c_int, C.c_int, C.c_double, P], C.c_int),
            ("orc_flux_hll", [P, P, C.c_int, C.c_int, C.c_double, P], C.c_int),
            ("orc_entropy", [P, C.c_int, C.c_double], C.c_double),
            ("orc_entropy_vars", [P, C.c_int, C.c_double, P], C.c_int),
            ("orc_num_nodes", [CP], C.c_int64),
            ("orc_node_coords", [CP, P], C.c_int),
            ("orc_rhs", [CP, P, P], C.c_int),
            ("orc_indicator", [CP, P, P, P], C.c_int),
            ("orc_indicator_energy", [CP, P, P], C.c_int),
            ("orc_rhs_alpha", [CP, P, P, P], C.c_int),
            ("orc_max_dt", [CP, P, C.c_double, P], C.c_int),
            ("orc_lsrk_coeffs", [P, P, P], C.c_int),
            ("orc_step", [CP, P, C.c_int32, C.c_double, C.c_double, P], C.c_int),
            ("orc_integrals", [CP, P, P, P], C.c_int),
            ("orc_num_threads", [], C.c_int),
            ("orc_set_num_threads", [C.c_int], C.c_int),
            ("orc_curv_map", [C.c_double, P, P], C.c_int),
            ("orc_curv_mms", [C.c_double, P, C.c_double, P, P], C.c_int),
            ("orc_curv_num_nodes", [C.POINTER(_CurvCfg)], C.c_int64),
            ("orc_curv_geometry", [C.POINTER(_CurvCfg), P, P, P], C.c_int),
            ("orc_curv_initial", [C.POINTER(_CurvCfg), C.c_double, P], C.c_int),
            ("orc_curv_rhs", [C.POINTER(_CurvCfg), P, C.c_double, P], C.c_int),
            ("orc_curv_max_dt", [C.POINTER(_CurvCfg), P, C.c_double, P], C.c_int),
            ("orc_curv_step", [C.POINTER(_CurvCfg), P, C.c_int32, C.c_double, C.c_double, P],
             C.c_int),
            ("orc_mhd_flux", [P, C.c_int, C.c_double, P], C.c_int),
            ("orc_mhd_surface_flux", [C.c_int, P, P, C.c_int, C.c_double, P], C.c_int),
            ("orc_mhd_fast_speed", [P, C.c_int, C.c_double], C.c_double),
            ("orc_mhd_num_nodes", [C.POINTER(_MhdCfg)], C.c_int64),
            ("orc_mhd_rhs", [C.POINTER(_MhdCfg), P, P], C.c_int),
            ("orc_mhd_max_dt", [C.POINTER(_MhdCfg), P, C.c_double, P], C.c_int),
            ("orc_mhd_step", [C.POINTER(_MhdCfg), P, C.c_int32, C.c_double, C.c_double, P],
             C.c_int),
            ("orc_mhd_alfven", [C.c_double, P, C.c_double, P], C.c_int),
            ("orc_mhd_ec_flux", [P, P, C.c_int, C.c_double, P], C.c_int),
            ("orc_mhd_entropy", [P, C.c_double], C.c_double),
            ("orc_mhd_entropy_vars", [P, C.c_double, P], C.c_int),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st == 0:
        return
    if st == 4:
        raise NonPhysicalState(f"{what}: non-physical state (rho <= 0, p <= 0 or NaN)")
    raise OracleError(f"{what}: error code {st}")


# --------------------------------------------------------------------------- tables
def lgl(N):
    """LGL nodes, weights and differentiation matrix D[i, j] = l_j'(x_i)."""
    n = N + 1
    x, w, D = np.zeros(n), np.zeros(n), np.zeros(n * n)
    _check(lib().orc_lgl(N, _p(x), _p(w), _p(D)), "lgl")
    return x, w, D.reshape(n, n)


def legendre_vinv(N):
    n = N + 1
    V = np.zeros(n * n)
    _check(lib().orc_legendre_vinv(N, _p(V)), "legendre_vinv")
    return V.reshape(n, n)


def lsrk_coeffs():
    A, B, c = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().orc_lsrk_coeffs(_p(A), _p(B), _p(c))
    return A, B, c


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads of the following oracle calls; returns the previous number."""
    return lib().orc_set_num_threads(int(n))


# --------------------------------------------------------------------------- pointwise
def ln_mean(x, y):
    return lib().orc_ln_mean(float(x), float(y))


def _pw(name, *us, d, dim, gamma):
    f = np.zeros(dim + 2)
    args = [_p(_f64(u)) for u in us]
    st = getattr(lib(), name)(*args, d, dim, gamma, _p(f))
    _check(st, name)
    return f


def flux_phys(u, d, dim=3, gamma=1.4):
    return _pw("orc_flux_phys", u, d=d, dim=dim, gamma=gamma)


def flux_ec(uL, uR, d, dim=3, gamma=1.4):
    return _pw("orc_flux_ec", uL, uR, d=d, dim=dim, gamma=gamma)


def flux_central(uL, uR, d, dim=3, gamma=1.4):
    return _pw("orc_flux_central", uL, uR, d=d, dim=dim, gamma=gamma)


def flux_llf(uL, uR, d, dim=3, gamma=1.4):
    return _pw("orc_flux_llf", uL, uR, d=d, dim=dim, gamma=gamma)


def flux_hll(uL, uR, d, dim=3, gamma=1.4):
    return _pw("orc_flux_hll", uL, uR, d=d, dim=dim, gamma=gamma)


def entropy(u, dim=3, gamma=1.4):
    return lib().orc_entropy(_p(_f64(u)), dim, gamma)


def entropy_vars(u, dim=3, gamma=1.4):
    w = np.zeros(dim + 2)
    _check(lib().orc_entropy_vars(_p(_f64(u)), dim, gamma, _p(w)), "entropy_vars")
    return w


# --------------------------------------------------------------------------- solver
class Oracle:
    """Oracle semidiscretisation on a uniform periodic Cartesian grid."""

    def __init__(self, dim, polydeg, cells, xmin, xmax, gamma=1.4, volume="ec", surface="llf",
                 fv_flux="llf", alpha_max=0.5, alpha_min=0.001, alpha_smooth=True, **_ignored):
        c = _Cfg()
        c.dim = dim
        c.polydeg = polydeg
        cells = list(cells) + [1] * (3 - len(cells))
        xmin = list(xmin) + [0.0] * (3 - len(xmin))
        xmax = list(xmax) + [1.0] * (3 - len(xmax))
        for d in range(3):
            c.cells[d] = int(cells[d])
            c.xmin[d] = float(xmin[d])
            c.xmax[d] = float(xmax[d])
        c.gamma = gamma
        c.volume = VOLUME[volume] if isinstance(volume, str) else int(volume)
        c.surface = SURFACE[surface] if isinstance(surface, str) else int(surface)
        c.fv_flux = SURFACE[fv_flux] if isinstance(fv_flux, str) else int(fv_flux)
        c.alpha_max = alpha_max
        c.alpha_min = alpha_min
        c.alpha_smooth = 1 if alpha_smooth else 0
        self.cfg = c
        self.dim, self.N = dim, polydeg
        self.n = polydeg + 1
        self.NN = self.n ** dim
        self.nvar = dim + 2
        nn = lib().orc_num_nodes(C.byref(c))
        if nn < 0:
            raise OracleError("invalid configuration")
        self.num_nodes = int(nn)
        self.E = self.num_nodes // self.NN
        self.shape = (self.nvar, self.E, self.NN)

    def _u(self, u):
        u = _f64(u)
        if u.size != self.nvar * self.num_nodes:
            raise ValueError(f"state has {u.size} entries, expected {self.nvar * self.num_nodes}")
        return u

    def node_coords(self):
        xyz = np.zeros((self.dim, self.E, self.NN))
        _check(lib().orc_node_coords(C.byref(self.cfg), _p(xyz)), "node_coords")
        return xyz

    def rhs(self, u):
        u = self._u(u)
        du = np.zeros(self.shape)
        _check(lib().orc_rhs(C.byref(self.cfg), _p(u), _p(du)), "rhs")
        return du

    def rhs_alpha(self, u, alpha):
        u = self._u(u)
        alpha = _f64(alpha)
        du = np.zeros(self.shape)
        _check(lib().orc_rhs_alpha(C.byref(self.cfg), _p(u), _p(alpha), _p(du)), "rhs_alpha")
        return du

    def indicator(self, u):
        """(alpha_raw, alpha): clipped per-element alpha, and after neighbour smoothing."""
        u = self._u(u)
        ar, a = np.zeros(self.E), np.zeros(self.E)
        _check(lib().orc_indicator(C.byref(self.cfg), _p(u), _p(ar), _p(a)), "indicator")
        return ar, a

    def indicator_energy(self, u):
        u = self._u(u)
        en = np.zeros(self.E)
        _check(lib().orc_indicator_energy(C.byref(self.cfg), _p(u), _p(en)), "indicator_energy")
        return en

    def max_dt(self, u, cfl):
        u = self._u(u)
        dt = C.c_double(0.0)
        _check(lib().orc_max_dt(C.byref(self.cfg), _p(u), cfl, C.byref(dt)), "max_dt")
        return dt.value

    def step(self, u, nsteps, cfl=0.5, dt_fixed=0.0, t=0.0):
        """Advance a copy of u by nsteps; returns (u_new, t_new)."""
        u = self._u(u).copy()
        tt = C.c_double(t)
        _check(lib().orc_step(C.byref(self.cfg), _p(u), int(nsteps), cfl, dt_fixed,
                              C.byref(tt)), "step")
        return u, tt.value

    def integrals(self, u, du=None):
        u = self._u(u)
        out = np.zeros(7)
        dd = None if du is None else self._u(du)
        _check(lib().orc_integrals(C.byref(self.cfg), _p(u), _p(dd), _p(out)), "integrals")
        return out


# --------------------------------------------------------------------------- curvilinear
def curv_map(xi, warp=0.15):
    """The Eq. (2) mapping of one reference point."""
    x = np.zeros(3)
    _check(lib().orc_curv_map(float(warp), _p(_f64(xi)), _p(x)), "curv_map")
    return x


def curv_mms(x, t, gamma=1.4):
    """Manufactured solution u(x, t) and its source s(x, t) at one point."""
    u, s = np.zeros(5), np.zeros(5)
    _check(lib().orc_curv_mms(gamma, _p(_f64(x)), float(t), _p(u), _p(s)), "curv_mms")
    return u, s


class CurvOracle:
    """The warped periodic box of the PID study (cells^3 elements on [-1,1]^3, Eq. (2))."""

    def __init__(self, polydeg, cells, warp=0.15, gamma=1.4, volume="ec", surface="llf",
                 source="mms"):
        c = _CurvCfg()
        c.polydeg, c.cells, c.warp, c.gamma = polydeg, cells, warp, gamma
        c.volume = VOLUME[volume]
        c.surface = SURFACE[surface]
        c.source = {"none": 0, "mms": 1}[source]
        self.cfg = c
        self.N, self.K, self.n = polydeg, cells, polydeg + 1
        self.NN = self.n ** 3
        self.E = cells ** 3
        self.dim = 3
        if lib().orc_curv_num_nodes(C.byref(c)) < 0:
            raise OracleError("invalid curvilinear configuration")

    def _u(self, u):
        u = _f64(u)
        if u.size != 5 * self.E * self.NN:
            raise ValueError("state has the wrong size")
        return u

    def geometry(self):
        n = self.E * self.NN
        xyz, Ja, J = np.zeros(3 * n), np.zeros(9 * n), np.zeros(n)
        _check(lib().orc_curv_geometry(C.byref(self.cfg), _p(xyz), _p(Ja), _p(J)), "geometry")
        return (xyz.reshape(3, self.E, self.NN), Ja.reshape(3, 3, self.E, self.NN),
                J.reshape(self.E, self.NN))

    def initial(self, t=0.0):
        u = np.zeros((5, self.E, self.NN))
        _check(lib().orc_curv_initial(C.byref(self.cfg), float(t), _p(u)), "initial")
        return u

    def rhs(self, u, t=0.0):
        u = self._u(u)
        du = np.zeros_like(u)
        _check(lib().orc_curv_rhs(C.byref(self.cfg), _p(u), float(t), _p(du)), "rhs")
        return du.reshape(5, self.E, self.NN)

    def max_dt(self, u, cfl):
        dt = C.c_double(0.0)
        _check(lib().orc_curv_max_dt(C.byref(self.cfg), _p(self._u(u)), cfl, C.byref(dt)),
               "max_dt")
        return dt.value

    def step(self, u, nsteps, cfl=0.5, dt_fixed=0.0, t=0.0):
        u = self._u(u).copy()
        tt = C.c_double(t)
        _check(lib().orc_curv_step(C.byref(self.cfg), _p(u), int(nsteps), cfl, dt_fixed,
                                   C.byref(tt)), "step")
        return u.reshape(5, self.E, self.NN), tt.value


# --------------------------------------------------------------------------- ideal MHD
def mhd_flux(u, d, gamma=1.4):
    f = np.zeros(8)
    _check(lib().orc_mhd_flux(_p(_f64(u)), d, gamma, _p(f)), "mhd_flux")
    return f


def mhd_surface_flux(kind, uL, uR, d, gamma=1.4):
    f = np.zeros(8)
    _check(lib().orc_mhd_surface_flux(SURFACE[kind], _p(_f64(uL)), _p(_f64(uR)), d, gamma,
                                      _p(f)), "mhd_surface_flux")
    return f


def mhd_ec_flux(uL, uR, d, gamma=1.4):
    f = np.zeros(8)
    _check(lib().orc_mhd_ec_flux(_p(_f64(uL)), _p(_f64(uR)), d, gamma, _p(f)), "mhd_ec_flux")
    return f


def mhd_entropy(u, gamma=1.4):
    return lib().orc_mhd_entropy(_p(_f64(u)), gamma)


def mhd_entropy_vars(u, gamma=1.4):
    w = np.zeros(8)
    _check(lib().orc_mhd_entropy_vars(_p(_f64(u)), gamma, _p(w)), "mhd_entropy_vars")
    return w


def mhd_fast_speed(u, d, gamma=1.4):
    return lib().orc_mhd_fast_speed(_p(_f64(u)), d, gamma)


def mhd_alfven(x, t, gamma=1.4):
    u = np.zeros(8)
    _check(lib().orc_mhd_alfven(gamma, _p(_f64(x)), float(t), _p(u)), "mhd_alfven")
    return u


class MhdOracle:
    """Ideal MHD on [-1,1]^3 with cells^3 elements: weak form ("weak") or entropy-conservative
    flux differencing with Powell's non-conservative term ("ec"); HLL, LLF or EC surface."""

    def __init__(self, polydeg, cells, gamma=5.0 / 3.0, surface="hll", volume="weak"):
        c = _MhdCfg()
        c.polydeg, c.cells, c.gamma, c.surface = polydeg, cells, gamma, SURFACE[surface]
        c.volume = VOLUME[volume]
        self.cfg = c
        self.N, self.K, self.n = polydeg, cells, polydeg + 1
        self.NN, self.E, self.gamma = self.n ** 3, cells ** 3, gamma
        if lib().orc_mhd_num_nodes(C.byref(c)) < 0:
            raise OracleError("invalid MHD configuration")
        self._cart = Oracle(dim=3, polydeg=polydeg, cells=(cells,) * 3, xmin=(-1,) * 3,
                            xmax=(1,) * 3, gamma=gamma)

    def node_coords(self):
        return self._cart.node_coords()

    def _u(self, u):
        u = _f64(u)
        if u.size != 8 * self.E * self.NN:
            raise ValueError("state has the wrong size")
        return u

    def alfven(self, t=0.0):
        xyz = self.node_coords().reshape(3, -1)
        u = np.stack([mhd_alfven(xyz[:, i], t, self.gamma) for i in range(xyz.shape[1])], axis=1)
        return u.reshape(8, self.E, self.NN)

    def rhs(self, u):
        u = self._u(u)
        du = np.zeros_like(u)
        _check(lib().orc_mhd_rhs(C.byref(self.cfg), _p(u), _p(du)), "mhd_rhs")
        return du.reshape(8, self.E, self.NN)

    def max_dt(self, u, cfl):
        dt = C.c_double(0.0)
        _check(lib().orc_mhd_max_dt(C.byref(self.cfg), _p(self._u(u)), cfl, C.byref(dt)),
               "mhd_max_dt")
        return dt.value

    def step(self, u, nsteps, cfl=0.5, dt_fixed=0.0, t=0.0):
        u = self._u(u).copy()
        tt = C.c_double(t)
        _check(lib().orc_mhd_step(C.byref(self.cfg), _p(u), int(nsteps), cfl, dt_fixed,
                                  C.byref(tt)), "mhd_step")
        return u.reshape(8, self.E, self.NN), tt.value
