"""Python binding of the dgx C ABI (``include/dgx.h``): argument marshalling only.

Every step of the right-hand side, the indicator, the time step and the Runge-Kutta
update runs in the HIP kernels of ``libdgx.so``; PyTorch supplies device memory and the
current stream.  There is no CPU fallback: without the built library (or without a GPU)
every call raises.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgx.so")

VOLUME = {"ec": 0, "central": 1, "shockcap_hg": 2, "weak": 3, "none": 4, "weak_mfma": 5}
SURFACE = {"llf": 0, "hll": 1, "ec": 2, "none": 3}
PRECISION = {"fp64": 0, "mixed": 1}
STATUS = {0: "DGX_OK", 1: "DGX_EINVAL", 2: "DGX_EHIP", 3: "DGX_ENOMEM", 4: "DGX_ENONPHYS",
          5: "DGX_EUNSUPPORTED"}

# every symbol declared in include/dgx.h
EXPORTS = ["dgx_create", "dgx_destroy", "dgx_set_stream", "dgx_num_nodes", "dgx_num_elements",
           "dgx_node_coords", "dgx_rhs", "dgx_indicator", "dgx_rhs_alpha", "dgx_max_dt",
           "dgx_max_dt_noalloc",
           "dgx_step", "dgx_integrals", "dgx_check", "dgx_last_error", "dgx_profile_enable",
           "dgx_profile_read", "dgx_batch_create", "dgx_batch_destroy", "dgx_batch_num_nodes",
           "dgx_batch_step", "dgx_batch_rhs", "dgx_batch_tune", "dgx_batch_set_shape", "dgx_batch_shape",
           "dgx_batch_check", "dgx_batch_last_error", "dgx_create_curved", "dgx_geometry",
           "dgx_create_mhd", "dgx_measure_peak"]


class DgxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class NonPhysicalState(DgxError):
    pass


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("polydeg", C.c_int32), ("cells", C.c_int32 * 3),
                ("xmin", C.c_double * 3), ("xmax", C.c_double * 3), ("gamma", C.c_double),
                ("volume", C.c_int32), ("surface", C.c_int32), ("fv_flux", C.c_int32),
                ("alpha_max", C.c_double), ("alpha_min", C.c_double),
                ("alpha_smooth", C.c_int32), ("precision", C.c_int32)]


class CurvConfig(C.Structure):
    _fields_ = [("polydeg", C.c_int32), ("cells", C.c_int32), ("warp", C.c_double),
                ("gamma", C.c_double), ("volume", C.c_int32), ("surface", C.c_int32),
                ("source", C.c_int32)]


SOURCE = {"none": 0, "mms": 1}


class MhdConfig(C.Structure):
    _fields_ = [("polydeg", C.c_int32), ("cells", C.c_int32), ("gamma", C.c_double),
                ("surface", C.c_int32), ("volume", C.c_int32)]

_lib = None


def lib():
    """Load libdgx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
        sig = {
            "dgx_create": ([C.POINTER(Config), vp, C.POINTER(vp)], C.c_int),
            "dgx_destroy": ([vp], C.c_int),
            "dgx_set_stream": ([vp, vp], C.c_int),
            "dgx_num_nodes": ([vp], i64),
            "dgx_num_elements": ([vp], i64),
            "dgx_node_coords": ([vp, vp], C.c_int),
            "dgx_rhs": ([vp, vp, vp, C.c_double], C.c_int),
            "dgx_indicator": ([vp, vp, vp, vp, vp], C.c_int),
            "dgx_rhs_alpha": ([vp, vp, vp, vp], C.c_int),
            "dgx_max_dt": ([vp, vp, C.c_double, vp], C.c_int),
            "dgx_max_dt_noalloc": ([vp, vp, C.c_double, vp], C.c_int),
            "dgx_step": ([vp, vp, C.c_int32, C.c_double, C.c_double, vp], C.c_int),
            "dgx_integrals": ([vp, vp, vp, vp], C.c_int),
            "dgx_check": ([vp, C.POINTER(C.c_int32)], C.c_int),
            "dgx_last_error": ([vp], C.c_char_p),
            "dgx_profile_enable": ([vp, C.c_int32], C.c_int),
            "dgx_profile_read": ([vp, dp, C.POINTER(i64), C.POINTER(C.c_char_p)], C.c_int),
            "dgx_batch_create": ([C.POINTER(Config), C.c_int32, vp, C.POINTER(vp)], C.c_int),
            "dgx_batch_destroy": ([vp], C.c_int),
            "dgx_batch_num_nodes": ([vp, C.c_int32], i64),
            "dgx_batch_step": ([vp, C.POINTER(vp), C.c_int32, C.c_double, vp], C.c_int),
            "dgx_batch_rhs": ([vp, C.POINTER(vp), C.POINTER(vp)], C.c_int),
            "dgx_batch_tune": ([vp, C.POINTER(vp), C.c_int32], C.c_int),
            "dgx_batch_set_shape": ([vp, C.c_int32, C.c_int32], C.c_int),
            "dgx_batch_shape": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
            "dgx_batch_check": ([vp, C.POINTER(C.c_int32)], C.c_int),
            "dgx_batch_last_error": ([vp], C.c_char_p),
            "dgx_create_curved": ([C.POINTER(CurvConfig), vp, C.POINTER(vp)], C.c_int),
            "dgx_geometry": ([vp, vp, vp], C.c_int),
            "dgx_create_mhd": ([C.POINTER(MhdConfig), vp, C.POINTER(vp)], C.c_int),
            "dgx_measure_peak": ([C.c_int32, C.c_int32, dp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


PEAK_KINDS = {"hbm_copy_GBs": 0, "fp64_fma_TFLOPs": 1}


def measure_peak(kind, device=None):
    """dgx_measure_peak: the measured HBM copy bandwidth (GB/s) or FP64 FMA rate (TFLOP/s)
    of a device (default: torch's current one); blocks while it runs."""
    dev = torch.cuda.current_device() if device is None else int(device)
    v = C.c_double(0.0)
    st = lib().dgx_measure_peak(C.c_int32(dev), C.c_int32(PEAK_KINDS[kind]), C.byref(v))
    if st != 0:
        raise RuntimeError(f"dgx_measure_peak({kind}) failed with status {st}")
    return v.value


def make_config(dim, polydeg, cells, xmin, xmax, gamma=1.4, volume="ec", surface="llf",
                fv_flux="llf", alpha_max=0.5, alpha_min=0.001, alpha_smooth=True,
                precision="fp64", **_ignored):
    c = Config()
    c.dim = dim
    c.polydeg = polydeg
    cells = list(cells) + [1] * (3 - len(cells))
    xmin = list(xmin) + [0.0] * (3 - len(xmin))
    xmax = list(xmax) + [1.0] * (3 - len(xmax))
    for d in range(3):
        c.cells[d] = int(cells[d]) if d < dim else 1
        c.xmin[d] = float(xmin[d])
        c.xmax[d] = float(xmax[d])
    c.gamma = gamma
    c.volume = VOLUME[volume] if isinstance(volume, str) else int(volume)
    c.surface = SURFACE[surface] if isinstance(surface, str) else int(surface)
    c.fv_flux = SURFACE[fv_flux] if isinstance(fv_flux, str) else int(fv_flux)
    c.alpha_max = alpha_max
    c.alpha_min = alpha_min
    c.alpha_smooth = 1 if alpha_smooth else 0
    c.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    return c


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


class Solver:
    """One DGSEM semidiscretisation on the GPU (an opaque dgx handle)."""

    def __init__(self, dim, polydeg, cells, xmin, xmax, **kw):
        self.cfg = make_config(dim, polydeg, cells, xmin, xmax, **kw)
        L = lib()
        h = C.c_void_p()
        st = L.dgx_create(C.byref(self.cfg), _stream(), C.byref(h))
        if st != 0:
            raise DgxError(st, "dgx_create failed (configuration not supported or invalid)")
        self._h = h
        self.dim, self.N = dim, polydeg
        self.n = polydeg + 1
        self.NN = self.n ** dim
        self.nvar = dim + 2
        self.num_nodes = int(L.dgx_num_nodes(h))
        self.E = int(L.dgx_num_elements(h))
        self.shape = (self.nvar, self.E, self.NN)

    def close(self):
        if getattr(self, "_h", None):
            lib().dgx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fname, *args):
        L = lib()
        L.dgx_set_stream(self._h, _stream())
        st = getattr(L, fname)(self._h, *args)
        if st != 0:
            msg = L.dgx_last_error(self._h).decode()
            if st == 4:
                raise NonPhysicalState(st, msg)
            raise DgxError(st, f"{fname}: {msg}")

    def empty_state(self):
        return torch.empty(self.shape, dtype=torch.float64, device="cuda")

    def node_coords(self):
        xyz = torch.empty((self.dim, self.E, self.NN), dtype=torch.float64, device="cuda")
        self._call("dgx_node_coords", _ptr(xyz, "xyz"))
        return xyz

    def rhs(self, u, du=None, t=0.0):
        n = self.nvar * self.num_nodes
        if du is None:
            du = torch.empty_like(u)
        self._call("dgx_rhs", _ptr(u, "u", n), _ptr(du, "du", n), C.c_double(t))
        return du

    def rhs_alpha(self, u, alpha, du=None):
        n = self.nvar * self.num_nodes
        if du is None:
            du = torch.empty_like(u)
        self._call("dgx_rhs_alpha", _ptr(u, "u", n), _ptr(alpha, "alpha", self.E),
                   _ptr(du, "du", n))
        return du

    def indicator(self, u):
        """(alpha, alpha_raw, energy) as device tensors [E]."""
        a = torch.empty(self.E, dtype=torch.float64, device="cuda")
        ar = torch.empty_like(a)
        en = torch.empty_like(a)
        self._call("dgx_indicator", _ptr(u, "u", self.nvar * self.num_nodes), _ptr(a, "alpha"),
                   _ptr(ar, "alpha_raw"), _ptr(en, "energy"))
        return a, ar, en

    def max_dt(self, u, cfl, out=None):
        out = torch.empty(1, dtype=torch.float64, device="cuda") if out is None else out
        self._call("dgx_max_dt", _ptr(u, "u", self.nvar * self.num_nodes), C.c_double(cfl),
                   _ptr(out, "dt"))
        return out

    def max_dt_noalloc(self, u, cfl, out):
        """dgx_max_dt into the caller's device scalar `out` (float64 [1]); the library
        allocates nothing for it (its partials live in a static device array)."""
        self._call("dgx_max_dt_noalloc", _ptr(u, "u", self.nvar * self.num_nodes),
                   C.c_double(cfl), _ptr(out, "dt", 1))
        return out

    def step(self, u, nsteps, cfl=0.5, dt_fixed=0.0, t=None):
        """Advance u in place; t (device float64 [1]) is advanced by every dt."""
        self._call("dgx_step", _ptr(u, "u", self.nvar * self.num_nodes), C.c_int32(nsteps),
                   C.c_double(cfl), C.c_double(dt_fixed), _ptr(t, "t"))
        return u

    def integrals(self, u, du=None):
        out = torch.empty(7, dtype=torch.float64, device="cuda")
        n = self.nvar * self.num_nodes
        self._call("dgx_integrals", _ptr(u, "u", n), _ptr(du, "du", n), _ptr(out, "out7"))
        return out

    def check(self):
        """Synchronise; return 1 if a kernel met a non-physical state since the last check."""
        L = lib()
        f = C.c_int32(0)
        st = L.dgx_check(self._h, C.byref(f))
        if st not in (0, 4):
            raise DgxError(st, L.dgx_last_error(self._h).decode())
        return int(f.value)

    def profile_enable(self, on=True):
        self._call("dgx_profile_enable", C.c_int32(1 if on else 0))

    def profile_read(self):
        avg = C.c_double(0.0)
        n = C.c_int64(0)
        name = C.c_char_p()
        self._call("dgx_profile_read", C.byref(avg), C.byref(n), C.byref(name))
        return avg.value, int(n.value), name.value.decode()


class Batch:
    """An ensemble of independent 3D runs (dgx_batch handle)."""

    def __init__(self, configs):
        L = lib()
        arr = (Config * len(configs))(*[make_config(**c) for c in configs])
        h = C.c_void_p()
        st = L.dgx_batch_create(arr, len(configs), _stream(), C.byref(h))
        if st != 0:
            raise DgxError(st, "dgx_batch_create failed")
        self._h = h
        self.nruns = len(configs)
        self.configs = list(configs)
        self.num_nodes = [int(L.dgx_batch_num_nodes(h, r)) for r in range(self.nruns)]

    def close(self):
        if getattr(self, "_h", None):
            lib().dgx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts, name):
        if len(ts) != self.nruns:
            raise ValueError(f"{name}: need {self.nruns} tensors")
        return (C.c_void_p * self.nruns)(*[_ptr(t, f"{name}[{r}]", 5 * self.num_nodes[r])
                                           for r, t in enumerate(ts)])

    def _call(self, fname, *args):
        st = getattr(lib(), fname)(self._h, *args)
        if st != 0:
            msg = lib().dgx_batch_last_error(self._h).decode()
            raise DgxError(st, f"{fname}: {msg}")

    def step(self, us, nsteps, cfl=0.5, t=None):
        self._call("dgx_batch_step", self._ptrs(us, "u"), C.c_int32(nsteps), C.c_double(cfl),
                   _ptr(t, "t", self.nruns) if t is not None else None)

    def rhs(self, us, dus):
        self._call("dgx_batch_rhs", self._ptrs(us, "u"), self._ptrs(dus, "du"))

    def tune(self, us, budget_ms=2000):
        self._call("dgx_batch_tune", self._ptrs(us, "u"), C.c_int32(budget_ms))
        return self.shape()

    def set_shape(self, block, grid):
        """block: 256 or 512 threads; grid: 0 (one block per work item) or a multiple of 8
        (persistent blocks when below the number of work items)."""
        self._call("dgx_batch_set_shape", C.c_int32(block), C.c_int32(grid))
        return self.shape()

    def shape(self):
        b, g = C.c_int32(0), C.c_int32(0)
        self._call("dgx_batch_shape", C.byref(b), C.byref(g))
        return b.value, g.value

    def check(self):
        f = C.c_int32(0)
        st = lib().dgx_batch_check(self._h, C.byref(f))
        if st not in (0, 4):
            raise DgxError(st, lib().dgx_batch_last_error(self._h).decode())
        return int(f.value)


class CurvSolver(Solver):
    """The warped periodic box of the PID study (cells^3 hexahedra on [-1,1]^3, Eq. (2)),
    EC or central flux differencing, FP64; source="mms" adds the manufactured solution's
    source term (dgx_create_curved)."""

    def __init__(self, polydeg, cells, warp=0.15, gamma=1.4, volume="ec", surface="llf",
                 source="mms"):
        c = CurvConfig()
        c.polydeg, c.cells, c.warp, c.gamma = polydeg, cells, warp, gamma
        c.volume = VOLUME[volume] if isinstance(volume, str) else int(volume)
        c.surface = SURFACE[surface] if isinstance(surface, str) else int(surface)
        c.source = SOURCE[source] if isinstance(source, str) else int(source)
        self.ccfg = c
        L = lib()
        h = C.c_void_p()
        st = L.dgx_create_curved(C.byref(c), _stream(), C.byref(h))
        if st != 0:
            raise DgxError(st, "dgx_create_curved failed (configuration not supported or invalid)")
        self._h = h
        self.dim, self.N = 3, polydeg
        self.n = polydeg + 1
        self.NN = self.n ** 3
        self.nvar = 5
        self.num_nodes = int(L.dgx_num_nodes(h))
        self.E = int(L.dgx_num_elements(h))
        self.shape = (5, self.E, self.NN)

    def geometry(self):
        """(Ja [3][3][E][NN] = (J a^i)_n, J [E][NN]) as device tensors."""
        ja = torch.empty((3, 3, self.E, self.NN), dtype=torch.float64, device="cuda")
        jac = torch.empty((self.E, self.NN), dtype=torch.float64, device="cuda")
        self._call("dgx_geometry", _ptr(ja, "ja"), _ptr(jac, "jac"))
        return ja, jac


class MhdSolver(Solver):
    """Ideal MHD (8 variables) on [-1,1]^3 with cells^3 elements (dgx_create_mhd): weak form
    ("weak", HLL or LLF) or entropy-conservative flux differencing with Powell's term ("ec",
    EC, LLF or HLL surface)."""

    def __init__(self, polydeg, cells, gamma=5.0 / 3.0, surface="hll", volume="weak"):
        c = MhdConfig()
        c.polydeg, c.cells, c.gamma = polydeg, cells, gamma
        c.surface = SURFACE[surface] if isinstance(surface, str) else int(surface)
        c.volume = VOLUME[volume] if isinstance(volume, str) else int(volume)
        self.mcfg = c
        L = lib()
        h = C.c_void_p()
        st = L.dgx_create_mhd(C.byref(c), _stream(), C.byref(h))
        if st != 0:
            raise DgxError(st, "dgx_create_mhd failed (configuration not supported or invalid)")
        self._h = h
        self.dim, self.N = 3, polydeg
        self.n = polydeg + 1
        self.NN = self.n ** 3
        self.nvar = 8
        self.num_nodes = int(L.dgx_num_nodes(h))
        self.E = int(L.dgx_num_elements(h))
        self.shape = (8, self.E, self.NN)
