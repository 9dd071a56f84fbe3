"""ctypes binding of libmb4.so, the MI355X MB4 integrator (include/mb4.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Functions keep the C names; host arrays are numpy float64
arrays, device arrays are raw device pointers (ints), e.g. a torch tensor's
``data_ptr()``.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int, c_int32,
                    c_int64, c_uint32, c_uint64, c_void_p)

import numpy as np

MB4_OK = 0
MB4_EINVAL = -1
MB4_ENOMEM = -2
MB4_EDEVICE = -3
MB4_ENOCONV = -4

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmb4.so")


class mb4_lattice(Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("t_hop", c_double), ("diag_shift", c_double)]


class mb4_nonlinearity(Structure):
    _fields_ = [("g", c_double)]


class mb4_options(Structure):
    _fields_ = [("eps", c_double), ("max_newton", c_int32), ("inner_sweeps", c_int32),
                ("stream", c_void_p), ("mem_budget", c_uint64), ("flags", c_uint32)]


MB4_FLAG_NO_GRAPHS = 1
MB4_FLAG_RELATIVE_EPS = 2
MB4_FLAG_FP32_SOLVE = 4
MB4_FLAG_SPECTRAL_SOLVE = 8

MB4_REGION_32x32 = 0
MB4_REGION_64x16 = 1
MB4_REGION_32x16 = 2
MB4_REGION_COUNT = 3
REGION_NAMES = ("32x32", "64x16", "32x16")


MB4_REQ_QUEUED = 0
MB4_REQ_ACTIVE = 1
MB4_REQ_DONE = 2
MB4_REQ_FAILED = 3


class mb4_request_info(Structure):
    _fields_ = [("status", c_int32), ("nx", c_int32), ("ny", c_int32), ("steps", c_int64),
                ("steps_done", c_int64), ("t_submit", c_double), ("t_admit", c_double),
                ("t_done", c_double), ("energy_start", c_double), ("energy_end", c_double),
                ("last_newton_iters", c_int32), ("error", c_int32)]


class mb4_server_info(Structure):
    _fields_ = [("capacity_sites", c_int64), ("used_sites", c_int64), ("queued", c_int32),
                ("active", c_int32), ("batches", c_int64), ("site_steps", c_double)]


class Mb4Error(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__(f"{where}: {detail or strerror(code)} (code {code})")


_lib = None

_SIGNATURES = {
    "mb4_options_default": (None, [POINTER(mb4_options)]),
    "mb4_create": (c_int, [POINTER(mb4_lattice), POINTER(c_double), POINTER(mb4_nonlinearity),
                           c_double, POINTER(mb4_options), POINTER(c_void_p)]),
    "mb4_destroy": (None, [c_void_p]),
    "mb4_set_state": (c_int, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    "mb4_get_state": (c_int, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    "mb4_set_state_device": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mb4_get_state_device": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mb4_step": (c_int, [c_void_p, c_int64]),
    "mb4_energy": (c_int, [c_void_p, POINTER(c_double)]),
    "mb4_energy_components": (c_int, [c_void_p, POINTER(c_double)]),
    "mb4_energy_components_noalloc": (c_int, [POINTER(mb4_lattice), POINTER(mb4_nonlinearity),
                                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mb4_set_h": (c_int, [c_void_p, c_double]),
    "mb4_set_nonlinearity_sites": (c_int, [c_void_p, POINTER(c_double)]),
    "mb4_set_region": (c_int, [c_void_p, c_int32]),
    "mb4_region": (c_int32, [c_void_p]),
    "mb4_set_sweeps": (c_int, [c_void_p, c_int32]),
    "mb4_sweeps": (c_int32, [c_void_p]),
    "mb4_tune": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32),
                         POINTER(c_double)]),
    "mb4_steps_done": (c_int64, [c_void_p]),
    "mb4_last_stats": (c_int, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_double)]),
    "mb4_newton_update": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "mb4_stage_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_int32]),
    "mb4_last_residuals": (c_int, [c_void_p, POINTER(c_double), c_int32, POINTER(c_int32)]),
    "mb4_profile_enable": (c_int, [c_void_p, c_int32]),
    "mb4_profile_classes": (c_int32, []),
    "mb4_profile_name": (c_char_p, [c_int32]),
    "mb4_profile_read": (c_int, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_double)]),
    "mb4_ensemble_create": (c_int, [c_int32, POINTER(mb4_lattice), POINTER(POINTER(c_double)),
                                    POINTER(mb4_nonlinearity), POINTER(c_double),
                                    POINTER(mb4_options), POINTER(c_void_p)]),
    "mb4_ensemble_destroy": (None, [c_void_p]),
    "mb4_ensemble_size": (c_int32, [c_void_p]),
    "mb4_ensemble_set_state": (c_int, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double)]),
    "mb4_ensemble_get_state": (c_int, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double)]),
    "mb4_ensemble_step": (c_int, [c_void_p, c_int64]),
    "mb4_ensemble_energy_components": (c_int, [c_void_p, POINTER(c_double)]),
    "mb4_ensemble_member_stats": (c_int, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_int32)]),
    "mb4_ensemble_set_region": (c_int, [c_void_p, c_int32]),
    "mb4_ensemble_region": (c_int32, [c_void_p]),
    "mb4_ensemble_tune": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_double)]),
    "mb4_ensemble_set_sweeps": (c_int, [c_void_p, c_int32]),
    "mb4_ensemble_sweeps": (c_int32, [c_void_p]),
    "mb4_ensemble_tune_all": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32),
                                      POINTER(c_double)]),
    "mb4_ensemble_set_persistent": (c_int, [c_void_p, c_int32]),
    "mb4_ensemble_persistent": (c_int32, [c_void_p]),
    "mb4_ensemble_tune_launch": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_double)]),
    "mb4_server_create": (c_int, [c_uint64, c_int32, c_int32, POINTER(mb4_options),
                                  POINTER(c_void_p)]),
    "mb4_server_destroy": (None, [c_void_p]),
    "mb4_server_clock": (c_double, [c_void_p]),
    "mb4_server_submit": (c_int, [c_void_p, POINTER(mb4_lattice), POINTER(c_double),
                                  POINTER(mb4_nonlinearity), c_double, POINTER(c_double),
                                  POINTER(c_double), c_int64, POINTER(c_int64)]),
    "mb4_server_poll": (c_int, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "mb4_server_request": (c_int, [c_void_p, c_int64, POINTER(mb4_request_info)]),
    "mb4_server_result": (c_int, [c_void_p, c_int64, POINTER(c_double), POINTER(c_double)]),
    "mb4_server_release": (c_int, [c_void_p, c_int64]),
    "mb4_server_stats": (c_int, [c_void_p, POINTER(mb4_server_info)]),
    "mb4_strerror": (c_char_p, [c_int]),
    "mb4_error_detail": (c_char_p, []),
}


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Loads libmb4.so (once).  Raises FileNotFoundError if it is not built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(
            f"{p} is missing: build it with `python -m paper_2003_04345_amd._build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().mb4_strerror(code).decode()


def error_detail() -> str:
    return load_library().mb4_error_detail().decode()


def _check(rc: int, where: str) -> int:
    if rc != MB4_OK:
        raise Mb4Error(rc, where, error_detail())
    return rc


def _host(a, n: int) -> np.ndarray:
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.size != n:
        raise ValueError(f"expected {n} values, got {arr.size}")
    return arr


def _dptr(a) -> int:
    return a if isinstance(a, int) else int(a.data_ptr())


def mb4_options_default() -> mb4_options:
    o = mb4_options()
    load_library().mb4_options_default(byref(o))
    return o


def mb4_create(lattice: mb4_lattice, potential, nonlinearity: mb4_nonlinearity, h: float,
               opt: mb4_options | None = None) -> c_void_p:
    """Creates a state; raises Mb4Error on failure (see mb4_create in mb4.h)."""
    n = int(lattice.nx) * int(lattice.ny)
    v = _host(potential, n) if n > 0 else np.zeros(1)
    out = c_void_p()
    rc = load_library().mb4_create(byref(lattice), v.ctypes.data_as(POINTER(c_double)),
                                   byref(nonlinearity), float(h),
                                   byref(opt) if opt is not None else None, byref(out))
    _check(rc, "mb4_create")
    return out


def mb4_destroy(state) -> None:
    load_library().mb4_destroy(state)


def mb4_set_state(state, p, q, sites: int) -> None:
    p = _host(p, sites)
    q = _host(q, sites)
    _check(load_library().mb4_set_state(state, p.ctypes.data_as(POINTER(c_double)),
                                        q.ctypes.data_as(POINTER(c_double))), "mb4_set_state")


def mb4_get_state(state, sites: int) -> tuple[np.ndarray, np.ndarray]:
    p = np.empty(sites)
    q = np.empty(sites)
    _check(load_library().mb4_get_state(state, p.ctypes.data_as(POINTER(c_double)),
                                        q.ctypes.data_as(POINTER(c_double))), "mb4_get_state")
    return p, q


def mb4_set_state_device(state, d_p, d_q) -> None:
    _check(load_library().mb4_set_state_device(state, _dptr(d_p), _dptr(d_q)),
           "mb4_set_state_device")


def mb4_get_state_device(state, d_p, d_q) -> None:
    _check(load_library().mb4_get_state_device(state, _dptr(d_p), _dptr(d_q)),
           "mb4_get_state_device")


def mb4_step(state, nsteps: int) -> int:
    """Returns MB4_OK, or MB4_ENOCONV (not raised: the state stays valid)."""
    rc = load_library().mb4_step(state, int(nsteps))
    if rc not in (MB4_OK, MB4_ENOCONV):
        _check(rc, "mb4_step")
    return rc


def mb4_energy(state) -> float:
    h = c_double()
    _check(load_library().mb4_energy(state, byref(h)), "mb4_energy")
    return h.value


def mb4_energy_components(state) -> dict:
    out = (c_double * 6)()
    _check(load_library().mb4_energy_components(state, out), "mb4_energy_components")
    keys = ("H", "U_K", "U_I", "U_E", "prob", "participation")
    return {k: out[i] for i, k in enumerate(keys)}


def mb4_energy_components_noalloc(nx: int, ny: int, g: float, d_potential, d_p, d_q, d_out,
                                  t_hop: float = 1.0, diag_shift: float = 0.0,
                                  stream: int = 0) -> None:
    """Enqueues the energy components of the device field (d_p, d_q) into the
    device array d_out[6] on `stream`; allocates nothing."""
    lat = mb4_lattice(int(nx), int(ny), float(t_hop), float(diag_shift))
    nl = mb4_nonlinearity(float(g))
    _check(load_library().mb4_energy_components_noalloc(
        byref(lat), byref(nl), _dptr(d_potential), _dptr(d_p), _dptr(d_q), _dptr(d_out),
        c_void_p(int(stream)) if stream else None), "mb4_energy_components_noalloc")


def mb4_set_nonlinearity_sites(state, g, sites: int) -> None:
    """g: nx*ny values g_j, or None for the state's uniform g."""
    if g is None:
        ptr = None
    else:
        arr = _host(g, sites)
        ptr = arr.ctypes.data_as(POINTER(c_double))
    _check(load_library().mb4_set_nonlinearity_sites(state, ptr), "mb4_set_nonlinearity_sites")


def mb4_set_h(state, h: float) -> None:
    _check(load_library().mb4_set_h(state, float(h)), "mb4_set_h")


def mb4_set_region(state, region: int) -> None:
    _check(load_library().mb4_set_region(state, int(region)), "mb4_set_region")


def mb4_region(state) -> int:
    return int(load_library().mb4_region(state))


def mb4_set_sweeps(state, sweeps: int) -> None:
    _check(load_library().mb4_set_sweeps(state, int(sweeps)), "mb4_set_sweeps")


def mb4_sweeps(state) -> int:
    return int(load_library().mb4_sweeps(state))


def mb4_tune(state, steps: int = 32) -> tuple[int, int, dict]:
    """Autotuner of a single state over region and sweeps: (region, sweeps,
    {(region, sweeps): ms per step}) for the pairs timed."""
    region = c_int32()
    sweeps = c_int32()
    ms = (c_double * (4 * MB4_REGION_COUNT))()
    _check(load_library().mb4_tune(state, int(steps), byref(region), byref(sweeps), ms),
           "mb4_tune")
    times = {(r, sw + 1): ms[sw * MB4_REGION_COUNT + r]
             for sw in range(4) for r in range(MB4_REGION_COUNT)
             if ms[sw * MB4_REGION_COUNT + r] >= 0}
    return region.value, sweeps.value, times


def mb4_steps_done(state) -> int:
    return int(load_library().mb4_steps_done(state))


def mb4_last_stats(state) -> dict:
    it = c_int32()
    sw = c_int32()
    rn = c_double()
    _check(load_library().mb4_last_stats(state, byref(it), byref(sw), byref(rn)),
           "mb4_last_stats")
    return {"newton_iters": it.value, "inner_sweeps": sw.value, "last_rnorm": rn.value}


def mb4_last_residuals(state, n: int = 1000) -> list[float]:
    out = (c_double * max(n, 1))()
    cnt = c_int32()
    _check(load_library().mb4_last_residuals(state, out, int(n), byref(cnt)),
           "mb4_last_residuals")
    return [out[i] for i in range(cnt.value)]


def mb4_profile_enable(state, enable: bool = True) -> None:
    _check(load_library().mb4_profile_enable(state, 1 if enable else 0), "mb4_profile_enable")


def mb4_profile_read(state) -> dict:
    """{kernel name: (launches, total milliseconds)} since profiling was enabled."""
    lib = load_library()
    out = {}
    for k in range(lib.mb4_profile_classes()):
        n = c_int64()
        ms = c_double()
        _check(lib.mb4_profile_read(state, k, byref(n), byref(ms)), "mb4_profile_read")
        out[lib.mb4_profile_name(k).decode()] = (n.value, ms.value)
    return out


def mb4_newton_update(state, d_U, d_rbar, d_phibar) -> float:
    rn = c_double()
    rb = None if d_rbar is None else _dptr(d_rbar)
    _check(load_library().mb4_newton_update(state, _dptr(d_U), rb, _dptr(d_phibar), byref(rn)),
           "mb4_newton_update")
    return rn.value


def mb4_stage_solve(state, d_phibar, d_rbar, sweeps: int) -> None:
    _check(load_library().mb4_stage_solve(state, _dptr(d_phibar), _dptr(d_rbar), int(sweeps)),
           "mb4_stage_solve")


class MB4State:
    """Owning wrapper of one mb4_state (destroyed on close or garbage collection)."""

    def __init__(self, nx: int, ny: int, potential, g: float, h: float, t_hop: float = 1.0,
                 diag_shift: float = 0.0, eps: float = 0.0, max_newton: int = 0,
                 inner_sweeps: int = 0, stream: int | None = None, mem_budget: int = 0,
                 graphs: bool = True, relative_eps: bool = False, fp32_solve: bool = False,
                 spectral_solve: bool = False):
        self.nx, self.ny = int(nx), int(ny)
        self.sites = self.nx * self.ny
        opt = mb4_options_default()
        if eps:
            opt.eps = eps
        if max_newton:
            opt.max_newton = max_newton
        if inner_sweeps:
            opt.inner_sweeps = inner_sweeps
        opt.stream = stream
        opt.mem_budget = mem_budget
        opt.flags = ((0 if graphs else MB4_FLAG_NO_GRAPHS) |
                     (MB4_FLAG_RELATIVE_EPS if relative_eps else 0) |
                     (MB4_FLAG_FP32_SOLVE if fp32_solve else 0) |
                     (MB4_FLAG_SPECTRAL_SOLVE if spectral_solve else 0))
        self._h = mb4_create(mb4_lattice(self.nx, self.ny, t_hop, diag_shift), potential,
                             mb4_nonlinearity(g), h, opt)

    @property
    def handle(self):
        return self._h

    def set_state(self, p, q) -> None:
        mb4_set_state(self._h, p, q, self.sites)

    def get_state(self) -> tuple[np.ndarray, np.ndarray]:
        return mb4_get_state(self._h, self.sites)

    def psi(self) -> np.ndarray:
        p, q = self.get_state()
        return p + 1j * q

    def step(self, nsteps: int) -> int:
        return mb4_step(self._h, nsteps)

    def energy(self) -> float:
        return mb4_energy(self._h)

    def energy_components(self) -> dict:
        return mb4_energy_components(self._h)

    def set_nonlinearity_sites(self, g) -> None:
        mb4_set_nonlinearity_sites(self._h, g, self.sites)

    def set_h(self, h: float) -> None:
        mb4_set_h(self._h, h)

    def steps_done(self) -> int:
        return mb4_steps_done(self._h)

    def set_region(self, region: int) -> None:
        mb4_set_region(self._h, region)

    def region(self) -> int:
        return mb4_region(self._h)

    def set_sweeps(self, sweeps: int) -> None:
        mb4_set_sweeps(self._h, sweeps)

    def sweeps(self) -> int:
        return mb4_sweeps(self._h)

    def tune(self, steps: int = 32) -> tuple[int, int, dict]:
        return mb4_tune(self._h, steps)

    def last_stats(self) -> dict:
        return mb4_last_stats(self._h)

    def last_residuals(self) -> list[float]:
        return mb4_last_residuals(self._h)

    def profile_enable(self, enable: bool = True) -> None:
        mb4_profile_enable(self._h, enable)

    def profile_read(self) -> dict:
        return mb4_profile_read(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            mb4_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Ensembles (mb4_ensemble_*).

def mb4_ensemble_create(lattices, potentials, gs, hs, opt: mb4_options | None = None) -> int:
    n = len(lattices)
    if not (len(potentials) == len(gs) == len(hs) == n):
        raise ValueError("lattices, potentials, gs and hs must have the same length")
    lats = (mb4_lattice * n)(*lattices)
    pots = [np.ascontiguousarray(v, dtype=np.float64) for v in potentials]
    for lat, v in zip(lattices, pots):
        if v.size != lat.nx * lat.ny:
            raise ValueError("potential size does not match its lattice")
    ptrs = (POINTER(c_double) * n)(*[v.ctypes.data_as(POINTER(c_double)) for v in pots])
    nls = (mb4_nonlinearity * n)(*[mb4_nonlinearity(float(g)) for g in gs])
    hh = (c_double * n)(*[float(h) for h in hs])
    out = c_void_p()
    _check(load_library().mb4_ensemble_create(n, lats, ptrs, nls, hh,
                                              byref(opt) if opt is not None else None,
                                              byref(out)), "mb4_ensemble_create")
    return out.value


class MB4Ensemble:
    """Owning wrapper of one mb4_ensemble.  members: sequence of objects with
    nx, ny, g, h, t_hop and diag_shift (e.g. lattice_inputs.LatticeProblem);
    potentials: one array of nx*ny values per member."""

    def __init__(self, members, potentials, eps: float = 0.0, max_newton: int = 0,
                 inner_sweeps: int = 0, stream: int | None = None, mem_budget: int = 0,
                 graphs: bool = True, relative_eps: bool = False, fp32_solve: bool = False):
        self.shapes = [(int(m.nx), int(m.ny)) for m in members]
        opt = mb4_options_default()
        if eps:
            opt.eps = eps
        if max_newton:
            opt.max_newton = max_newton
        if inner_sweeps:
            opt.inner_sweeps = inner_sweeps
        opt.stream = stream
        opt.mem_budget = mem_budget
        opt.flags = ((0 if graphs else MB4_FLAG_NO_GRAPHS) |
                     (MB4_FLAG_RELATIVE_EPS if relative_eps else 0) |
                     (MB4_FLAG_FP32_SOLVE if fp32_solve else 0))
        lats = [mb4_lattice(nx, ny, float(getattr(m, "t_hop", 1.0)),
                            float(getattr(m, "diag_shift", 0.0)))
                for (nx, ny), m in zip(self.shapes, members)]
        self._e = mb4_ensemble_create(lats, potentials, [m.g for m in members],
                                      [m.h for m in members], opt)

    @property
    def handle(self):
        return self._e

    def __len__(self) -> int:
        return len(self.shapes)

    def set_state(self, member: int, p, q) -> None:
        nx, ny = self.shapes[member]
        pp = _host(p, nx * ny)
        qq = _host(q, nx * ny)
        _check(load_library().mb4_ensemble_set_state(
            self._e, member, pp.ctypes.data_as(POINTER(c_double)),
            qq.ctypes.data_as(POINTER(c_double))), "mb4_ensemble_set_state")

    def get_state(self, member: int) -> tuple[np.ndarray, np.ndarray]:
        nx, ny = self.shapes[member]
        p = np.empty(nx * ny)
        q = np.empty(nx * ny)
        _check(load_library().mb4_ensemble_get_state(
            self._e, member, p.ctypes.data_as(POINTER(c_double)),
            q.ctypes.data_as(POINTER(c_double))), "mb4_ensemble_get_state")
        return p, q

    def psi(self, member: int) -> np.ndarray:
        p, q = self.get_state(member)
        return p + 1j * q

    def step(self, nsteps: int) -> int:
        """Advances every member; returns the status code (MB4_ENOCONV keeps
        each member's last accepted step)."""
        return load_library().mb4_ensemble_step(self._e, int(nsteps))

    def energy_components(self) -> np.ndarray:
        """(members, 6) array: H, U_K, U_I, U_E, sum |psi|^2, sum |psi|^4."""
        out = np.empty(6 * len(self.shapes))
        _check(load_library().mb4_ensemble_energy_components(
            self._e, out.ctypes.data_as(POINTER(c_double))), "mb4_ensemble_energy_components")
        return out.reshape(-1, 6)

    def energies(self) -> np.ndarray:
        return self.energy_components()[:, 0]

    def member_stats(self, member: int) -> dict:
        done = c_int64()
        iters = c_int32()
        _check(load_library().mb4_ensemble_member_stats(self._e, member, byref(done),
                                                        byref(iters)),
               "mb4_ensemble_member_stats")
        return {"steps_done": done.value, "newton_iters": iters.value}

    def set_region(self, region: int) -> None:
        _check(load_library().mb4_ensemble_set_region(self._e, region), "mb4_ensemble_set_region")

    def region(self) -> int:
        return load_library().mb4_ensemble_region(self._e)

    def tune(self, steps: int = 32) -> tuple[int, list[float]]:
        """Autotuner: (chosen region, ms per step of each region or -1)."""
        best = c_int32()
        ms = (c_double * MB4_REGION_COUNT)()
        _check(load_library().mb4_ensemble_tune(self._e, int(steps), byref(best), ms),
               "mb4_ensemble_tune")
        return best.value, list(ms)

    def set_sweeps(self, sweeps: int) -> None:
        _check(load_library().mb4_ensemble_set_sweeps(self._e, int(sweeps)),
               "mb4_ensemble_set_sweeps")

    def sweeps(self) -> int:
        return load_library().mb4_ensemble_sweeps(self._e)

    def tune_all(self, steps: int = 32) -> tuple[int, int, dict]:
        """Autotuner over region and sweeps: (region, sweeps, {(region,
        sweeps): ms per step}) for the pairs tried."""
        region = c_int32()
        sweeps = c_int32()
        ms = (c_double * (4 * MB4_REGION_COUNT))()
        _check(load_library().mb4_ensemble_tune_all(self._e, int(steps), byref(region),
                                                    byref(sweeps), ms),
               "mb4_ensemble_tune_all")
        times = {(r, sw + 1): ms[sw * MB4_REGION_COUNT + r]
                 for sw in range(4) for r in range(MB4_REGION_COUNT)
                 if ms[sw * MB4_REGION_COUNT + r] >= 0}
        return region.value, sweeps.value, times

    def set_persistent(self, on: bool) -> None:
        """One persistent launch per batch (True) or one launch per Newton
        phase (False, the default); the same results bit for bit."""
        _check(load_library().mb4_ensemble_set_persistent(self._e, 1 if on else 0),
               "mb4_ensemble_set_persistent")

    def persistent(self) -> bool:
        return load_library().mb4_ensemble_persistent(self._e) == 1

    def tune_launch(self, steps: int = 32) -> tuple[bool, list[float]]:
        """Autotuner over the launch form at the current region and sweeps:
        (persistent kept, [ms per step per-phase, persistent])."""
        pe = c_int32()
        ms = (c_double * 2)()
        _check(load_library().mb4_ensemble_tune_launch(self._e, int(steps), byref(pe), ms),
               "mb4_ensemble_tune_launch")
        return pe.value == 1, list(ms)

    def close(self) -> None:
        if getattr(self, "_e", None) is not None:
            load_library().mb4_ensemble_destroy(self._e)
            self._e = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Serving (mb4_server_*).

class MB4Server:
    """Owning wrapper of one mb4_server: a request loop with continuous
    batching.  submit() queues a request, poll() runs one scheduling round
    (admission, one batch of steps for every active request, retirement)."""

    def __init__(self, arena_bytes: int, max_active: int = 256, batch_steps: int = 8,
                 eps: float = 0.0, max_newton: int = 0, inner_sweeps: int = 0,
                 fp32_solve: bool = False, relative_eps: bool = False,
                 stream: int | None = None):
        opt = mb4_options_default()
        if eps:
            opt.eps = eps
        if max_newton:
            opt.max_newton = max_newton
        if inner_sweeps:
            opt.inner_sweeps = inner_sweeps
        opt.stream = stream
        opt.flags = ((MB4_FLAG_FP32_SOLVE if fp32_solve else 0) |
                     (MB4_FLAG_RELATIVE_EPS if relative_eps else 0))
        out = c_void_p()
        _check(load_library().mb4_server_create(int(arena_bytes), int(max_active),
                                                int(batch_steps), byref(opt), byref(out)),
               "mb4_server_create")
        self._s = out.value
        self._shape = {}

    def clock(self) -> float:
        return load_library().mb4_server_clock(self._s)

    def submit(self, problem, potential, p, q, steps: int) -> int:
        """problem: object with nx, ny, g, h (t_hop, diag_shift optional)."""
        nx, ny = int(problem.nx), int(problem.ny)
        n = nx * ny
        lat = mb4_lattice(nx, ny, float(getattr(problem, "t_hop", 1.0)),
                          float(getattr(problem, "diag_shift", 0.0)))
        v = _host(potential, n)
        pp = _host(p, n)
        qq = _host(q, n)
        rid = c_int64()
        _check(load_library().mb4_server_submit(
            self._s, byref(lat), v.ctypes.data_as(POINTER(c_double)),
            byref(mb4_nonlinearity(float(problem.g))), float(problem.h),
            pp.ctypes.data_as(POINTER(c_double)), qq.ctypes.data_as(POINTER(c_double)),
            int(steps), byref(rid)), "mb4_server_submit")
        self._shape[rid.value] = n
        return rid.value

    def poll(self) -> tuple[int, int]:
        queued = c_int32()
        active = c_int32()
        _check(load_library().mb4_server_poll(self._s, byref(queued), byref(active)),
               "mb4_server_poll")
        return queued.value, active.value

    def request(self, rid: int) -> dict:
        info = mb4_request_info()
        _check(load_library().mb4_server_request(self._s, int(rid), byref(info)),
               "mb4_server_request")
        return {name: getattr(info, name) for name, _ in mb4_request_info._fields_}

    def result(self, rid: int) -> tuple[np.ndarray, np.ndarray]:
        n = self._shape[rid]
        p = np.empty(n)
        q = np.empty(n)
        _check(load_library().mb4_server_result(self._s, int(rid),
                                                p.ctypes.data_as(POINTER(c_double)),
                                                q.ctypes.data_as(POINTER(c_double))),
               "mb4_server_result")
        return p, q

    def release(self, rid: int) -> None:
        _check(load_library().mb4_server_release(self._s, int(rid)), "mb4_server_release")
        self._shape.pop(rid, None)

    def stats(self) -> dict:
        info = mb4_server_info()
        _check(load_library().mb4_server_stats(self._s, byref(info)), "mb4_server_stats")
        return {name: getattr(info, name) for name, _ in mb4_server_info._fields_}

    def close(self) -> None:
        if getattr(self, "_s", None) is not None:
            load_library().mb4_server_destroy(self._s)
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
