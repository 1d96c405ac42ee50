"""Thin ctypes binding of libmemd (include/memd.h): the same entry points,
argument marshalling only.

Array arguments may be numpy arrays (host memory), torch tensors (host or
device; their data_ptr() is passed), or raw integer addresses.  Every call
checks the returned status and raises MemdError on failure.  There is no
fallback: without the built HIP library the import of the binding fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmemd.so")

OK, EINVAL, ENOMEM, ENONNEUTRAL, EUNSTABLE, ESTATE, ENOCONV, EDEVICE, ESIZE = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32_MIXED = 0, 1
SELF_GREEN, SELF_DIRECT = 0, 1
EPS_UNIFORM, EPS_SITE, EPS_LINK, EPS_ZSITE = 0, 1, 2, 3
FAMILIES = {"leapfrog": 0, "deposit": 1, "forces": 2, "audit": 3, "energy": 4, "dipole": 5, "salt": 6}


class MemdError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


class memd_params(C.Structure):
    _fields_ = [("L", C.c_int), ("a", C.c_double), ("dt", C.c_double), ("c", C.c_double),
                ("precision", C.c_int), ("audit_every", C.c_int), ("energy_every", C.c_int)]


class memd_energy_t(C.Structure):
    _fields_ = [("W_E", C.c_double), ("W_B", C.c_double), ("U_self", C.c_double),
                ("U_dip", C.c_double), ("E_corrected", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load libmemd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmemd.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, dp = C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_double)
    sigs = {
        "memd_init_lattice": [C.POINTER(vp), C.POINTER(memd_params), i, vp, vp, vp],
        "memd_set_permittivity": [vp, i, vp, d],
        "memd_set_salt_permittivity": [vp, d, d, d, i],
        "memd_initial_gauss_solve": [vp, d, i, C.POINTER(i), dp],
        "memd_step": [vp, vp, i],
        "memd_md_step": [vp, vp, vp, i],
        "memd_forces": [vp, vp],
        "memd_energy": [vp, C.POINTER(memd_energy_t)],
        "memd_gauss_residual": [vp, dp, dp],
        "memd_gauss_residual_noalloc": [i, d, i, vp, vp, vp, i, vp, vp],
        "memd_dipole": [vp, vp],
        "memd_history": [vp, vp, vp, i, C.POINTER(i), C.POINTER(i)],
        "memd_get_state": [vp, vp, vp, vp],
        "memd_set_state": [vp, vp, vp, vp],
        "memd_get_stream": [vp, C.POINTER(vp)],
        "memd_get_params": [vp, dp, vp, dp],
        "memd_profile_enable": [vp, i, i],
        "memd_profile_read": [vp, i, dp, C.POINTER(C.c_long)],
        "memd_set_tiling": [vp, i, i],
        "memd_autotune": [vp, i, C.c_char_p, C.POINTER(i), C.POINTER(i), dp],
        "memd_step_seeded": [vp, C.c_uint64, d, i],
        "memd_set_options": [vp, i, i],
        "memd_set_dipole_correction": [vp, i],
        "memd_set_final_forces": [vp, i],
        "memd_set_self_scheme": [vp, i],
        "memd_counters": [vp, C.POINTER(C.c_ulong), C.POINTER(i)],
        "memd_seeded_displacements": [C.c_uint64, i, i, d, vp],
        "memd_server_create": [C.POINTER(vp), C.c_size_t, i, i, d, C.c_char_p, vp],
        "memd_server_submit": [vp, C.POINTER(memd_params), i, vp, vp, i, vp, i, C.c_uint64, d,
                               C.POINTER(C.c_uint64)],
        "memd_server_progress": [vp, i, C.POINTER(i), C.POINTER(i), C.POINTER(i)],
        "memd_server_poll": [vp, C.c_uint64, C.POINTER(i), vp, C.POINTER(memd_energy_t), dp, dp, dp],
        "memd_server_stats": [vp, C.POINTER(C.c_long), C.POINTER(C.c_long), C.POINTER(C.c_size_t)],
        "memd_server_destroy": [vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.memd_destroy.argtypes = [vp]
    lib.memd_destroy.restype = None
    lib.memd_strerror.argtypes = [C.c_int]
    lib.memd_strerror.restype = C.c_char_p
    lib.memd_version.restype = C.c_int
    lib.memd_server_last_error.argtypes = [vp]
    lib.memd_server_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().memd_strerror(status).decode()


def _check(status: int, where: str):
    if status != OK:
        raise MemdError(status, where)


def _addr(x, dtype=np.float64, writable=False):
    """Address of an array argument (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):  # torch tensor
        import torch
        assert x.dtype == torch.float64 and x.is_contiguous(), "FP64 contiguous tensors only"
        return x.data_ptr()
    assert isinstance(x, np.ndarray) and x.dtype == dtype and x.flags.c_contiguous, \
        "contiguous float64 numpy arrays only"
    if writable:
        assert x.flags.writeable
    return x.ctypes.data


def _f64(x):
    if x is None or isinstance(x, int) or hasattr(x, "data_ptr"):
        return x
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ------------------------------------------------------------ entry points

def memd_init_lattice(params: memd_params, q, r0, hip_stream=None) -> int:
    ctx = C.c_void_p()
    q, r0 = _f64(q), _f64(r0)
    n = (q.numel() if hasattr(q, "numel") else len(q)) if q is not None else 0
    _check(load().memd_init_lattice(C.byref(ctx), C.byref(params), n, _addr(q), _addr(r0),
                                    hip_stream), "memd_init_lattice")
    return ctx.value


def memd_set_permittivity(ctx: int, mode: int, eps, interface_ratio: float = 4.0):
    eps = _f64(eps)
    _check(load().memd_set_permittivity(ctx, mode, _addr(eps), interface_ratio),
           "memd_set_permittivity")


def memd_set_salt_permittivity(ctx: int, eps_w=80.0, slope=15.0, eps_floor=1.0, every=0):
    _check(load().memd_set_salt_permittivity(ctx, eps_w, slope, eps_floor, every),
           "memd_set_salt_permittivity")


def memd_initial_gauss_solve(ctx: int, tol: float = 1e-13, max_iter: int = 0, check=True):
    it = C.c_int(0)
    res = C.c_double(0.0)
    st = load().memd_initial_gauss_solve(ctx, tol, max_iter, C.byref(it), C.byref(res))
    if check:
        _check(st, "memd_initial_gauss_solve")
    return st, it.value, res.value


def memd_step(ctx: int, disp, nsteps: int):
    disp = _f64(disp)
    _check(load().memd_step(ctx, _addr(disp), nsteps), "memd_step")


def memd_forces(ctx: int, F_out):
    _check(load().memd_forces(ctx, _addr(F_out, writable=True)), "memd_forces")
    return F_out


def memd_energy(ctx: int) -> dict:
    e = memd_energy_t()
    _check(load().memd_energy(ctx, C.byref(e)), "memd_energy")
    return e.as_dict()


def memd_gauss_residual(ctx: int):
    m = C.c_double()
    s = C.c_double()
    _check(load().memd_gauss_residual(ctx, C.byref(m), C.byref(s)), "memd_gauss_residual")
    return m.value, s.value


def memd_gauss_residual_noalloc(L: int, a: float, n: int, q, r, D, precision: int, out,
                                hip_stream=None):
    """The allocation-free audit on device buffers.  q, r, D: torch tensors on
    the current device (D FP64 or FP32 as precision says) or raw addresses;
    out: a float64 array of 2 on the host or the device."""
    def dev(x):
        if x is None or isinstance(x, int):
            return x
        return x.data_ptr() if hasattr(x, "data_ptr") else x.ctypes.data
    o = dev(out) if hasattr(out, "data_ptr") or isinstance(out, int) else _addr(out, writable=True)
    _check(load().memd_gauss_residual_noalloc(L, a, n, dev(q), dev(r), dev(D), precision, o, hip_stream),
           "memd_gauss_residual_noalloc")
    return out


def memd_dipole(ctx: int) -> np.ndarray:
    P = np.zeros(3)
    _check(load().memd_dipole(ctx, _addr(P)), "memd_dipole")
    return P


def memd_history(ctx: int, max_entries: int = 4096):
    na = C.c_int()
    ne = C.c_int()
    A = np.zeros(2 * max_entries)
    E = np.zeros(5 * max_entries)
    _check(load().memd_history(ctx, _addr(A), _addr(E), max_entries, C.byref(na), C.byref(ne)),
           "memd_history")
    ka, ke = min(na.value, max_entries), min(ne.value, max_entries)
    return A[:2 * ka].reshape(ka, 2), E[:5 * ke].reshape(ke, 5)


def memd_get_state(ctx: int, D=None, B=None, r=None):
    _check(load().memd_get_state(ctx, _addr(D, writable=True), _addr(B, writable=True),
                                 _addr(r, writable=True)), "memd_get_state")
    return D, B, r


def memd_set_state(ctx: int, D=None, B=None, r=None):
    D, B, r = _f64(D), _f64(B), _f64(r)
    _check(load().memd_set_state(ctx, _addr(D), _addr(B), _addr(r)), "memd_set_state")


def memd_get_stream(ctx: int) -> int:
    s = C.c_void_p()
    _check(load().memd_get_stream(ctx, C.byref(s)), "memd_get_stream")
    return s.value or 0


def memd_get_params(ctx: int):
    c = C.c_double()
    eh = np.zeros(3)
    em = C.c_double()
    _check(load().memd_get_params(ctx, C.byref(c), _addr(eh), C.byref(em)), "memd_get_params")
    return c.value, eh, em.value


def memd_profile_enable(ctx: int, families=None, every: int = 1):
    """Time the kernel families named in `families` (all when None, none when
    empty) on one launch in `every`."""
    if families is None:
        mask = -1
    else:
        mask = 0
        for f in families:
            mask |= 1 << (FAMILIES[f] if isinstance(f, str) else int(f))
    _check(load().memd_profile_enable(ctx, mask, every), "memd_profile_enable")


def memd_profile_read(ctx: int, family) -> tuple:
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    ms = C.c_double()
    cnt = C.c_long()
    _check(load().memd_profile_read(ctx, fam, C.byref(ms), C.byref(cnt)), "memd_profile_read")
    return ms.value, cnt.value


def memd_set_tiling(ctx: int, rows_per_thread: int = 0, planes_per_chunk: int = 0):
    _check(load().memd_set_tiling(ctx, rows_per_thread, planes_per_chunk), "memd_set_tiling")


def memd_autotune(ctx: int, reps: int = 10, cache_path: str | None = None):
    rr = C.c_int()
    pp = C.c_int()
    us = C.c_double()
    path = cache_path.encode() if cache_path else None
    _check(load().memd_autotune(ctx, reps, path, C.byref(rr), C.byref(pp), C.byref(us)),
           "memd_autotune")
    return rr.value, pp.value, us.value


def memd_set_options(ctx: int, fuse_deposit: int = 1, sort_every: int = 64):
    _check(load().memd_set_options(ctx, int(fuse_deposit), int(sort_every)), "memd_set_options")


def memd_set_final_forces(ctx: int, on: bool):
    _check(load().memd_set_final_forces(ctx, 1 if on else 0), "memd_set_final_forces")


def memd_set_dipole_correction(ctx: int, on: bool):
    _check(load().memd_set_dipole_correction(ctx, 1 if on else 0), "memd_set_dipole_correction")


def memd_set_self_scheme(ctx: int, scheme: int):
    _check(load().memd_set_self_scheme(ctx, int(scheme)), "memd_set_self_scheme")


def memd_counters(ctx: int):
    b = C.c_ulong()
    f = C.c_int()
    _check(load().memd_counters(ctx, C.byref(b), C.byref(f)), "memd_counters")
    return b.value, f.value


def memd_md_step(ctx: int, v, mass, nsteps: int):
    """Velocity-Verlet steps of the ions under their MEMD forces; v (3n
    doubles, host numpy or device tensor) is updated in place."""
    _check(load().memd_md_step(ctx, _addr(v, writable=True), _addr(mass), int(nsteps)), "memd_md_step")


def memd_step_seeded(ctx: int, seed: int, sigma: float, nsteps: int):
    _check(load().memd_step_seeded(ctx, int(seed), float(sigma), int(nsteps)), "memd_step_seeded")


def memd_seeded_displacements(seed: int, step: int, n: int, sigma: float) -> np.ndarray:
    out = np.zeros(3 * n)
    _check(load().memd_seeded_displacements(int(seed), int(step), int(n), float(sigma), _addr(out)),
           "memd_seeded_displacements")
    return out.reshape(n, 3)


# ---------------------------------------------------------------- serving

REQ_PENDING, REQ_INIT, REQ_READY, REQ_ACTIVE, REQ_DONE, REQ_FAILED = range(6)


def memd_server_create(hbm_budget_bytes: int, max_slots: int = 512, init_workers: int = 4,
                       solve_tol: float = 1e-8, tune_cache: str | None = None, hip_stream=None) -> int:
    srv = C.c_void_p()
    _check(load().memd_server_create(C.byref(srv), int(hbm_budget_bytes), int(max_slots),
                                     int(init_workers), float(solve_tol),
                                     tune_cache.encode() if tune_cache else None, hip_stream),
           "memd_server_create")
    return srv.value


def memd_server_submit(srv: int, params: memd_params, q, r0, eps_mode: int, eps, nsteps: int,
                       seed: int, sigma: float) -> int:
    q, r0, eps = _f64(q), _f64(r0), _f64(np.atleast_1d(eps))
    rid = C.c_uint64()
    _check(load().memd_server_submit(srv, C.byref(params), len(q), _addr(q), _addr(r0), eps_mode,
                                     _addr(eps), int(nsteps), int(seed), float(sigma), C.byref(rid)),
           "memd_server_submit")
    return rid.value


def memd_server_progress(srv: int, global_steps: int):
    a, p, f = C.c_int(), C.c_int(), C.c_int()
    st = load().memd_server_progress(srv, int(global_steps), C.byref(a), C.byref(p), C.byref(f))
    if st != OK:
        raise MemdError(st, "memd_server_progress (" + memd_server_last_error(srv) + ")")
    return a.value, p.value, f.value


def memd_server_last_error(srv: int) -> str:
    return (load().memd_server_last_error(srv) or b"").decode()


def memd_server_poll(srv: int, req_id: int, n: int):
    """Returns (state, status, F (n,3) or None, energy dict or None, gauss, t_arrival, t_done)."""
    st = C.c_int()
    F = np.zeros(3 * max(n, 1))
    E = memd_energy_t()
    g, ta, td = C.c_double(), C.c_double(), C.c_double()
    status = load().memd_server_poll(srv, int(req_id), C.byref(st), _addr(F), C.byref(E), C.byref(g),
                                     C.byref(ta), C.byref(td))
    done = st.value == REQ_DONE
    return (st.value, status, F[:3 * n].reshape(n, 3) if done else None,
            E.as_dict() if done else None, g.value, ta.value, td.value)


def memd_server_stats(srv: int):
    gs, rs, by = C.c_long(), C.c_long(), C.c_size_t()
    _check(load().memd_server_stats(srv, C.byref(gs), C.byref(rs), C.byref(by)), "memd_server_stats")
    return gs.value, rs.value, by.value


def memd_server_destroy(srv: int):
    if srv:
        _check(load().memd_server_destroy(srv), "memd_server_destroy")


def memd_destroy(ctx: int):
    if ctx:
        load().memd_destroy(ctx)


def memd_version() -> int:
    return load().memd_version()


def make_params(L, a=1.0, dt=0.01, c=0.0, precision=FP64, audit_every=0, energy_every=0):
    return memd_params(int(L), float(a), float(dt), float(c), int(precision), int(audit_every),
                       int(energy_every))


class Context:
    """Owning wrapper around a memd_ctx handle (convenience for tests and the bench)."""

    def __init__(self, L, q, r0, a=1.0, dt=0.01, c=0.0, precision=FP64, audit_every=0,
                 energy_every=0, stream=None):
        self.params = make_params(L, a, dt, c, precision, audit_every, energy_every)
        self.L = int(L)
        self.n = len(q) if not hasattr(q, "numel") else q.numel()
        self.Ns = self.L ** 3
        self.ctx = memd_init_lattice(self.params, q, r0, stream)

    def close(self):
        if self.ctx:
            memd_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_permittivity(self, mode, eps, ratio=4.0):
        memd_set_permittivity(self.ctx, mode, np.atleast_1d(np.asarray(eps, dtype=np.float64)), ratio)

    def set_salt(self, eps_w=80.0, slope=15.0, eps_floor=1.0, every=0):
        memd_set_salt_permittivity(self.ctx, eps_w, slope, eps_floor, every)

    def solve(self, tol=1e-13, max_iter=0, check=True):
        return memd_initial_gauss_solve(self.ctx, tol, max_iter, check)

    def step(self, disp, nsteps=None):
        if nsteps is None:
            nsteps = 1 if getattr(disp, "ndim", 1) <= 2 else disp.shape[0]
        memd_step(self.ctx, disp, nsteps)

    def md_step(self, v, mass, nsteps=1):
        """Velocity-Verlet steps; v ([n, 3] float64, host or device) is updated in place."""
        memd_md_step(self.ctx, v, mass, nsteps)

    def forces(self) -> np.ndarray:
        F = np.zeros(3 * self.n)
        memd_forces(self.ctx, F)
        return F.reshape(self.n, 3)

    def energy(self) -> dict:
        return memd_energy(self.ctx)

    def gauss_residual(self):
        return memd_gauss_residual(self.ctx)

    def dipole(self):
        return memd_dipole(self.ctx)

    def state(self):
        D = np.zeros(3 * self.Ns)
        B = np.zeros(3 * self.Ns)
        r = np.zeros(3 * self.n)
        memd_get_state(self.ctx, D, B, r)
        return D, B, r

    def set_state(self, D=None, B=None, r=None):
        memd_set_state(self.ctx, D, B, r)

    def history(self, max_entries=4096):
        return memd_history(self.ctx, max_entries)

    def set_dipole_correction(self, on: bool):
        memd_set_dipole_correction(self.ctx, on)

    def set_final_forces(self, on: bool):
        memd_set_final_forces(self.ctx, on)

    def set_self_scheme(self, scheme: int):
        memd_set_self_scheme(self.ctx, scheme)

    def params_in_use(self):
        return memd_get_params(self.ctx)
