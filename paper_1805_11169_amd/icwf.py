"""Python binding of the ICWF C ABI (include/icwf.h): argument marshalling only.

Every step of the method runs in libicwf.so's HIP kernels.  PyTorch provides
the device workspace (one uint8 tensor) and the HIP stream; nothing is
computed here.  If the library is not built, or no GPU is present, the calls
raise -- there is no fallback.
"""

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libicwf.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ENODE, ESOLVE, ESTATE, ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6, -7, -8
MODEL_SHIN_METIU, MODEL_CAVITY = 1, 2
PREC_FP64, PREC_MIXED, PREC_SEPARABLE = 0, 1, 2
SOLVER_AUTO, SOLVER_TRIANGULAR, SOLVER_INVERSE = 0, 1, 2
PROP_SPLIT, PROP_CRANK_NICOLSON = 0, 1
TRAJ_EULER, TRAJ_HEUN = 0, 1

# the entry points include/icwf.h declares
EXPORTS = ("icwf_workspace_bytes", "icwf_create", "icwf_step", "icwf_step_batch", "icwf_sync", "icwf_observables",
           "icwf_get_state", "icwf_get_matrices", "icwf_velocities", "icwf_set_timing", "icwf_kernel_time",
           "icwf_contraction_rank",
           "icwf_destroy", "icwf_last_error", "icwf_status_string")
# the entry points include/icwf_serve.h declares
SERVE_EXPORTS = ("icwf_server_create", "icwf_server_submit", "icwf_server_wait", "icwf_server_result",
                 "icwf_server_get_stats", "icwf_server_clock", "icwf_server_destroy")
# the entry points include/icwf_exact.h declares
EXACT_EXPORTS = ("icwf_exact_workspace_bytes", "icwf_exact_create", "icwf_exact_step", "icwf_exact_observables",
                 "icwf_exact_get_psi", "icwf_exact_destroy", "icwf_grid_observables_noalloc")
# the entry points include/icwf_bo.h declares
BO_EXPORTS = ("icwf_bo_workspace_bytes", "icwf_bo_states")
BO_MAX_STATES = 8


class Config(ctypes.Structure):
    _fields_ = [("n_traj", c_int32), ("n_r", c_int32), ("n_R", c_int32),
                ("r_min", c_double), ("r_max", c_double), ("R_min", c_double), ("R_max", c_double),
                ("m_r", c_double), ("m_R", c_double), ("dt", c_double),
                ("model", c_int32), ("model_params", c_double * 8), ("tikhonov_eps", c_double),
                ("precision", c_int32), ("n_bo", c_int32), ("solver", c_int32),
                ("propagator", c_int32), ("trajectories", c_int32)]


_DP = POINTER(c_double)


class Obs(ctypes.Structure):
    _fields_ = [("t", c_double), ("step", c_int64), ("norm", c_double),
                ("rho_r", _DP), ("rho_R", _DP), ("pop", _DP), ("D", _DP),
                ("r", _DP), ("R", _DP), ("C", _DP),
                ("n_out_of_box", c_int32), ("min_abs_psi", c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_active", c_int32), ("steps_per_turn", c_int32), ("turns_ahead", c_int32),
                ("device", c_int32), ("batch", c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", c_int64), ("status", c_int32), ("slot", c_int32), ("steps", c_int64),
                ("t_submit", c_double), ("t_admit", c_double), ("t_done", c_double),
                ("workspace_bytes", c_size_t), ("message", ctypes.c_char * 192)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("admitted", c_int64), ("completed", c_int64), ("failed", c_int64),
                ("active", c_int32), ("pending", c_int32), ("arena_bytes", c_size_t),
                ("arena_in_use", c_size_t), ("arena_peak", c_size_t), ("peak_active", c_int32)]


class BoInfo(ctypes.Structure):
    _fields_ = [("tol", c_double), ("max_iter", c_int32), ("iterations", c_int32), ("max_residual", c_double),
                ("unconverged", c_int32)]


class ICWFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libicwf.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1805_11169_amd.build`")
        # torch first: its HIP runtime (same soname) then also serves libicwf.so, so the
        # workspace, the streams and the kernels live in one runtime instance
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.icwf_workspace_bytes.argtypes = [POINTER(Config)]
        L.icwf_workspace_bytes.restype = c_size_t
        L.icwf_create.argtypes = [POINTER(Config), _DP, _DP, _DP, _DP, _DP, _DP, _DP, c_void_p, c_size_t,
                                  c_void_p, POINTER(c_void_p)]
        L.icwf_create.restype = c_int32
        L.icwf_step.argtypes = [c_void_p, c_int32]
        L.icwf_step.restype = c_int32
        L.icwf_step_batch.argtypes = [POINTER(c_void_p), c_int32, c_int32]
        L.icwf_step_batch.restype = c_int32
        L.icwf_sync.argtypes = [c_void_p]
        L.icwf_sync.restype = c_int32
        L.icwf_observables.argtypes = [c_void_p, POINTER(Obs)]
        L.icwf_observables.restype = c_int32
        L.icwf_get_state.argtypes = [c_void_p, _DP, _DP, _DP, _DP, _DP]
        L.icwf_get_state.restype = c_int32
        L.icwf_get_matrices.argtypes = [c_void_p, _DP, _DP, _DP]
        L.icwf_get_matrices.restype = c_int32
        L.icwf_velocities.argtypes = [c_void_p, _DP, _DP, _DP]
        L.icwf_velocities.restype = c_int32
        L.icwf_set_timing.argtypes = [c_void_p, c_int32]
        L.icwf_set_timing.restype = c_int32
        L.icwf_kernel_time.argtypes = [c_void_p, c_char_p, POINTER(c_int64), POINTER(c_double)]
        L.icwf_kernel_time.restype = c_int32
        L.icwf_contraction_rank.argtypes = [c_void_p, POINTER(c_int32)]
        L.icwf_contraction_rank.restype = c_int32
        L.icwf_destroy.argtypes = [c_void_p]
        L.icwf_destroy.restype = None
        L.icwf_last_error.argtypes = [c_void_p]
        L.icwf_last_error.restype = c_char_p
        L.icwf_status_string.argtypes = [c_int32]
        L.icwf_status_string.restype = c_char_p
        L.icwf_server_create.argtypes = [POINTER(ServerConfig), c_void_p, c_size_t, POINTER(c_void_p)]
        L.icwf_server_create.restype = c_int32
        L.icwf_server_submit.argtypes = [c_void_p, POINTER(Config), _DP, _DP, _DP, _DP, _DP, _DP, _DP, c_int32,
                                         POINTER(c_int64)]
        L.icwf_server_submit.restype = c_int32
        L.icwf_server_wait.argtypes = [c_void_p, c_int64, c_double]
        L.icwf_server_wait.restype = c_int32
        L.icwf_server_result.argtypes = [c_void_p, c_int64, POINTER(Obs), POINTER(RequestInfo)]
        L.icwf_server_result.restype = c_int32
        L.icwf_server_get_stats.argtypes = [c_void_p, POINTER(ServerStats)]
        L.icwf_server_get_stats.restype = c_int32
        L.icwf_server_clock.argtypes = [c_void_p]
        L.icwf_server_clock.restype = c_double
        L.icwf_server_destroy.argtypes = [c_void_p]
        L.icwf_server_destroy.restype = None
        L.icwf_exact_workspace_bytes.argtypes = [POINTER(Config)]
        L.icwf_exact_workspace_bytes.restype = c_size_t
        L.icwf_exact_create.argtypes = [POINTER(Config), _DP, _DP, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
        L.icwf_exact_create.restype = c_int32
        L.icwf_exact_step.argtypes = [c_void_p, c_int64]
        L.icwf_exact_step.restype = c_int32
        L.icwf_exact_observables.argtypes = [c_void_p, POINTER(Obs)]
        L.icwf_exact_observables.restype = c_int32
        L.icwf_exact_get_psi.argtypes = [c_void_p, _DP]
        L.icwf_exact_get_psi.restype = c_int32
        L.icwf_exact_destroy.argtypes = [c_void_p]
        L.icwf_exact_destroy.restype = None
        L.icwf_grid_observables_noalloc.argtypes = [c_int32, c_int32, c_double, c_double, c_int32, c_void_p, c_void_p,
                                                    c_void_p, c_void_p]
        L.icwf_grid_observables_noalloc.restype = c_int32
        L.icwf_bo_workspace_bytes.argtypes = [POINTER(Config), c_int32, c_int32]
        L.icwf_bo_workspace_bytes.restype = c_size_t
        L.icwf_bo_states.argtypes = [POINTER(Config), _DP, c_int32, c_int32, _DP, _DP, c_void_p, c_size_t, c_void_p,
                                     POINTER(BoInfo)]
        L.icwf_bo_states.restype = c_int32
        _lib = L
    return _lib


def status_string(st):
    return lib().icwf_status_string(st).decode()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a, n=None):
    """Contiguous float64 view; complex arrays become interleaved (re, im)."""
    if a is None:
        return None
    a = np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a, dtype=np.complex128).view(np.float64)
    else:
        a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def make_config(n_traj, n_r, n_R, r_box, R_box, m_r, m_R, dt, model, model_params, eps=1e-8,
                precision=PREC_FP64, n_bo=0, solver=SOLVER_AUTO, propagator=PROP_SPLIT, trajectories=TRAJ_EULER):
    c = Config()
    c.n_traj, c.n_r, c.n_R = int(n_traj), int(n_r), int(n_R)
    c.r_min, c.r_max = float(r_box[0]), float(r_box[1])
    c.R_min, c.R_max = float(R_box[0]), float(R_box[1])
    c.m_r, c.m_R, c.dt = float(m_r), float(m_R), float(dt)
    c.model = int(model)
    params = list(model_params) + [0.0] * (8 - len(model_params))
    for i in range(8):
        c.model_params[i] = float(params[i])
    c.tikhonov_eps = float(eps)
    c.precision = int(precision)
    c.n_bo = int(n_bo)
    c.solver = int(solver)
    c.propagator = int(propagator)
    c.trajectories = int(trajectories)
    return c


def config_from_workload(wl, precision=PREC_FP64, eps=None, solver=SOLVER_AUTO, propagator=PROP_SPLIT,
                         trajectories=TRAJ_EULER):
    return make_config(wl.n_traj, wl.n_r, wl.n_R, (wl.r_min, wl.r_max), (wl.R_min, wl.R_max), wl.m_r, wl.m_R,
                       wl.dt, wl.model, wl.model_params, wl.eps if eps is None else eps, precision, wl.n_bo,
                       solver, propagator, trajectories)


def workspace_bytes(cfg):
    return int(lib().icwf_workspace_bytes(byref(cfg)))


def step_batch(sims, n_steps=1):
    """icwf_step_batch over Simulation objects that share a stream."""
    arr = (c_void_p * len(sims))(*[sm.h for sm in sims])
    st = lib().icwf_step_batch(arr, len(sims), int(n_steps))
    if st != OK:
        lead = sims[0].h if sims else None
        raise ICWFError(st, lib().icwf_last_error(lead).decode())


def bo_workspace_bytes(cfg, n_values, n_states):
    return int(lib().icwf_bo_workspace_bytes(byref(cfg), int(n_values), int(n_states)))


def bo_states(cfg, R_values, n_states, tol=0.0, max_iter=0, device=0, check=True):
    """The n_states lowest eigenpairs of h_e(R_j) for every R_j (include/icwf_bo.h):
    returns (states [n_values][n_states][n_r], energies [n_values][n_states],
    info dict with iterations, max_residual, unconverged, status)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the ICWF library needs a GPU; none is visible")
    L = lib()
    Rv = np.ascontiguousarray(R_values, dtype=np.float64)
    nv = Rv.size
    nbytes = L.icwf_bo_workspace_bytes(byref(cfg), nv, int(n_states))
    if nbytes == 0:
        raise ICWFError(EINVAL, "invalid arguments to icwf_bo_states")
    dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    aligned = (ws.data_ptr() + 255) & ~255
    stream = torch.cuda.current_stream(dev)
    states = np.zeros((nv, int(n_states), cfg.n_r))
    energies = np.zeros((nv, int(n_states)))
    info = BoInfo(float(tol), int(max_iter), 0, 0.0, 0)
    st = L.icwf_bo_states(byref(cfg), _ptr(Rv), nv, int(n_states), _ptr(states), _ptr(energies), c_void_p(aligned),
                          c_size_t(nbytes), c_void_p(stream.cuda_stream), byref(info))
    del ws
    out = dict(iterations=info.iterations, max_residual=info.max_residual, unconverged=info.unconverged, status=st)
    if check and st != OK:
        raise ICWFError(st, L.icwf_last_error(None).decode())
    return states, energies, out


def grid_observables_noalloc(n_r, n_R, h_r, h_R, n_bo, psi_ptr, bo_ptr, out_ptr, stream_ptr):
    """icwf_grid_observables_noalloc on caller-held device pointers (ints); returns the status."""
    return int(lib().icwf_grid_observables_noalloc(int(n_r), int(n_R), float(h_r), float(h_R), int(n_bo),
                                                   c_void_p(psi_ptr), c_void_p(bo_ptr) if bo_ptr else None,
                                                   c_void_p(out_ptr), c_void_p(stream_ptr)))


class Simulation:
    """One ICWF simulation on one GPU (icwf_create ... icwf_destroy)."""

    def __init__(self, cfg, r0, R0, psi1, psi2, C0=None, b0=None, bo=None, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the ICWF library needs a GPU; none is visible")
        L = lib()
        self.cfg = cfg
        self.N, self.n_r, self.n_R, self.n_bo = cfg.n_traj, cfg.n_r, cfg.n_R, cfg.n_bo
        nbytes = L.icwf_workspace_bytes(byref(cfg))
        if nbytes == 0:
            raise ICWFError(EINVAL, "invalid configuration")
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        keep = [_f64(r0), _f64(R0), _f64(psi1), _f64(psi2), _f64(C0), _f64(b0), _f64(bo)]
        handle = c_void_p()
        st = L.icwf_create(byref(cfg), *[_ptr(a) for a in keep], c_void_p(aligned), c_size_t(nbytes),
                           c_void_p(self.stream.cuda_stream), byref(handle))
        if st != OK:
            raise ICWFError(st, L.icwf_last_error(None).decode())
        self.h = handle

    @classmethod
    def from_workload(cls, wl, precision=PREC_FP64, C0=None, solver=SOLVER_AUTO, propagator=PROP_SPLIT,
                      trajectories=TRAJ_EULER, **kw):
        cfg = config_from_workload(wl, precision, solver=solver, propagator=propagator, trajectories=trajectories)
        return cls(cfg, wl.r0, wl.R0, wl.psi1, wl.psi2, C0=C0, b0=None if C0 is not None else wl.b0,
                   bo=wl.bo, **kw)

    def _check(self, st):
        if st != OK:
            raise ICWFError(st, lib().icwf_last_error(self.h).decode())
        return st

    def step(self, n=1):
        self._check(lib().icwf_step(self.h, int(n)))

    def sync(self):
        return self._check(lib().icwf_sync(self.h))

    def observables(self, check=True):
        N, nr, nR, nb = self.N, self.n_r, self.n_R, self.n_bo
        out = dict(rho_r=np.zeros(nr), rho_R=np.zeros(nR), pop=np.zeros(max(nb, 1)),
                   D=np.zeros(max(nb * nb, 1)), r=np.zeros(N), R=np.zeros(N), C=np.zeros(2 * N))
        o = Obs()
        for k, v in out.items():
            setattr(o, k, _ptr(v))
        st = lib().icwf_observables(self.h, byref(o))
        if check:
            self._check(st)
        res = dict(t=o.t, step=o.step, norm=o.norm, rho_r=out["rho_r"], rho_R=out["rho_R"],
                   r=out["r"], R=out["R"], C=out["C"].view(np.complex128), n_out_of_box=o.n_out_of_box,
                   min_abs_psi=o.min_abs_psi, status=st)
        if nb:
            res["pop"] = out["pop"][:nb]
            res["D"] = out["D"][:nb * nb].reshape(nb, nb)
        return res

    def state(self):
        N, nr, nR = self.N, self.n_r, self.n_R
        r, R = np.zeros(N), np.zeros(N)
        p1, p2 = np.zeros((N, nr), np.complex128), np.zeros((N, nR), np.complex128)
        C = np.zeros(N, np.complex128)
        self._check(lib().icwf_get_state(self.h, _ptr(r), _ptr(R), _ptr(p1.view(np.float64)),
                                         _ptr(p2.view(np.float64)), _ptr(C.view(np.float64))))
        return dict(r=r, R=R, psi1=p1, psi2=p2, C=C)

    def matrices(self):
        N = self.N
        S, K, W = (np.zeros((N, N), np.complex128) for _ in range(3))
        self._check(lib().icwf_get_matrices(self.h, _ptr(S.view(np.float64)), _ptr(K.view(np.float64)),
                                            _ptr(W.view(np.float64))))
        return S, K, W

    def velocities(self):
        N = self.N
        vr, vR = np.zeros(N), np.zeros(N)
        pa = np.zeros(N, np.complex128)
        self._check(lib().icwf_velocities(self.h, _ptr(vr), _ptr(vR), _ptr(pa.view(np.float64))))
        return vr, vR, pa

    def set_timing(self, enable):
        self._check(lib().icwf_set_timing(self.h, 1 if enable else 0))

    def kernel_time(self, name):
        n, ms = c_int64(), c_double()
        self._check(lib().icwf_kernel_time(self.h, name.encode(), byref(n), byref(ms)))
        return n.value, ms.value

    def contraction_rank(self):
        k = c_int32()
        self._check(lib().icwf_contraction_rank(self.h, byref(k)))
        return k.value

    def close(self):
        if getattr(self, "h", None):
            lib().icwf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ExactPropagator:
    """Grid propagation of the full wavefunction Psi(r_i, R_j) (include/icwf_exact.h):
    the reference the ansatz converges to.  psi0 is [n_r][n_R] complex."""

    def __init__(self, cfg, psi0, bo=None, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the ICWF library needs a GPU; none is visible")
        L = lib()
        self.cfg = cfg
        self.n_r, self.n_R, self.n_bo = cfg.n_r, cfg.n_R, cfg.n_bo
        nbytes = L.icwf_exact_workspace_bytes(byref(cfg))
        if nbytes == 0:
            raise ICWFError(EINVAL, "invalid configuration")
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self.ws.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        p0 = np.ascontiguousarray(psi0, dtype=np.complex128)
        if p0.shape != (cfg.n_r, cfg.n_R):
            raise ValueError(f"psi0 must be [{cfg.n_r}][{cfg.n_R}]")
        keep = [_f64(p0), _f64(bo)]
        handle = c_void_p()
        st = L.icwf_exact_create(byref(cfg), _ptr(keep[0]), _ptr(keep[1]), c_void_p(aligned), c_size_t(nbytes),
                                 c_void_p(self.stream.cuda_stream), byref(handle))
        if st != OK:
            raise ICWFError(st, L.icwf_last_error(None).decode())
        self.h = handle

    def _check(self, st):
        if st != OK:
            raise ICWFError(st, lib().icwf_last_error(None).decode())
        return st

    def step(self, n=1):
        self._check(lib().icwf_exact_step(self.h, int(n)))

    def observables(self):
        nr, nR, nb = self.n_r, self.n_R, self.n_bo
        out = dict(rho_r=np.zeros(nr), rho_R=np.zeros(nR), pop=np.zeros(max(nb, 1)), D=np.zeros(max(nb * nb, 1)))
        o = Obs()
        for k, v in out.items():
            setattr(o, k, _ptr(v))
        self._check(lib().icwf_exact_observables(self.h, byref(o)))
        res = dict(t=o.t, step=o.step, norm=o.norm, rho_r=out["rho_r"], rho_R=out["rho_R"])
        if nb:
            res["pop"] = out["pop"][:nb]
            res["D"] = out["D"][:nb * nb].reshape(nb, nb)
        return res

    def psi(self):
        p = np.zeros((self.n_r, self.n_R), np.complex128)
        self._check(lib().icwf_exact_get_psi(self.h, _ptr(p.view(np.float64))))
        return p

    def close(self):
        if getattr(self, "h", None):
            lib().icwf_exact_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching of independent simulations (include/icwf_serve.h).

    The arena is one torch uint8 tensor of ``arena_bytes`` on the device; the
    library's scheduler thread admits submitted simulations into it as slots
    and memory free up and steps them concurrently."""

    def __init__(self, arena_bytes, max_active=8, steps_per_turn=10, turns_ahead=2, device=0, batch=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the ICWF library needs a GPU; none is visible")
        L = lib()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        aligned = (self.arena.data_ptr() + 255) & ~255
        cfg = ServerConfig(int(max_active), int(steps_per_turn), int(turns_ahead), dev.index or 0, 1 if batch else 0)
        h = c_void_p()
        st = L.icwf_server_create(byref(cfg), c_void_p(aligned), c_size_t(int(arena_bytes)), byref(h))
        if st != OK:
            raise ICWFError(st, "icwf_server_create failed")
        self.h = h
        self._cfgs = {}

    def submit(self, cfg, r0, R0, psi1, psi2, C0=None, b0=None, bo=None, n_steps=1):
        keep = [_f64(r0), _f64(R0), _f64(psi1), _f64(psi2), _f64(C0), _f64(b0), _f64(bo)]
        rid = c_int64()
        st = lib().icwf_server_submit(self.h, byref(cfg), *[_ptr(a) for a in keep], int(n_steps), byref(rid))
        if st != OK:
            raise ICWFError(st, "icwf_server_submit refused the request")
        self._cfgs[rid.value] = (cfg.n_traj, cfg.n_r, cfg.n_R, cfg.n_bo)
        return rid.value

    def submit_workload(self, wl, n_steps, precision=PREC_FP64, C0=None):
        cfg = config_from_workload(wl, precision)
        return self.submit(cfg, wl.r0, wl.R0, wl.psi1, wl.psi2, C0=C0, b0=None if C0 is not None else wl.b0,
                           bo=wl.bo, n_steps=n_steps)

    def wait(self, rid, timeout=-1.0):
        st = lib().icwf_server_wait(self.h, int(rid), float(timeout))
        if st == ETIMEDOUT:
            return False
        if st != OK:
            raise ICWFError(st, f"unknown request {rid}")
        return True

    def result(self, rid):
        """Final observables and timing of a finished request (then forgotten)."""
        N, nr, nR, nb = self._cfgs.pop(rid)
        out = dict(rho_r=np.zeros(nr), rho_R=np.zeros(nR), pop=np.zeros(max(nb, 1)),
                   D=np.zeros(max(nb * nb, 1)), r=np.zeros(N), R=np.zeros(N), C=np.zeros(2 * N))
        o = Obs()
        for k, v in out.items():
            setattr(o, k, _ptr(v))
        info = RequestInfo()
        st = lib().icwf_server_result(self.h, int(rid), byref(o), byref(info))
        res = dict(t=o.t, step=o.step, norm=o.norm, rho_r=out["rho_r"], rho_R=out["rho_R"], r=out["r"],
                   R=out["R"], C=out["C"].view(np.complex128), n_out_of_box=o.n_out_of_box,
                   min_abs_psi=o.min_abs_psi, status=st, slot=info.slot, t_submit=info.t_submit,
                   t_admit=info.t_admit, t_done=info.t_done, workspace_bytes=info.workspace_bytes,
                   message=info.message.decode(errors="replace"))
        if nb:
            res["pop"] = out["pop"][:nb]
            res["D"] = out["D"][:nb * nb].reshape(nb, nb)
        return res

    def stats(self):
        s = ServerStats()
        lib().icwf_server_get_stats(self.h, byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def clock(self):
        return lib().icwf_server_clock(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().icwf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
