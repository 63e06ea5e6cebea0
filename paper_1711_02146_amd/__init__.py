"""Population annealing (Amey & Machta, arXiv:1711.02146) on AMD MI355X.

Thin Python binding of ``libpa.so`` (C ABI declared in ``include/pa.h``): the
functions ``pa_*`` below carry the C names and only marshal arguments; every
step of the annealing path runs in the library's HIP kernels and its C++ host
code.  PyTorch supplies the device workspace and the HIP stream.

There is no CPU fallback: if the library is not built, importing a function
raises ``ImportError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpa.so")

PA_OK = 0
PA_EINVAL = -1
PA_ENOMEM = -2
PA_ECAPACITY = -3
PA_EDEVICE = -4
PA_ESTATE = -5
PA_ESCHEDULE = -6
PA_ECHECK = -7

PA_FLAG_CHECK_ENERGY = 1
PA_FLAG_FAULT_HOOK = 2
PA_FLAG_TIME_SWEEPS = 4
PA_INJECT_FAIL_AFTER = 1
PA_INJECT_ENERGY = 2

PA_MODEL_PM = 0
PA_MODEL_GAUSS16 = 1
PA_MODEL_GAUSS = 2
MODELS = {"pm": PA_MODEL_PM, "gauss16": PA_MODEL_GAUSS16, "gauss": PA_MODEL_GAUSS}

PA_LAYOUT_AUTO = 0
PA_LAYOUT_INT8 = 1
PA_LAYOUT_BITPACK64 = 2
LAYOUTS = {"auto": PA_LAYOUT_AUTO, "int8": PA_LAYOUT_INT8, "bitpack64": PA_LAYOUT_BITPACK64}


class pa_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("R", ctypes.c_uint32), ("capacity", ctypes.c_uint32),
                ("layout", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("model", ctypes.c_uint32)]


class pa_obs(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("dbeta", ctypes.c_double), ("lnQ", ctypes.c_double),
                ("beta_F", ctypes.c_double), ("mean_E", ctypes.c_double), ("rho_t", ctypes.c_double),
                ("eps_expected", ctypes.c_double), ("R_tilde", ctypes.c_uint32),
                ("n_culled", ctypes.c_uint32), ("E_min", ctypes.c_int32), ("step", ctypes.c_uint32),
                ("sum_eta2", ctypes.c_uint64), ("sweeps_done", ctypes.c_uint64),
                ("n_at_E_min", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("sum_lnQ", ctypes.c_double), ("sweep_ms", ctypes.c_double),
                ("E_lowest", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class pa_ceilings(ctypes.Structure):
    _fields_ = [("valu_lane_ops_per_s", ctypes.c_double), ("valu3_lane_ops_per_s", ctypes.c_double),
                ("philox_draws_per_s", ctypes.c_double)]


class PAError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {pa_strerror(status)} ({status})")


_lib = None
_vp = ctypes.c_void_p
_P = ctypes.POINTER


def lib():
    """Load libpa.so (built in-tree by ``python -m paper_1711_02146_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1711_02146_amd.build` "
                          "(the HIP library is the only implementation)")
    # torch brings its own HIP runtime; it must be loaded before libpa so that
    # libpa binds to that runtime (the one that owns torch's device memory and
    # streams) rather than to a second copy
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "pa_workspace_bytes": (ctypes.c_size_t, [_P(pa_params)]),
        "pa_init_instance": (ctypes.c_int, [_P(pa_params), _vp, _vp, ctypes.c_size_t, _vp,
                                            _P(_vp)]),
        "pa_sweep": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_uint32]),
        "pa_resample": (ctypes.c_int, [_vp, ctypes.c_double, _P(pa_obs)]),
        "pa_choose_beta": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double,
                                          _P(ctypes.c_double)]),
        "pa_observables": (ctypes.c_int, [_vp, _P(pa_obs)]),
        "pa_overlap_hist": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _vp]),
        "pa_link_overlap_hist": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _vp]),
        "pa_export_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _P(ctypes.c_uint32)]),
        "pa_export_counts": (ctypes.c_int, [_vp, _vp, _vp, _P(ctypes.c_uint32)]),
        "pa_import_state": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_uint32, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_double, ctypes.c_double]),
        "pa_free": (ctypes.c_int, [_vp]),
        "pa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "pa_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32,
                                                       ctypes.c_uint32, ctypes.c_uint32]),
        "pa_batch_create": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, ctypes.c_uint32, _vp,
                                           ctypes.c_uint32, ctypes.c_uint32, _vp, ctypes.c_size_t,
                                           _P(_vp)]),
        "pa_batch_run": (ctypes.c_int, [_vp, ctypes.c_uint32]),
        "pa_batch_results": (ctypes.c_int, [_vp, _vp, _vp, _vp, _P(ctypes.c_uint32)]),
        "pa_batch_free": (ctypes.c_int, [_vp]),
        "pa_stepper_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32]),
        "pa_stepper_create": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _vp,
                                             ctypes.c_size_t, _vp, _P(_vp)]),
        "pa_stepper_step": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _vp, _vp, _vp, _vp]),
        "pa_stepper_free": (ctypes.c_int, [_vp]),
        "pa_autotune_sweep": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                             _vp, _vp]),
        "pa_autotune_reset": (ctypes.c_int, []),
        "pa_autotune_set": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_uint32]),
        "pa_probe_scratch_bytes": (ctypes.c_size_t, []),
        "pa_make_couplings_pm": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, _vp]),
        "pa_probe_ceilings": (ctypes.c_int, [_vp, ctypes.c_size_t, _vp, _P(pa_ceilings)]),
        "pa_debug_inject": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32]),
        "pa_anneal_step": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                          _P(ctypes.c_double), _P(pa_obs)]),
        "pa_anneal_run": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                         ctypes.c_uint32, _vp, _P(ctypes.c_uint32)]),
        "pa_link_overlap_hist_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _vp]),
        "pa_autotune_layout_workspace_bytes": (ctypes.c_size_t, [_P(pa_params)]),
        "pa_init_instance_real": (ctypes.c_int, [_P(pa_params), _vp, _vp, ctypes.c_size_t, _vp,
                                                 _P(_vp)]),
        "pa_export_energies": (ctypes.c_int, [_vp, _vp]),
        "pa_autotune_layout": (ctypes.c_int, [_P(pa_params), _vp, _vp, ctypes.c_size_t, _vp,
                                              ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                              _P(ctypes.c_uint32), _vp]),
        "pa_layout_choice": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                            _P(ctypes.c_uint32)]),
        "pa_autotune_set_layout": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_uint64, ctypes.c_uint32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ["pa_workspace_bytes", "pa_init_instance", "pa_sweep", "pa_resample", "pa_choose_beta",
            "pa_observables", "pa_overlap_hist", "pa_export_state", "pa_export_counts",
            "pa_import_state", "pa_free", "pa_strerror", "pa_batch_workspace_bytes",
            "pa_batch_create", "pa_batch_run", "pa_batch_results", "pa_batch_free",
            "pa_stepper_workspace_bytes", "pa_stepper_create", "pa_stepper_step",
            "pa_stepper_free", "pa_autotune_sweep", "pa_autotune_reset", "pa_probe_scratch_bytes",
            "pa_probe_ceilings", "pa_make_couplings_pm", "pa_autotune_set",
            "pa_link_overlap_hist", "pa_debug_inject", "pa_anneal_step", "pa_anneal_run",
            "pa_link_overlap_hist_noalloc", "pa_autotune_layout_workspace_bytes",
            "pa_autotune_layout", "pa_layout_choice", "pa_autotune_set_layout",
            "pa_init_instance_real", "pa_export_energies"]


# --- the C entry points, one Python function each ---------------------------
def pa_workspace_bytes(params: pa_params) -> int:
    return int(lib().pa_workspace_bytes(ctypes.byref(params)))


def pa_strerror(status: int) -> str:
    return lib().pa_strerror(int(status)).decode()


def _check(rc: int, what: str):
    if rc != PA_OK:
        raise PAError(rc, what)


def pa_init_instance(params: pa_params, J: np.ndarray, workspace_ptr: int, ws_bytes: int,
                     stream_handle: int) -> int:
    J = np.ascontiguousarray(J, np.int8)
    out = _vp()
    _check(lib().pa_init_instance(ctypes.byref(params), J.ctypes.data, workspace_ptr, ws_bytes,
                                  stream_handle, ctypes.byref(out)), "pa_init_instance")
    return out.value


def pa_sweep(handle: int, beta: float, n_sweeps: int):
    _check(lib().pa_sweep(handle, float(beta), int(n_sweeps)), "pa_sweep")


def pa_resample(handle: int, beta_next: float) -> dict:
    o = pa_obs()
    _check(lib().pa_resample(handle, float(beta_next), ctypes.byref(o)), "pa_resample")
    return o.as_dict()


def pa_choose_beta(handle: int, eps_target: float, beta_max: float) -> float:
    b = ctypes.c_double(0.0)
    _check(lib().pa_choose_beta(handle, float(eps_target), float(beta_max), ctypes.byref(b)),
           "pa_choose_beta")
    return b.value


def pa_anneal_step(handle: int, eps_target: float, beta_max: float, n_sweeps: int,
                   beta_next: float = 0.0):
    """-> (beta reached, observables dict).  eps_target < 0: step to beta_next."""
    b = ctypes.c_double(float(beta_next))
    o = pa_obs()
    _check(lib().pa_anneal_step(handle, float(eps_target), float(beta_max), int(n_sweeps),
                                ctypes.byref(b), ctypes.byref(o)), "pa_anneal_step")
    return b.value, o.as_dict()


def pa_anneal_run(handle: int, eps_target: float, beta_max: float, n_sweeps: int,
                  max_steps: int):
    """-> list of observables dicts, one per step taken (at most max_steps;
    fewer when beta_max is reached).  A failing step raises PAError after the
    steps before it have been taken."""
    obs = (pa_obs * max(int(max_steps), 1))()
    done = ctypes.c_uint32(0)
    rc = lib().pa_anneal_run(handle, float(eps_target), float(beta_max), int(n_sweeps),
                             int(max_steps), ctypes.cast(obs, _vp), ctypes.byref(done))
    out = [obs[k].as_dict() for k in range(done.value)]
    if rc != PA_OK:
        err = PAError(rc, "pa_anneal_run")
        err.steps = out
        raise err
    return out


def pa_observables(handle: int) -> dict:
    o = pa_obs()
    _check(lib().pa_observables(handle, ctypes.byref(o)), "pa_observables")
    return o.as_dict()


def pa_overlap_hist(a: int, b: int, nbins: int = 65) -> np.ndarray:
    h = np.zeros(nbins, np.uint64)
    _check(lib().pa_overlap_hist(a, b, nbins, h.ctypes.data), "pa_overlap_hist")
    return h


PA_NOALLOC_MAX_BINS = 5185


def pa_link_overlap_hist_noalloc(a: int, b: int, nbins: int) -> np.ndarray:
    h = np.zeros(nbins, np.uint64)
    _check(lib().pa_link_overlap_hist_noalloc(a, b, nbins, h.ctypes.data),
           "pa_link_overlap_hist_noalloc")
    return h


def pa_link_overlap_hist(a: int, b: int, nbins: int) -> np.ndarray:
    h = np.zeros(nbins, np.uint64)
    _check(lib().pa_link_overlap_hist(a, b, nbins, h.ctypes.data), "pa_link_overlap_hist")
    return h


def pa_export_state(handle: int, N: int, spins=True, U=True, family=True):
    n = ctypes.c_uint32(0)
    _check(lib().pa_export_state(handle, None, None, None, ctypes.byref(n)), "pa_export_state")
    R = n.value
    s = np.zeros((R, N), np.int8) if spins else None
    u = np.zeros(R, np.uint32) if U else None
    f = np.zeros(R, np.uint32) if family else None
    _check(lib().pa_export_state(handle, s.ctypes.data if spins else None,
                                 u.ctypes.data if U else None, f.ctypes.data if family else None,
                                 ctypes.byref(n)), "pa_export_state")
    return s, u, f


def pa_init_instance_real(params: pa_params, J: np.ndarray, workspace_ptr: int, ws_bytes: int,
                          stream_handle: int) -> int:
    J = np.ascontiguousarray(J, np.float64)
    out = _vp()
    _check(lib().pa_init_instance_real(ctypes.byref(params), J.ctypes.data, workspace_ptr,
                                       ws_bytes, stream_handle, ctypes.byref(out)),
           "pa_init_instance_real")
    return out.value


def pa_export_energies(handle: int) -> np.ndarray:
    """Energies of the current population in units of J (FP64, exact)."""
    n = ctypes.c_uint32(0)
    _check(lib().pa_export_state(handle, None, None, None, ctypes.byref(n)), "pa_export_state")
    E = np.zeros(n.value, np.float64)
    _check(lib().pa_export_energies(handle, E.ctypes.data), "pa_export_energies")
    return E


def pa_export_counts(handle: int):
    n = ctypes.c_uint32(0)
    _check(lib().pa_export_counts(handle, None, None, ctypes.byref(n)), "pa_export_counts")
    c = np.zeros(n.value, np.uint32)
    o = np.zeros(n.value, np.uint32)
    _check(lib().pa_export_counts(handle, c.ctypes.data, o.ctypes.data, ctypes.byref(n)),
           "pa_export_counts")
    return c, o


def pa_import_state(handle: int, spins: np.ndarray, family: np.ndarray, sweeps_done: int,
                    step: int, beta: float, sum_lnQ: float):
    spins = np.ascontiguousarray(spins, np.int8)
    family = np.ascontiguousarray(family, np.uint32)
    _check(lib().pa_import_state(handle, spins.ctypes.data, family.ctypes.data, family.size,
                                 int(sweeps_done), int(step), float(beta), float(sum_lnQ)),
           "pa_import_state")


def pa_make_couplings_pm(L: int, coupling_seed: int) -> np.ndarray:
    """+-J couplings of one disorder sample from the library's Philox stream."""
    out = np.zeros(3 * int(L) ** 3, np.int8)
    _check(lib().pa_make_couplings_pm(int(coupling_seed), int(L), out.ctypes.data),
           "pa_make_couplings_pm")
    return out


def pa_free(handle: int):
    _check(lib().pa_free(handle), "pa_free")


def pa_debug_inject(handle: int, what: int, arg: int):
    _check(lib().pa_debug_inject(handle, int(what), int(arg)), "pa_debug_inject")


def linear_schedule(beta_max: float, n_temps: int):
    """beta_k = (beta_max k) / (N_T - 1), k = 0 .. N_T - 1, each formed that way
    in FP64 (not accumulated): the ascending linear schedule of N_T temperatures
    from 0 to beta_max (Sec. II loop)."""
    return [(beta_max * k) / (n_temps - 1) for k in range(n_temps)]


def pa_batch_workspace_bytes(n_pops: int, n_pairs: int, n_steps: int, max_L: int) -> int:
    return int(lib().pa_batch_workspace_bytes(n_pops, n_pairs, n_steps, max_L))


def pa_batch_create(handles, pairs, betas, n_sweeps: int, workspace_ptr: int,
                    ws_bytes: int) -> int:
    hs = (_vp * len(handles))(*handles)
    pr = np.ascontiguousarray(np.asarray(pairs, np.uint32).reshape(-1))
    bt = np.ascontiguousarray(betas, np.float64)
    out = _vp()
    _check(lib().pa_batch_create(ctypes.cast(hs, _vp), len(handles),
                                 pr.ctypes.data if pr.size else None, pr.size // 2,
                                 bt.ctypes.data, bt.size - 1, int(n_sweeps), workspace_ptr,
                                 ws_bytes, ctypes.byref(out)), "pa_batch_create")
    return out.value


def pa_batch_run(batch: int, n_steps: int):
    _check(lib().pa_batch_run(batch, int(n_steps)), "pa_batch_run")


def pa_batch_results(batch: int, n_pops: int, n_pairs: int, max_steps: int):
    """-> (records [steps][pops] of pa_obs dicts as a structured array, qhist, status)."""
    obs = (pa_obs * (max_steps * n_pops))()
    q = np.zeros((max_steps, max(n_pairs, 1), 65), np.uint64)
    st = np.zeros(n_pops, np.int32)
    done = ctypes.c_uint32(0)
    _check(lib().pa_batch_results(batch, ctypes.cast(obs, _vp), q.ctypes.data if n_pairs else None,
                                  st.ctypes.data, ctypes.byref(done)), "pa_batch_results")
    n = done.value
    recs = [[obs[s * n_pops + p].as_dict() for p in range(n_pops)] for s in range(n)]
    return recs, q[:n, :n_pairs], st


def pa_batch_free(batch: int):
    _check(lib().pa_batch_free(batch), "pa_batch_free")


def pa_stepper_workspace_bytes(max_pops: int, max_L: int) -> int:
    return int(lib().pa_stepper_workspace_bytes(int(max_pops), int(max_L)))


def pa_stepper_create(max_pops: int, max_L: int, workspace_ptr: int, ws_bytes: int,
                      stream_handle: int) -> int:
    out = _vp()
    _check(lib().pa_stepper_create(int(max_pops), int(max_L), workspace_ptr, ws_bytes,
                                   stream_handle, ctypes.byref(out)), "pa_stepper_create")
    return out.value


def pa_stepper_step(stepper: int, handles, beta_next, n_sweeps):
    """-> (list of pa_obs dicts, status array); one step for every handle."""
    n = len(handles)
    hs = (_vp * max(n, 1))(*handles)
    bt = np.ascontiguousarray(beta_next, np.float64)
    ns = np.ascontiguousarray(n_sweeps, np.uint32)
    if bt.size != n or ns.size != n:
        raise PAError(PA_EINVAL, "pa_stepper_step")
    obs = (pa_obs * max(n, 1))()
    st = np.zeros(max(n, 1), np.int32)
    _check(lib().pa_stepper_step(stepper, ctypes.cast(hs, _vp), n, bt.ctypes.data, ns.ctypes.data,
                                 ctypes.cast(obs, _vp), st.ctypes.data), "pa_stepper_step")
    return [obs[p].as_dict() for p in range(n)], st[:n]


def pa_stepper_free(stepper: int):
    _check(lib().pa_stepper_free(stepper), "pa_stepper_free")


def pa_autotune_sweep(handle: int, beta: float = 1.0, n_sweeps: int = 10, repeats: int = 3) -> dict:
    split = ctypes.c_uint32(0)
    ms = (ctypes.c_float * 2)()
    _check(lib().pa_autotune_sweep(handle, float(beta), int(n_sweeps), int(repeats),
                                   ctypes.byref(split), ctypes.cast(ms, _vp)), "pa_autotune_sweep")
    return {"split": split.value, "ms_split4": ms[0], "ms_split8": ms[1]}


def pa_autotune_reset():
    _check(lib().pa_autotune_reset(), "pa_autotune_reset")


def pa_autotune_set(L: int, R_tilde: int, split: int, layout: str = "bitpack64",
                    model: str = "pm"):
    """Pin the sweep form (4 or 8 waves per tile) for populations of this shape."""
    tiles = (int(R_tilde) + 63) // 64
    _check(lib().pa_autotune_set(MODELS[model], LAYOUTS[layout], int(L), tiles, int(split)),
           "pa_autotune_set")


LAYOUT_NAMES = {PA_LAYOUT_INT8: "int8", PA_LAYOUT_BITPACK64: "bitpack64"}


def pa_layout_choice(L: int, R: int, model: str = "pm") -> str:
    """The concrete layout "auto" resolves to now for populations of this shape."""
    out = ctypes.c_uint32(0)
    _check(lib().pa_layout_choice(MODELS[model], int(L), int(R), ctypes.byref(out)),
           "pa_layout_choice")
    return LAYOUT_NAMES[out.value]


def pa_autotune_set_layout(L: int, R: int, layout: str, model: str = "pm"):
    """Pin the layout "auto" resolves to for populations of this shape."""
    tiles = (int(R) + 63) // 64
    _check(lib().pa_autotune_set_layout(MODELS[model], int(L), tiles, LAYOUTS[layout]),
           "pa_autotune_set_layout")


def pa_autotune_layout(L: int, R: int, J: np.ndarray, seed: int = 0, beta: float = 1.0,
                       n_sweeps: int = 10, repeats: int = 3, model: str = "pm", capacity: int = 0,
                       device=None, stream=None) -> dict:
    """Time both spin layouts (each with its faster sweep form) on this shape
    and record the faster for "auto" -> {"layout", "ms_int8", "ms_bitpack64"}.
    The workspace is a temporary torch allocation on the device."""
    import torch

    params = pa_params(L=L, R=R, capacity=capacity, layout=PA_LAYOUT_AUTO, seed=seed, flags=0,
                       model=MODELS[model])
    nbytes = lib().pa_autotune_layout_workspace_bytes(ctypes.byref(params))
    if nbytes == 0:
        raise PAError(PA_EINVAL, "pa_autotune_layout_workspace_bytes")
    dev = torch.device(device) if device is not None else torch.device("cuda")
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    Jc = np.ascontiguousarray(J, dtype=np.int8)
    out = ctypes.c_uint32(0)
    ms = (ctypes.c_float * 2)()
    _check(lib().pa_autotune_layout(ctypes.byref(params), Jc.ctypes.data, ws.data_ptr(), nbytes,
                                    stream.cuda_stream, float(beta), int(n_sweeps), int(repeats),
                                    ctypes.byref(out), ctypes.cast(ms, _vp)), "pa_autotune_layout")
    del ws
    return {"layout": LAYOUT_NAMES[out.value], "ms_int8": ms[0], "ms_bitpack64": ms[1]}


def pa_probe_ceilings(stream=None, device=None) -> dict:
    """This device's sustained VALU lane-op rate and Philox draw rate (scratch
    from torch on the device; stream defaults to the current one)."""
    import torch

    dev = torch.device(device) if device is not None else torch.device("cuda")
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    nbytes = lib().pa_probe_scratch_bytes()
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = pa_ceilings()
    _check(lib().pa_probe_ceilings(scratch.data_ptr(), nbytes, stream.cuda_stream,
                                   ctypes.byref(out)), "pa_probe_ceilings")
    return {"valu_lane_ops_per_s": out.valu_lane_ops_per_s,
            "valu3_lane_ops_per_s": out.valu3_lane_ops_per_s,
            "philox_draws_per_s": out.philox_draws_per_s}


# --- convenience object owning the workspace ---------------------------------
class Population:
    """One PA population on a GPU: workspace tensor + library handle."""

    def __init__(self, L: int, R: int, J: np.ndarray, seed: int, capacity: int = 0,
                 layout: str = "auto", device=None, stream=None, model: str = "pm",
                 flags: int = 0):
        """model "pm": J holds +-1; "gauss16": J holds k = 16 J in [-127, 127];
        "gauss": J holds real couplings (FP64, |J| < 8, rounded to the grid 2^-32).
        layout: "int8", "bitpack64" or "auto" (the autotuner's choice for this
        shape, resolved once here).  flags: PA_FLAG_* bits (debugging aids)."""
        import torch

        self.L, self.N, self.R = int(L), int(L) ** 3, int(R)
        self.model = model
        if layout == "auto":
            layout = pa_layout_choice(L, R, model)
        self.layout = layout
        self.params = pa_params(L=L, R=R, capacity=capacity, layout=LAYOUTS[layout], seed=seed,
                                flags=int(flags), model=MODELS[model])
        nbytes = pa_workspace_bytes(self.params)
        if nbytes == 0:
            raise PAError(PA_EINVAL, "pa_workspace_bytes")
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        init = pa_init_instance_real if model == "gauss" else pa_init_instance
        self.handle = init(self.params, J, self.workspace.data_ptr(), nbytes,
                           self.stream.cuda_stream)

    def sweep(self, beta: float, n_sweeps: int):
        pa_sweep(self.handle, beta, n_sweeps)

    def resample(self, beta_next: float) -> dict:
        return pa_resample(self.handle, beta_next)

    def choose_beta(self, eps_target: float, beta_max: float) -> float:
        return pa_choose_beta(self.handle, eps_target, beta_max)

    def observables(self) -> dict:
        return pa_observables(self.handle)

    def anneal_step(self, eps_target: float, beta_max: float, n_sweeps: int):
        """One constant-culling step (choose beta, resample, sweep, measure) with
        one synchronisation -> (beta, observables)."""
        return pa_anneal_step(self.handle, eps_target, beta_max, n_sweeps)

    def anneal_run(self, eps_target: float, beta_max: float, n_sweeps: int, max_steps: int):
        """Up to max_steps constant-culling steps (stops at beta_max) in one call
        -> list of observables dicts."""
        return pa_anneal_run(self.handle, eps_target, beta_max, n_sweeps, max_steps)

    def step_to(self, beta_next: float, n_sweeps: int) -> dict:
        """One step to the given beta (resample, sweep, measure) -> observables."""
        return pa_anneal_step(self.handle, -1.0, 0.0, n_sweeps, beta_next)[1]

    def export_state(self, spins=True, U=True, family=True):
        """(spins, energy words, family labels); for model "gauss" the energies
        in units of J (FP64) stand in for the energy words."""
        if self.model == "gauss":
            s, _, f = pa_export_state(self.handle, self.N, spins, False, family)
            return s, (pa_export_energies(self.handle) if U else None), f
        return pa_export_state(self.handle, self.N, spins, U, family)

    def export_energies(self) -> np.ndarray:
        return pa_export_energies(self.handle)

    def export_counts(self):
        return pa_export_counts(self.handle)

    def import_state(self, spins, family, sweeps_done, step, beta, sum_lnQ):
        pa_import_state(self.handle, spins, family, sweeps_done, step, beta, sum_lnQ)

    def autotune(self, beta: float = 1.0, n_sweeps: int = 10, repeats: int = 3) -> dict:
        """Time both sweep forms on this population's shape at inverse
        temperature beta; later launches of that shape (any instance, batch or
        stepper) use the faster."""
        return pa_autotune_sweep(self.handle, beta, n_sweeps, repeats)

    def close(self):
        if getattr(self, "handle", None):
            pa_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def overlap_hist(a: Population, b: Population) -> np.ndarray:
    return pa_overlap_hist(a.handle, b.handle, 65)


def link_overlap_hist(a: Population, b: Population) -> np.ndarray:
    """Counts of D = 0..3N over the slot pairs (i, i) of a and b: D bonds whose
    two ends differ in s^a s^b, i.e. link overlap q_l = 1 - 2 D / (3N)."""
    return pa_link_overlap_hist(a.handle, b.handle, 3 * a.N + 1)


class Batch:
    """Populations advanced together through one schedule (one graph replay per step).

    The populations must live on a created (non-default) stream, share it, and
    sit at betas[0].  ``pairs`` lists (a, b) index pairs whose overlap
    histogram is recorded after every step.
    """

    def __init__(self, pops, betas, n_sweeps: int, pairs=()):
        import torch

        self.pops = list(pops)
        self.n_pops = len(self.pops)
        self.pairs = [tuple(p) for p in pairs]
        self.n_steps = len(betas) - 1
        max_L = max(p.L for p in self.pops)
        nbytes = pa_batch_workspace_bytes(self.n_pops, len(self.pairs), self.n_steps, max_L)
        if nbytes == 0:
            raise PAError(PA_EINVAL, "pa_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.pops[0].device)
        self.handle = pa_batch_create([p.handle for p in self.pops], self.pairs, betas, n_sweeps,
                                      self.workspace.data_ptr(), nbytes)

    def run(self, n_steps: int | None = None):
        pa_batch_run(self.handle, self.n_steps if n_steps is None else n_steps)

    def results(self):
        return pa_batch_results(self.handle, self.n_pops, len(self.pairs), self.n_steps)

    def close(self):
        if getattr(self, "handle", None):
            pa_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stepper:
    """Continuous batching: one temperature step for any set of Populations
    (all created on ``stream``) per call, in one set of launches."""

    def __init__(self, max_pops: int, max_L: int, stream, device=None):
        import torch

        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.stream = stream
        self.max_pops, self.max_L = int(max_pops), int(max_L)
        nbytes = pa_stepper_workspace_bytes(self.max_pops, self.max_L)
        if nbytes == 0:
            raise PAError(PA_EINVAL, "pa_stepper_workspace_bytes")
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = pa_stepper_create(self.max_pops, self.max_L, self.workspace.data_ptr(),
                                        nbytes, stream.cuda_stream)

    def step(self, pops, beta_next, n_sweeps):
        return pa_stepper_step(self.handle, [p.handle for p in pops], beta_next, n_sweeps)

    def close(self):
        if getattr(self, "handle", None):
            pa_stepper_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
