"""Population annealing for the 2D Ising model on AMD Instinct MI355X.

A thin ctypes binding of libpa (include/pa.h).  Every step of the method runs
in the library's HIP kernels; this module only marshals arguments.  PyTorch
supplies device memory (the workspace) and the HIP stream.

The functions keep the C names (pa_create, pa_anneal_step, ...); ``Run`` and
``Batch`` bundle a handle with its torch-allocated workspace.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
from typing import IO, Iterable, List, Optional, Sequence, Union

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpa.so")

PA_OK = 0
PA_ERR_ARG, PA_ERR_NOMEM, PA_ERR_DEVICE, PA_ERR_CAPACITY = -1, -2, -3, -4
PA_ERR_DONE, PA_ERR_STATE, PA_ERR_NUMERIC, PA_ERR_EXTINCT = -5, -6, -7, -8
PA_RESAMPLE_NEAREST, PA_RESAMPLE_MULTINOMIAL, PA_RESAMPLE_NONE, PA_RESAMPLE_POISSON = 0, 1, 2, 3
PA_UPDATE_METROPOLIS, PA_UPDATE_HEATBATH = 0, 1
UPDATE = {"metropolis": PA_UPDATE_METROPOLIS, "heatbath": PA_UPDATE_HEATBATH}
PA_LAYOUT_INT8, PA_LAYOUT_MSC64 = 0, 1
PA_MLP_IN, PA_MLP_HIDDEN = 35, 64
PA_MLP_PARAMS = 64 * 35 + 64 + 64 * 64 + 64 + 64 + 1

RESAMPLE = {"nearest": PA_RESAMPLE_NEAREST, "multinomial": PA_RESAMPLE_MULTINOMIAL,
            "none": PA_RESAMPLE_NONE, "poisson": PA_RESAMPLE_POISSON}
LAYOUT = {"int8": PA_LAYOUT_INT8, "msc64": PA_LAYOUT_MSC64}
_STATUS = {0: "PA_OK", -1: "PA_ERR_ARG", -2: "PA_ERR_NOMEM", -3: "PA_ERR_DEVICE",
           -4: "PA_ERR_CAPACITY", -5: "PA_ERR_DONE", -6: "PA_ERR_STATE", -7: "PA_ERR_NUMERIC",
           -8: "PA_ERR_EXTINCT"}


class pa_config(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("R", ctypes.c_int32),
                ("betas", ctypes.POINTER(ctypes.c_double)), ("n_steps", ctypes.c_int32),
                ("theta", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("resample", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("capacity", ctypes.c_int32), ("update", ctypes.c_int32)]


class pa_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int32), ("R_i", ctypes.c_int32), ("beta", ctypes.c_double),
                ("sum_E", ctypes.c_int64), ("sum_E2", ctypes.c_int64),
                ("sum_absM", ctypes.c_int64), ("sum_M2", ctypes.c_int64),
                ("e", ctypes.c_double), ("c_v", ctypes.c_double), ("m", ctypes.c_double),
                ("chi", ctypes.c_double), ("ln_Q", ctypes.c_double),
                ("minus_beta_F", ctypes.c_double), ("n_families", ctypes.c_int64),
                ("sum_fam2", ctypes.c_int64), ("sum_cnt2", ctypes.c_int64),
                ("rho_t", ctypes.c_double), ("rho_s", ctypes.c_double),
                ("rho_t_step", ctypes.c_double), ("r_eff_E", ctypes.c_double),
                ("r_eff_absM", ctypes.c_double), ("err_e", ctypes.c_double),
                ("err_m", ctypes.c_double), ("err_c_v", ctypes.c_double),
                ("err_chi", ctypes.c_double), ("jk_var_beta_F", ctypes.c_double),
                ("jk_cov_e", ctypes.c_double), ("jk_cov_m", ctypes.c_double),
                ("jk_cov_c_v", ctypes.c_double), ("jk_cov_chi", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class pa_weighted(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int32), ("n_runs", ctypes.c_int32), ("beta", ctypes.c_double)] + \
               [(n, ctypes.c_double) for n in (
                   "e", "m", "c_v", "chi", "e_mod", "m_mod", "c_v_mod", "chi_mod", "e_plain",
                   "m_plain", "c_v_plain", "chi_plain", "omega_max", "n_eff_runs", "var_beta_F",
                   "rho_f", "cov_e", "cov_m", "cov_c_v", "cov_chi")]


class PAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


_lib = None
# (name, restype, argtypes); every entry point of include/pa.h
_vp, _i32, _i64, _u32, _u64, _dbl, _flt = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                            ctypes.c_float)
_P = ctypes.POINTER
SIGNATURES = {
    "pa_workspace_size": (_i32, [_P(pa_config), _P(ctypes.c_size_t)]),
    "pa_create": (_i32, [_P(pa_config), _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "pa_anneal_step": (_i32, [_vp]),
    "pa_anneal_step_to": (_i32, [_vp, _dbl]),
    "pa_run": (_i32, [_vp, _i32]),
    "pa_sync": (_i32, [_vp]),
    "pa_observables": (_i32, [_vp, _i32, _P(pa_obs)]),
    "pa_current": (_i32, [_vp, _P(_i32), _P(_i32)]),
    "pa_energy_histogram": (_i32, [_vp, _P(_i32), _i32, _P(_i32), _P(_i32)]),
    "pa_copy_counts": (_i32, [_vp, _P(_i32), _i64, _P(_i64)]),
    "pa_get_population": (_i32, [_vp, _i32, _i32, _P(ctypes.c_int8), _P(_i32), _P(_i32), _P(_i32)]),
    "pa_get_state": (_i32, [_vp, _vp, ctypes.c_size_t, _P(ctypes.c_size_t)]),
    "pa_set_state": (_i32, [_vp, _vp, ctypes.c_size_t]),
    "pa_set_population": (_i32, [_vp, _i32, _i32, _P(ctypes.c_int8), _P(_i32), _dbl]),
    "pa_overlap": (_i32, [_vp, _dbl, _P(_dbl)]),
    "pa_adaptive_dbeta": (_i32, [_vp, _dbl, _dbl, _P(_dbl)]),
    "pa_adaptive_dbeta_noalloc": (_i32, [_vp, _i32, _i32, _dbl, _dbl, _vp, _vp]),
    "pa_destroy": (None, [_vp]),
    "pa_last_error": (ctypes.c_char_p, [_vp]),
    "pa_batch_workspace_size": (_i32, [_P(pa_config), _i32, _P(ctypes.c_size_t)]),
    "pa_batch_create": (_i32, [_P(pa_config), _i32, _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "pa_batch_run": (_i32, [_vp, _i32]),
    "pa_batch_observables": (_i32, [_vp, _i32, _i32, _P(pa_obs)]),
    "pa_batch_get_population": (_i32, [_vp, _i32, _i32, _i32, _P(ctypes.c_int8), _P(_i32),
                                       _P(_i32), _P(_i32)]),
    "pa_batch_weighted": (_i32, [_vp, _i32, _i32, _vp]),
    "pa_overlap_correlation": (_i32, [_vp, _i32, _vp]),
    "pa_batch_sync": (_i32, [_vp]),
    "pa_batch_destroy": (None, [_vp]),
    "pa_batch_last_error": (ctypes.c_char_p, [_vp]),
    "pa_philox4x32_10": (_i32, [_u32, _u32, _vp, _i64, _vp, _vp]),
    "pa_features": (_i32, [_vp, _vp]),
    "pa_mlp_forward": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "pa_mlp_backward": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "pa_mlp_train_step": (_i32, [_vp, _vp, _vp, _vp, _i32, _flt, _i32, _vp, _vp]),
    "pa_learned_dbeta": (_i32, [_vp, _vp, _dbl, _dbl, _dbl, _vp, _P(_dbl), _P(_i32)]),
    "pa_anneal_step_adaptive": (_i32, [_vp, _dbl, _dbl]),
    "pa_anneal_step_learned": (_i32, [_vp, _vp, _dbl, _dbl, _dbl]),
    "pa_schedule_log": (_i32, [_vp, _vp, _vp, _P(_i32), _P(_dbl), _i32, _P(_i32)]),
    "pa_profile": (_i32, [_vp, _i32]),
    "pa_set_sweep_launch": (_i32, [_vp, _i32, _i32, _i32, _i32]),
    "pa_get_sweep_launch": (_i32, [_vp, _i32, _P(_i32), _P(_i32), _P(_i32)]),
    "pa_batch_set_sweep_launch": (_i32, [_vp, _i32, _i32, _i32, _i32]),
    "pa_batch_get_sweep_launch": (_i32, [_vp, _i32, _P(_i32), _P(_i32), _P(_i32)]),
    "pa_profile_read": (_i32, [_vp, _P(_i32), _P(_dbl), _P(_dbl), _P(_dbl), _P(_u64), _P(_u64),
                               _P(_dbl)]),
}


def lib():
    """The loaded libpa; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpa.so is missing at %s: run __graft_entry__.build() or "
                               "python paper_2102_06611_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, handle=None, batch: bool = False):
    if status != PA_OK:
        L = lib()
        msg = (L.pa_batch_last_error(handle) if batch else L.pa_last_error(handle)) or b""
        raise PAError(status, msg.decode(errors="replace"))


def make_config(L: int, R: int, betas: Optional[Sequence[float]], theta: int, seed: int,
                resample: str = "nearest", layout: str = "msc64", capacity: int = 0,
                n_steps: Optional[int] = None, update: str = "metropolis"):
    """A pa_config plus the double array it points to (keep both alive)."""
    arr = None
    if betas is not None:
        arr = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
        n = len(arr) - 1
    else:
        n = int(n_steps)
    cfg = pa_config(L, R, arr.ctypes.data_as(_P(ctypes.c_double)) if arr is not None else None,
                    n, theta, seed, RESAMPLE[resample], LAYOUT[layout], capacity, UPDATE[update])
    return cfg, arr


def _stream_handle(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


class Run:
    """One population-annealing run: a pa_ctx with its torch workspace."""

    def __init__(self, L: int, R: int, betas: Optional[Sequence[float]], theta: int, seed: int,
                 resample: str = "nearest", layout: str = "msc64", capacity: int = 0,
                 n_steps: Optional[int] = None, device: str = "cuda:0", stream=None,
                 update: str = "metropolis"):
        import torch
        self.L, self.N, self.R = L, L * L, R
        self.cfg, self._betas = make_config(L, R, betas, theta, seed, resample, layout,
                                            capacity, n_steps, update)
        self.max_steps = self.cfg.n_steps
        self.meta = {"L": L, "R": R, "theta": theta, "seed": seed, "resample": resample,
                     "layout": layout, "update": update}
        nbytes = ctypes.c_size_t()
        _check(lib().pa_workspace_size(ctypes.byref(self.cfg), ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().pa_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                               nbytes.value, _stream_handle(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping
    def anneal_step(self):
        _check(lib().pa_anneal_step(self.h), self.h)

    def anneal_step_to(self, beta_next: float):
        _check(lib().pa_anneal_step_to(self.h, float(beta_next)), self.h)

    def run(self, n_steps: int):
        _check(lib().pa_run(self.h, int(n_steps)), self.h)

    def sync(self):
        _check(lib().pa_sync(self.h), self.h)

    # -- results
    def observables(self, step: int) -> dict:
        o = pa_obs()
        _check(lib().pa_observables(self.h, int(step), ctypes.byref(o)), self.h)
        return o.as_dict()

    def export_jsonl(self, dest: Union[str, IO[str]], first: int = 0,
                     last: Optional[int] = None) -> int:
        """Records first .. last (default: the current step) as JSON Lines, one
        object per step with the run's configuration (write_jsonl)."""
        if last is None:
            last = self.current()[0]
        return write_jsonl((self.observables(i) for i in range(first, last + 1)), dest,
                           **self.meta)

    def current(self):
        s, r = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pa_current(self.h, ctypes.byref(s), ctypes.byref(r)), self.h)
        return s.value, r.value

    def energy_histogram(self):
        kmin, nb = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pa_energy_histogram(self.h, None, 0, ctypes.byref(kmin), ctypes.byref(nb)), self.h)
        out = np.zeros(nb.value, dtype=np.int32)
        _check(lib().pa_energy_histogram(self.h, out.ctypes.data_as(_P(_i32)), nb.value,
                                         ctypes.byref(kmin), ctypes.byref(nb)), self.h)
        return kmin.value, out

    def copy_counts(self) -> np.ndarray:
        n = ctypes.c_int64()
        _check(lib().pa_copy_counts(self.h, None, 0, ctypes.byref(n)), self.h)
        out = np.zeros(n.value, dtype=np.int32)
        _check(lib().pa_copy_counts(self.h, out.ctypes.data_as(_P(_i32)), n.value,
                                    ctypes.byref(n)), self.h)
        return out

    def population(self, first: int = 0, count: Optional[int] = None, spins: bool = True):
        """(spins [count, N] int8, fam, E, M) of the current population."""
        _, R_i = self.current()
        if count is None:
            count = R_i - first
        s = np.zeros((count, self.N), dtype=np.int8) if spins else None
        fam = np.zeros(count, dtype=np.int32)
        E = np.zeros(count, dtype=np.int32)
        M = np.zeros(count, dtype=np.int32)
        _check(lib().pa_get_population(
            self.h, first, count, s.ctypes.data_as(_P(ctypes.c_int8)) if spins else None,
            fam.ctypes.data_as(_P(_i32)), E.ctypes.data_as(_P(_i32)),
            M.ctypes.data_as(_P(_i32))), self.h)
        return s, fam, E, M

    def set_population(self, step: int, spins: np.ndarray, fam: np.ndarray, minus_beta_F: float):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        fam = np.ascontiguousarray(fam, dtype=np.int32)
        _check(lib().pa_set_population(self.h, int(step), spins.shape[0],
                                       spins.ctypes.data_as(_P(ctypes.c_int8)),
                                       fam.ctypes.data_as(_P(_i32)), float(minus_beta_F)), self.h)

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(lib().pa_get_state(self.h, None, 0, ctypes.byref(n)), self.h)
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().pa_get_state(self.h, buf, n.value, ctypes.byref(n)), self.h)
        return buf.raw

    def set_state(self, blob: bytes):
        _check(lib().pa_set_state(self.h, blob, len(blob)), self.h)

    def overlap_correlation(self, d_max: int) -> np.ndarray:
        """C_q(d), d = 0 .. d_max, of the current population (pa_overlap_correlation)."""
        import torch
        dev = torch.empty(d_max + 1, dtype=torch.float64, device=self.workspace.device)
        _check(lib().pa_overlap_correlation(self.h, int(d_max), ctypes.c_void_p(dev.data_ptr())),
               self.h)
        self.sync()
        return dev.cpu().numpy()

    def overlap(self, dbeta: float) -> float:
        a = ctypes.c_double()
        _check(lib().pa_overlap(self.h, float(dbeta), ctypes.byref(a)), self.h)
        return a.value

    def adaptive_dbeta(self, alpha_target: float, dbeta_max: float) -> float:
        d = ctypes.c_double()
        _check(lib().pa_adaptive_dbeta(self.h, float(alpha_target), float(dbeta_max),
                                       ctypes.byref(d)), self.h)
        return d.value

    def features(self, dev_feat) -> None:
        _check(lib().pa_features(self.h, ctypes.c_void_p(dev_feat.data_ptr())), self.h)

    def set_sweep_launch(self, L: int, threads: int, groups_per_block: int, variant: int = 0):
        _check(lib().pa_set_sweep_launch(self.h, L, threads, groups_per_block, variant), self.h)

    def sweep_launch(self, L: int):
        t, g, v = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pa_get_sweep_launch(self.h, L, ctypes.byref(t), ctypes.byref(g),
                                         ctypes.byref(v)), self.h)
        return t.value, g.value, v.value

    def profile(self, enable: bool = True, count_calls: bool = False):
        _check(lib().pa_profile(self.h, (1 | (2 if count_calls else 0)) if enable else 0), self.h)

    def profile_read(self) -> dict:
        n = ctypes.c_int32()
        t = [ctypes.c_double() for _ in range(4)]
        calls, words = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pa_profile_read(self.h, ctypes.byref(n), *[ctypes.byref(x) for x in t[:3]],
                                     ctypes.byref(calls), ctypes.byref(words),
                                     ctypes.byref(t[3])), self.h)
        return {"steps": n.value, "ms_resample": t[0].value, "ms_sweep": t[1].value,
                "ms_measure": t[2].value, "ms_copy": t[3].value, "philox_calls": calls.value,
                "sweep_words": words.value}

    def anneal_step_adaptive(self, alpha_target: float, beta_final: float):
        _check(lib().pa_anneal_step_adaptive(self.h, float(alpha_target), float(beta_final)), self.h)

    def anneal_step_learned(self, params, alpha_min: float, alpha_target: float,
                            beta_final: float):
        _check(lib().pa_anneal_step_learned(self.h, ctypes.c_void_p(params.data_ptr()),
                                            float(alpha_min), float(alpha_target),
                                            float(beta_final)), self.h)

    def schedule_log(self, dev_feat=None, dev_target=None):
        """(n, accepted[n], alpha[n]); features/targets go to the given device tensors."""
        n = ctypes.c_int32()
        _check(lib().pa_schedule_log(self.h, None, None, None, None, 0, ctypes.byref(n)), self.h)
        acc = np.zeros(n.value, dtype=np.int32)
        alpha = np.zeros(n.value, dtype=np.float64)
        _check(lib().pa_schedule_log(
            self.h, ctypes.c_void_p(dev_feat.data_ptr()) if dev_feat is not None else None,
            ctypes.c_void_p(dev_target.data_ptr()) if dev_target is not None else None,
            acc.ctypes.data_as(_P(_i32)), alpha.ctypes.data_as(_P(_dbl)), n.value,
            ctypes.byref(n)), self.h)
        return n.value, acc, alpha

    def learned_dbeta(self, params, alpha_min: float, alpha_target: float, dbeta_max: float,
                      dev_feat=None):
        d, acc = ctypes.c_double(), ctypes.c_int32()
        _check(lib().pa_learned_dbeta(
            self.h, ctypes.c_void_p(params.data_ptr()), float(alpha_min), float(alpha_target),
            float(dbeta_max), ctypes.c_void_p(dev_feat.data_ptr()) if dev_feat is not None else None,
            ctypes.byref(d), ctypes.byref(acc)), self.h)
        return d.value, bool(acc.value)


class Batch:
    """Independent runs of uneven (L, R) in one engine (pa_batch)."""

    def __init__(self, specs: List[dict], device: str = "cuda:0", stream=None):
        import torch
        self._keep = []
        cfgs = (pa_config * len(specs))()
        for k, s in enumerate(specs):
            cfg, arr = make_config(s["L"], s["R"], s["betas"], s["theta"], s["seed"],
                                   s.get("resample", "nearest"), s.get("layout", "msc64"),
                                   s.get("capacity", 0), None, s.get("update", "metropolis"))
            cfgs[k] = cfg
            self._keep.append(arr)
        self.n = len(specs)
        self._L = [s["L"] for s in specs]
        self.meta = [{"run": k, "L": s["L"], "R": s["R"], "theta": s["theta"], "seed": s["seed"],
                      "resample": s.get("resample", "nearest"), "layout": s.get("layout", "msc64"),
                      "update": s.get("update", "metropolis")} for k, s in enumerate(specs)]
        self.steps = 0  # steps queued so far (every run advances together)
        nbytes = ctypes.c_size_t()
        _check(lib().pa_batch_workspace_size(cfgs, self.n, ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().pa_batch_create(cfgs, self.n, ctypes.c_void_p(self.workspace.data_ptr()),
                                     nbytes.value, _stream_handle(stream), ctypes.byref(h)))
        self.h = h
        self.stream = stream

    def run(self, n_steps: int):
        _check(lib().pa_batch_run(self.h, int(n_steps)), self.h, batch=True)
        self.steps += int(n_steps)

    def set_sweep_launch(self, L: int, threads: int, groups_per_block: int, variant: int = 0):
        _check(lib().pa_batch_set_sweep_launch(self.h, L, threads, groups_per_block, variant),
               self.h, batch=True)

    def sweep_launch(self, L: int):
        t, g, v = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pa_batch_get_sweep_launch(self.h, L, ctypes.byref(t), ctypes.byref(g),
                                               ctypes.byref(v)), self.h, batch=True)
        return t.value, g.value, v.value

    def sync(self):
        _check(lib().pa_batch_sync(self.h), self.h, batch=True)

    def observables(self, run: int, step: int) -> dict:
        o = pa_obs()
        _check(lib().pa_batch_observables(self.h, int(run), int(step), ctypes.byref(o)), self.h,
               batch=True)
        return o.as_dict()

    def population(self, run: int, first: int, count: int, spins: bool = True):
        """(spins [count, N] int8, fam, E, M) of replicas [first, first + count) of run `run`."""
        N = self._L[run] ** 2
        s = np.zeros((count, N), dtype=np.int8) if spins else None
        fam = np.zeros(count, dtype=np.int32)
        E = np.zeros(count, dtype=np.int32)
        M = np.zeros(count, dtype=np.int32)
        _check(lib().pa_batch_get_population(
            self.h, int(run), int(first), int(count),
            s.ctypes.data_as(_P(ctypes.c_int8)) if spins else None, fam.ctypes.data_as(_P(_i32)),
            E.ctypes.data_as(_P(_i32)), M.ctypes.data_as(_P(_i32))), self.h, batch=True)
        return s, fam, E, M

    def export_jsonl(self, dest: Union[str, IO[str]], runs: Optional[Sequence[int]] = None,
                     first: int = 0, last: Optional[int] = None) -> int:
        """Records first .. last (default: the last queued step) of the given runs
        (default: all) as JSON Lines, run by run, each object carrying its run's
        index and configuration (write_jsonl)."""
        if last is None:
            last = self.steps
        runs = range(self.n) if runs is None else runs
        recs = ({**self.meta[r], **self.observables(r, i)} for r in runs
                for i in range(first, last + 1))
        return write_jsonl(recs, dest)

    def weighted(self, first: int, count: int = 1) -> List[dict]:
        """The runs combined at steps first .. first + count - 1 (pa_batch_weighted)."""
        import torch
        dev = torch.empty(count * ctypes.sizeof(pa_weighted), dtype=torch.uint8,
                          device=self.workspace.device)
        _check(lib().pa_batch_weighted(self.h, int(first), int(count),
                                       ctypes.c_void_p(dev.data_ptr())), self.h, batch=True)
        torch.cuda.synchronize(dev.device)  # a run's device status does not stop the read
        host = dev.cpu().numpy().tobytes()
        arr = (pa_weighted * count).from_buffer_copy(host)
        return [{k: getattr(w, k) for k, _ in pa_weighted._fields_} for w in arr]

    def close(self):
        if getattr(self, "h", None):
            lib().pa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_NONFINITE = {"NaN": math.nan, "Infinity": math.inf, "-Infinity": -math.inf}


def _json_value(v):
    if isinstance(v, float) and not math.isfinite(v):
        return "NaN" if math.isnan(v) else ("Infinity" if v > 0 else "-Infinity")
    return v


def write_jsonl(records: Iterable[dict], dest: Union[str, IO[str]], **extra) -> int:
    """Per-step records (dicts from observables() or weighted()) as JSON Lines.

    One strict-JSON object per line: the `extra` keys first (e.g. the run's
    configuration), then the record's fields in their C order.  JSON has no
    non-finite numbers, so NaN (a blocked error with fewer than two blocks) and
    +-inf (R_eff of a population whose blocked variance is zero) are written as
    the strings "NaN", "Infinity" and "-Infinity"; read_jsonl turns them back.
    dest is a path (overwritten) or an open text file.  Returns the line count.
    """
    def emit(fh):
        n = 0
        for rec in records:
            obj = {k: _json_value(v) for k, v in {**extra, **rec}.items()}
            fh.write(json.dumps(obj, allow_nan=False) + "\n")
            n += 1
        return n

    if isinstance(dest, (str, os.PathLike)):
        with open(dest, "w") as fh:
            return emit(fh)
    return emit(dest)


def read_jsonl(src: Union[str, IO[str]]) -> List[dict]:
    """The records of a write_jsonl file, with non-finite values restored."""
    def load(fh):
        out = []
        for line in fh:
            if line.strip():
                obj = json.loads(line)
                out.append({k: _NONFINITE.get(v, v) if isinstance(v, str) else v
                            for k, v in obj.items()})
        return out

    if isinstance(src, (str, os.PathLike)):
        with open(src) as fh:
            return load(fh)
    return load(src)


def philox4x32_10(key: int, ctr_dev, out_dev, stream=None):
    """Device Philox4x32-10 over an [n, 4] uint32 (int32-typed) counter tensor."""
    n = ctr_dev.shape[0]
    _check(lib().pa_philox4x32_10(key & 0xFFFFFFFF, key >> 32, ctypes.c_void_p(ctr_dev.data_ptr()),
                                  n, ctypes.c_void_p(out_dev.data_ptr()), _stream_handle(stream)))


def mlp_forward(params, x, y, stream=None):
    _check(lib().pa_mlp_forward(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                x.shape[0], ctypes.c_void_p(y.data_ptr()), _stream_handle(stream)))


def mlp_backward(params, x, t, grad, loss, stream=None):
    _check(lib().pa_mlp_backward(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(t.data_ptr()), x.shape[0],
                                 ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                 _stream_handle(stream)))


def mlp_train_step(params, adam, x, t, lr: float, step: int, loss, stream=None):
    _check(lib().pa_mlp_train_step(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(adam.data_ptr()),
                                   ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                   x.shape[0], float(lr), int(step), ctypes.c_void_p(loss.data_ptr()),
                                   _stream_handle(stream)))


def adaptive_dbeta_noalloc(E_dev, L: int, alpha_target: float, dbeta_max: float, out_dev,
                           stream=None):
    """pa_adaptive_dbeta_noalloc: out_dev[0] = dbeta, out_dev[1] = its overlap, for
    the energies in the int32 device tensor E_dev (asynchronous)."""
    _check(lib().pa_adaptive_dbeta_noalloc(ctypes.c_void_p(E_dev.data_ptr()), E_dev.numel(),
                                           int(L), float(alpha_target), float(dbeta_max),
                                           ctypes.c_void_p(out_dev.data_ptr()),
                                           _stream_handle(stream)))
