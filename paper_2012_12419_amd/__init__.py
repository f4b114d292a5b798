"""Python binding of libmdpvi (ctypes): value iteration for the occupancy MDP
of vehicular bag-of-task placement on MI355X.

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI of ``include/mdpvi.h``.  torch tensors supply device memory and the
current HIP stream.  There is no CPU fallback: loading fails loudly when the
library is missing, and every call requires tensors on a GPU.

    import paper_2012_12419_amd as mdpvi
    mdp = mdpvi.MDP(K=3, C=8, size=[1, 2], lam=[.6, .3], mu=.1, nu=.02,
                    reward=[1, 2.5], gamma=.95)
    V = torch.zeros(mdp.num_states, device="cuda")
    stats = mdp.vi_solve(V, tol=1e-6)
    pi, gap = mdp.policy_extract(V)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmdpvi.so")

OK = 0
EINVAL = -1
ERANGE = -2
ENOCONV = -3
ENAN = -4
EDEVICE = -5
ENOMEM = -6
FORM_TILE = 16   # mdp_set_sweep_form: the tile form
FORM_ROW = 32    # mdp_set_sweep_form: the row form of the tile sweeps
ADJOINT_GROUP = 32   # mdp_set_adjoint_form: the group form of the adjoint sweep
ADJOINT_EXACT = 16   # mdp_set_adjoint_form: exact-shape adjoint kernels (+ occupancies per thread)
STATIC_PAID = -1    # static placement: the task went to the paid cloud
STATIC_EMPTY = -2   # static placement: empty task slot (need 0)
_NAMES = {EINVAL: "EINVAL", ERANGE: "ERANGE", ENOCONV: "ENOCONV", ENAN: "ENAN",
          EDEVICE: "EDEVICE", ENOMEM: "ENOMEM"}

# Every function the C ABI exports, with its ctypes signature.
_c_int64 = ctypes.c_int64
_c_int32 = ctypes.c_int32
_c_double = ctypes.c_double
_vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [("K", _c_int32), ("C", _c_int32), ("J", _c_int32),
                ("size", ctypes.POINTER(_c_int32)), ("lam", ctypes.POINTER(_c_double)),
                ("mu", _c_double), ("nu", _c_double),
                ("reward", ctypes.POINTER(_c_double)), ("reject_cost", ctypes.POINTER(_c_double)),
                ("gamma", _c_double), ("idle_unit_cost", _c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", _c_int64), ("residual_inf", _c_double), ("bound_inf", _c_double),
                ("seconds", _c_double), ("backups", _c_double), ("bytes", _c_double),
                ("sweep_seconds", _c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


SIGNATURES = {
    "mdp_build": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(_vp)]),
    "mdp_free": (None, [_vp]),
    "mdp_num_states": (_c_int64, [_vp]),
    "mdp_num_actions": (_c_int32, [_vp]),
    "mdp_feasible_pairs": (_c_int64, [_vp]),
    "vi_solve": (ctypes.c_int, [_vp, _vp, _c_double, _c_int64, _vp, ctypes.POINTER(Stats)]),
    "vi_solve_noalloc": (ctypes.c_int, [_vp, _vp, _c_double, _c_int64, _vp, ctypes.POINTER(Stats)]),
    "policy_extract": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "policy_extract_f64": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "policy_eval": (ctypes.c_int, [_vp, _vp, _vp, _c_double, _c_int64, _vp, ctypes.POINTER(Stats)]),
    "policy_greedy": (ctypes.c_int, [_vp, _c_int32, _vp, _vp]),
    "vi_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_c_double),
                                  ctypes.POINTER(_c_double), _c_double, _c_int64, _vp,
                                  ctypes.POINTER(Stats)]),
    "policy_objective": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_c_double), _vp]),
    "mdp_build_batch": (ctypes.c_int, [ctypes.POINTER(Params), _c_int32, ctypes.POINTER(_vp)]),
    "mdp_free_batch": (None, [_vp]),
    "batch_num_instances": (_c_int32, [_vp]),
    "batch_num_states": (_c_int64, [_vp, _c_int32]),
    "batch_feasible_pairs": (_c_int64, [_vp, _c_int32]),
    "batch_offsets": (ctypes.c_int, [_vp, ctypes.POINTER(_c_int64)]),
    "vi_solve_batch": (ctypes.c_int, [_vp, _vp, _c_double, _c_int64, _vp, ctypes.POINTER(Stats),
                                      ctypes.POINTER(_c_int64), ctypes.POINTER(_c_double)]),
    "policy_extract_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "policy_extract_batch_f64": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "policy_greedy_batch": (ctypes.c_int, [_vp, _c_int32, _vp, _vp]),
    "policy_eval_batch": (ctypes.c_int, [_vp, _vp, _vp, _c_double, _c_int64, _vp, ctypes.POINTER(Stats),
                                         ctypes.POINTER(_c_int64), ctypes.POINTER(_c_double)]),
    "vi_adjoint_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_c_double),
                                        ctypes.POINTER(_c_double), _c_double, _c_int64, _vp,
                                        ctypes.POINTER(Stats), ctypes.POINTER(_c_int64)]),
    "policy_iteration_batch": (ctypes.c_int, [_vp, _vp, _vp, _c_double, _c_int64, _c_double, _c_int64, _vp,
                                              ctypes.POINTER(Stats), ctypes.POINTER(_c_int64)]),
    "batch_set_round_form": (ctypes.c_int, [_vp, _c_int32, _c_int32]),
    "batch_round_forms": (ctypes.c_int, [_vp, ctypes.POINTER(_c_int32)]),
    "batch_set_tile_form": (ctypes.c_int, [_vp, _c_int32, _c_int32]),
    "batch_tile_form_instances": (_c_int32, [_vp, _c_int32]),
    "batch_autotune": (ctypes.c_int, [_vp, _c_int32, _vp, ctypes.POINTER(_c_int32),
                                      ctypes.POINTER(_c_double)]),
    "mdp_set_timing": (ctypes.c_int, [_vp, _c_int32]),
    "mdp_set_sweep_form": (ctypes.c_int, [_vp, _c_int32]),
    "vi_solve_bsdi": (ctypes.c_int, [_vp, _vp, _c_double, _c_int64, _c_int32, _vp, ctypes.POINTER(Stats)]),
    "policy_iteration": (ctypes.c_int, [_vp, _vp, _vp, _c_double, _c_int64, _c_double, _c_int64, _vp,
                                        ctypes.POINTER(Stats), ctypes.POINTER(_c_int64)]),
    "mdp_adjoint_form": (_c_int32, [_vp]),
    "mdp_set_adjoint_form": (ctypes.c_int, [_vp, _c_int32]),
    "mdp_sweep_forms": (ctypes.c_int, [_vp, ctypes.POINTER(_c_int32), ctypes.POINTER(_c_int32)]),
    "mdp_autotune": (ctypes.c_int, [_vp, _vp, _c_int32, _vp, ctypes.POINTER(_c_int32),
                                    ctypes.POINTER(_c_double)]),
    "static_first_fit": (ctypes.c_int, [_vp, _vp, _c_int64, _c_int32, _c_int64, _c_double, _c_double,
                                        _c_double, _vp, _vp, _vp, _vp, _vp, _vp]),
    "static_score": (ctypes.c_int, [_vp, _vp, _vp, _c_int64, _c_int32, _c_int64, _c_double, _c_double,
                                    _c_double, _vp, _vp, _vp, _vp, _vp]),
    "mdpvi_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmdpvi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2012_12419_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MdpviError(RuntimeError):
    def __init__(self, code: int, msg: str, stats: Optional[dict] = None):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.stats = stats


def _check(code: int, stats: Optional[Stats] = None):
    if code != OK:
        msg = load().mdpvi_last_error().decode()
        raise MdpviError(code, msg, stats.as_dict() if stats is not None else None)


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_tensor(t, dtype, n: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (there is no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def make_params(K: int, C: int, size: Sequence[int], lam: Sequence[float], mu: float, nu: float,
                reward: Sequence[float], gamma: float,
                reject_cost: Optional[Sequence[float]] = None, idle_unit_cost: float = 0.0):
    """ctypes Params plus the arrays it points into (keep both alive)."""
    J = len(size)
    keep = [(_c_int32 * J)(*[int(s) for s in size]), (_c_double * J)(*[float(x) for x in lam]),
            (_c_double * J)(*[float(x) for x in reward])]
    rc = (_c_double * J)(*[float(x) for x in reject_cost]) if reject_cost is not None else None
    keep.append(rc)
    p = Params(int(K), int(C), J, keep[0], keep[1], float(mu), float(nu), keep[2],
               ctypes.cast(rc, ctypes.POINTER(_c_double)) if rc is not None else None, float(gamma),
               float(idle_unit_cost))
    return p, keep


class MDP:
    """Handle of one MDP instance in libmdpvi."""

    def __init__(self, K: int, C: int, size: Sequence[int], lam: Sequence[float], mu: float,
                 nu: float, reward: Sequence[float], gamma: float,
                 reject_cost: Optional[Sequence[float]] = None, idle_unit_cost: float = 0.0):
        lib = load()
        p, keep = make_params(K, C, size, lam, mu, nu, reward, gamma, reject_cost, idle_unit_cost)
        h = ctypes.c_void_p()
        _check(lib.mdp_build(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.K, self.C, self.J = int(K), int(C), len(size)
        self.gamma = float(gamma)
        self.num_states = int(lib.mdp_num_states(h))
        self.num_actions = int(lib.mdp_num_actions(h))
        self.feasible_pairs = int(lib.mdp_feasible_pairs(h))
        self.n_occ = self.num_states // self.J

    @classmethod
    def from_instance(cls, inst) -> "MDP":
        return cls(inst.K, inst.C, inst.size, inst.lam, inst.mu, inst.nu, inst.reward,
                   inst.gamma, inst.reject_cost, getattr(inst, "idle_unit_cost", 0.0))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mdp_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on: bool = True):
        """Bracket every sweep with HIP events (stats['sweep_seconds'])."""
        _check(load().mdp_set_timing(self._h, 1 if on else 0))

    def set_sweep_form(self, slab_digits: int = -1):
        """-1 automatic, 0 direct, t in 1..K-1 LDS slab of t low digits,
        FORM_TILE the tile form (value iteration and evaluation)."""
        _check(load().mdp_set_sweep_form(self._h, int(slab_digits)))

    def sweep_forms(self):
        """(value-iteration form, evaluation form) the next solves will run."""
        a, b = _c_int32(), _c_int32()
        _check(load().mdp_sweep_forms(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def adjoint_form(self) -> int:
        """The adjoint sweep form the next vi_adjoint runs (mdp_adjoint_form)."""
        return int(load().mdp_adjoint_form(self._h))

    def set_adjoint_form(self, form: int = 0):
        """0 automatic, ADJOINT_GROUP the group form, ADJOINT_EXACT + t or t
        (t in 1, 2, 4 occupancies per thread) the exact-shape or generic
        kernels (mdp_set_adjoint_form)."""
        _check(load().mdp_set_adjoint_form(self._h, int(form)))

    def autotune(self, V=None, trials: int = 10, stream=None):
        """Time every sweep form on this instance; returns (best form, us per sweep)."""
        import torch
        if V is None:
            V = torch.zeros(self.num_states, dtype=torch.float32, device="cuda")
        f = _c_int32()
        us = _c_double()
        _check(load().mdp_autotune(self._h, _dev_tensor(V, torch.float32, self.num_states, "V"),
                                   int(trials), _stream_ptr(stream), ctypes.byref(f), ctypes.byref(us)))
        return f.value, us.value

    # --------------------------------------------------------------- calls
    def vi_solve(self, V, tol: float = 1e-6, max_iter: int = 1_000_000, stream=None) -> dict:
        import torch
        st = Stats()
        v = _dev_tensor(V, torch.float32, self.num_states, "V")
        _check(load().vi_solve(self._h, v, float(tol), int(max_iter), _stream_ptr(stream),
                               ctypes.byref(st)), st)
        return st.as_dict()

    def vi_solve_noalloc(self, V, tol: float = 1e-6, max_iter: int = 1_000_000, stream=None) -> dict:
        """vi_solve with all device scratch in the library's static array
        (vi_solve_noalloc: no device allocation; instances up to its 64 MiB)."""
        import torch
        st = Stats()
        v = _dev_tensor(V, torch.float32, self.num_states, "V")
        _check(load().vi_solve_noalloc(self._h, v, float(tol), int(max_iter), _stream_ptr(stream),
                                       ctypes.byref(st)), st)
        return st.as_dict()

    def vi_solve_bsdi(self, V, tol: float = 1e-6, inner: int = 4, max_iter: int = 1_000_000,
                      stream=None) -> dict:
        """Block-asynchronous passes of `inner` in-tile episodes (vi_solve_bsdi)."""
        import torch
        st = Stats()
        v = _dev_tensor(V, torch.float32, self.num_states, "V")
        _check(load().vi_solve_bsdi(self._h, v, float(tol), int(max_iter), int(inner), _stream_ptr(stream),
                                    ctypes.byref(st)), st)
        return st.as_dict()

    def policy_extract(self, V, pi=None, gap=None, want_gap: bool = True, stream=None):
        import torch
        n = self.num_states
        if pi is None:
            pi = torch.empty(n, dtype=torch.uint8, device=V.device)
        if gap is None and want_gap:
            gap = torch.empty(n, dtype=torch.float32, device=V.device)
        p = _dev_tensor(pi, torch.uint8, n, "pi")
        g = _dev_tensor(gap, torch.float32, n, "gap") if gap is not None else None
        if V.dtype == torch.float64:
            v = _dev_tensor(V, torch.float64, n, "V")
            _check(load().policy_extract_f64(self._h, v, p, g, _stream_ptr(stream)))
        else:
            v = _dev_tensor(V, torch.float32, n, "V")
            _check(load().policy_extract(self._h, v, p, g, _stream_ptr(stream)))
        return pi, gap

    def policy_eval(self, pi, V=None, tol: float = 1e-12, max_iter: int = 10_000_000,
                    stream=None):
        import torch
        n = self.num_states
        if V is None:
            V = torch.zeros(n, dtype=torch.float64, device=pi.device)
        st = Stats()
        _check(load().policy_eval(self._h, _dev_tensor(pi, torch.uint8, n, "pi"),
                                  _dev_tensor(V, torch.float64, n, "V"), float(tol),
                                  int(max_iter), _stream_ptr(stream), ctypes.byref(st)), st)
        return V, st.as_dict()

    def policy_iteration(self, pi, V=None, eval_tol: float = 1e-10, eval_max_iter: int = 10_000_000,
                         improve_tol: float = 1e-7, max_rounds: int = 100, stream=None):
        """Howard's policy iteration from pi (updated in place); returns
        (pi, V_pi, stats, rounds)."""
        import torch
        n = self.num_states
        if V is None:
            V = torch.zeros(n, dtype=torch.float64, device=pi.device)
        st = Stats()
        r = _c_int64()
        _check(load().policy_iteration(self._h, _dev_tensor(pi, torch.uint8, n, "pi"),
                                       _dev_tensor(V, torch.float64, n, "V"), float(eval_tol),
                                       int(eval_max_iter), float(improve_tol), int(max_rounds),
                                       _stream_ptr(stream),
                                       ctypes.byref(st), ctypes.byref(r)), st)
        return pi, V, st.as_dict(), r.value

    def policy_greedy(self, kind: str = "least_loaded", pi=None, stream=None):
        import torch
        code = {"least_loaded": 0, "first_fit": 1}[kind]
        if pi is None:
            pi = torch.empty(self.num_states, dtype=torch.uint8, device="cuda")
        _check(load().policy_greedy(self._h, code, _dev_tensor(pi, torch.uint8, self.num_states, "pi"),
                                    _stream_ptr(stream)))
        return pi

    def vi_adjoint(self, pi, V_pi, w=None, tol: float = 1e-10, max_iter: int = 10_000_000,
                   stream=None):
        """dJ/dtheta for theta = (lambda_1..J, mu, nu, r_1..J) at the fixed policy pi
        with value V_pi; returns (grad list, J, w, stats)."""
        import torch
        n = self.num_states
        if w is None:
            w = torch.zeros(n, dtype=torch.float32, device=pi.device)
        g = (_c_double * (2 * self.J + 2))()
        Jv = _c_double()
        st = Stats()
        _check(load().vi_adjoint(self._h, _dev_tensor(pi, torch.uint8, n, "pi"),
                                 _dev_tensor(V_pi, torch.float64, n, "V_pi"),
                                 _dev_tensor(w, torch.float32, n, "w"), g, ctypes.byref(Jv),
                                 float(tol), int(max_iter), _stream_ptr(stream), ctypes.byref(st)), st)
        return list(g), Jv.value, w, st.as_dict()

    def objective(self, V, stream=None) -> float:
        """J = sum_e lambda_e / sum_j lambda_j V(0, e) of a device FP64 value array."""
        import torch
        out = _c_double()
        _check(load().policy_objective(self._h, _dev_tensor(V, torch.float64, self.num_states, "V"),
                                       ctypes.byref(out), _stream_ptr(stream)))
        return out.value


class Batch:
    """Handle of a batch of independent instances (concatenated per-state arrays)."""

    def __init__(self, instances):
        lib = load()
        self._keep = []
        arr = (Params * len(instances))()
        for i, inst in enumerate(instances):
            prm, keep = make_params(inst.K, inst.C, inst.size, inst.lam, inst.mu, inst.nu,
                                    inst.reward, inst.gamma, inst.reject_cost,
                                    getattr(inst, "idle_unit_cost", 0.0))
            arr[i] = prm
            self._keep.append(keep)
        h = ctypes.c_void_p()
        _check(lib.mdp_build_batch(arr, len(instances), ctypes.byref(h)))
        self._h = h
        self.n = len(instances)
        self.num_states = int(lib.batch_num_states(h, -1))
        self.feasible_pairs = int(lib.batch_feasible_pairs(h, -1))
        offs = (_c_int64 * (self.n + 1))()
        _check(lib.batch_offsets(h, offs))
        self.offsets = list(offs)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mdp_free_batch(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    ROUND_OPS = {"vi": 0, "eval": 1, "adjoint": 2}

    def set_round_form(self, op: str, opt: int = 0):
        """Occupancies per thread (1, 2 or 4; 0 automatic) of the round
        kernels of op ("vi", "eval" or "adjoint")."""
        _check(load().batch_set_round_form(self._h, self.ROUND_OPS[op], int(opt)))

    def round_forms(self) -> dict:
        """The occupancies per thread the next calls use, per operation."""
        out = (_c_int32 * 3)()
        _check(load().batch_round_forms(self._h, out))
        return {k: int(out[v]) for k, v in self.ROUND_OPS.items()}

    def set_tile_form(self, op: str, mode: int = -1):
        """Tile form of the round kernels of op ("vi" or "eval") for the
        instances it covers: 1 on, 0 off, -1 automatic."""
        _check(load().batch_set_tile_form(self._h, self.ROUND_OPS[op], int(mode)))

    def tile_form_instances(self, op: str) -> int:
        """Instances the next call of op ("vi" or "eval") runs in the tile form."""
        return int(load().batch_tile_form_instances(self._h, self.ROUND_OPS[op]))

    def autotune(self, trials: int = 5, stream=None) -> dict:
        """Time the round kernels with 1, 2 and 4 occupancies per thread and
        record the fastest per operation, then the tile forms of "vi" and
        "eval" beside them; returns {op: (opt, us per round of the faster
        form)}."""
        opt = (_c_int32 * 3)(0, 0, 0)
        us = (_c_double * 3)(0.0, 0.0, 0.0)
        _check(load().batch_autotune(self._h, int(trials), _stream_ptr(stream), opt, us))
        return {k: (int(opt[v]), float(us[v])) for k, v in self.ROUND_OPS.items()}

    def vi_solve(self, V, tol: float = 1e-6, max_iter: int = 1_000_000, stream=None):
        """Returns (stats, iterations[n], residuals[n])."""
        import torch
        st = Stats()
        its = (_c_int64 * self.n)()
        res = (_c_double * self.n)()
        _check(load().vi_solve_batch(self._h, _dev_tensor(V, torch.float32, self.num_states, "V"),
                                     float(tol), int(max_iter), _stream_ptr(stream), ctypes.byref(st),
                                     its, res), st)
        return st.as_dict(), list(its), list(res)

    def policy_extract(self, V, pi=None, gap=None, want_gap: bool = True, stream=None):
        import torch
        n = self.num_states
        if pi is None:
            pi = torch.empty(n, dtype=torch.uint8, device=V.device)
        if gap is None and want_gap:
            gap = torch.empty(n, dtype=torch.float32, device=V.device)
        p = _dev_tensor(pi, torch.uint8, n, "pi")
        g = _dev_tensor(gap, torch.float32, n, "gap") if gap is not None else None
        if V.dtype == torch.float64:
            _check(load().policy_extract_batch_f64(self._h, _dev_tensor(V, torch.float64, n, "V"), p, g,
                                                   _stream_ptr(stream)))
        else:
            _check(load().policy_extract_batch(self._h, _dev_tensor(V, torch.float32, n, "V"), p, g,
                                               _stream_ptr(stream)))
        return pi, gap

    def policy_greedy(self, kind: str = "least_loaded", pi=None, stream=None):
        import torch
        if pi is None:
            pi = torch.empty(self.num_states, dtype=torch.uint8, device="cuda")
        _check(load().policy_greedy_batch(self._h, {"least_loaded": 0, "first_fit": 1}[kind],
                                          _dev_tensor(pi, torch.uint8, self.num_states, "pi"),
                                          _stream_ptr(stream)))
        return pi

    def policy_eval(self, pi, V=None, tol: float = 1e-12, max_iter: int = 10_000_000, stream=None):
        """Returns (V, stats, iterations[n], residuals[n])."""
        import torch
        n = self.num_states
        if V is None:
            V = torch.zeros(n, dtype=torch.float64, device=pi.device)
        st = Stats()
        its = (_c_int64 * self.n)()
        res = (_c_double * self.n)()
        _check(load().policy_eval_batch(self._h, _dev_tensor(pi, torch.uint8, n, "pi"),
                                        _dev_tensor(V, torch.float64, n, "V"), float(tol), int(max_iter),
                                        _stream_ptr(stream), ctypes.byref(st), its, res), st)
        return V, st.as_dict(), list(its), list(res)

    def policy_iteration(self, pi, V, eval_tol: float = 1e-12, eval_max_iter: int = 10_000_000,
                         improve_tol: float = 1e-9, max_rounds: int = 50, stream=None):
        """Per-instance policy iteration in place on pi (uint8) and V (FP64);
        returns (stats, evaluations per instance)."""
        import torch
        n = self.num_states
        st = Stats()
        rounds = (_c_int64 * self.n)()
        _check(load().policy_iteration_batch(self._h, _dev_tensor(pi, torch.uint8, n, "pi"),
                                             _dev_tensor(V, torch.float64, n, "V"), float(eval_tol),
                                             int(eval_max_iter), float(improve_tol), int(max_rounds),
                                             _stream_ptr(stream), ctypes.byref(st), rounds), st)
        return st.as_dict(), list(rounds)

    def vi_adjoint(self, pi, V_pi, J_sizes, w=None, tol: float = 1e-10, max_iter: int = 10_000_000,
                   stream=None):
        """Returns (list of per-instance gradients, objectives[n], w, stats, iterations[n])."""
        import torch
        n = self.num_states
        if w is None:
            w = torch.zeros(n, dtype=torch.float32, device=pi.device)
        total = sum(2 * J + 2 for J in J_sizes)
        g = (_c_double * total)()
        obj = (_c_double * self.n)()
        its = (_c_int64 * self.n)()
        st = Stats()
        _check(load().vi_adjoint_batch(self._h, _dev_tensor(pi, torch.uint8, n, "pi"),
                                       _dev_tensor(V_pi, torch.float64, n, "V_pi"),
                                       _dev_tensor(w, torch.float32, n, "w"), g, obj, float(tol),
                                       int(max_iter), _stream_ptr(stream), ctypes.byref(st), its), st)
        out, at = [], 0
        for J in J_sizes:
            out.append(list(g[at:at + 2 * J + 2]))
            at += 2 * J + 2
        return out, list(obj), w, st.as_dict(), list(its)


def _static_args(caps, need):
    import torch
    if caps.dim() != 2 or need.dim() != 2 or caps.shape[0] != need.shape[0]:
        raise ValueError("caps must be [B, K] and need [B, T] with the same B")
    B, K = caps.shape
    T = need.shape[1]
    c = _dev_tensor(caps, torch.int32, B * K, "caps")
    n = _dev_tensor(need, torch.int32, B * T, "need")
    out = dict(used=torch.empty((B, K), dtype=torch.int32, device=caps.device),
               totals=torch.empty((B, 3), dtype=torch.int64, device=caps.device),
               reward=torch.empty(B, dtype=torch.float64, device=caps.device),
               status=torch.empty(B, dtype=torch.int32, device=caps.device))
    return B, K, T, c, n, out


def static_first_fit(caps, need, beta_vc: float = 1.0, beta_tc: float = 1.2, gamma_vc: float = 1.0,
                     stream=None):
    """Fast greedy placement (Alg. 2) of B static scenarios: caps int32 [B, K]
    free VMs per VC, need int32 [B, T] VMs per task in arrival order (0 =
    empty slot).  Returns dict(place [B, T], used [B, K], totals [B, 3] =
    (VC VMs, paid VMs, idle VMs), reward [B], status [B]); asynchronous."""
    import torch
    B, K, T, c, n, out = _static_args(caps, need)
    out["place"] = torch.empty((B, T), dtype=torch.int32, device=caps.device)
    _check(load().static_first_fit(c, n, B, K, T, beta_vc, beta_tc, gamma_vc,
                                   ctypes.c_void_p(out["place"].data_ptr()),
                                   ctypes.c_void_p(out["used"].data_ptr()),
                                   ctypes.c_void_p(out["totals"].data_ptr()),
                                   ctypes.c_void_p(out["reward"].data_ptr()),
                                   ctypes.c_void_p(out["status"].data_ptr()), _stream_ptr(stream)))
    return out


def static_score(caps, need, place, beta_vc: float = 1.0, beta_tc: float = 1.2, gamma_vc: float = 1.0,
                 stream=None):
    """Cloud-wide reward (Eqs. (14)-(16)) of a given placement place int32
    [B, T] (VC index or STATIC_PAID).  Returns dict(used, totals, reward,
    status); asynchronous."""
    import torch
    B, K, T, c, n, out = _static_args(caps, need)
    p = _dev_tensor(place, torch.int32, B * T, "place")
    _check(load().static_score(c, n, p, B, K, T, beta_vc, beta_tc, gamma_vc,
                               ctypes.c_void_p(out["used"].data_ptr()),
                               ctypes.c_void_p(out["totals"].data_ptr()),
                               ctypes.c_void_p(out["reward"].data_ptr()),
                               ctypes.c_void_p(out["status"].data_ptr()), _stream_ptr(stream)))
    return out
