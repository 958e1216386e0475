"""ctypes binding of libfim (the C ABI declared in include/fim.h).

Argument marshalling only: every step of the solver runs in the HIP
kernels behind the C ABI.  There is no fallback: if the shared library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfim.so")

FIM_OK, FIM_NOT_CONVERGED = 0, 1
FIM_E_ARG, FIM_E_NOMEM, FIM_E_HIP, FIM_E_STATE, FIM_E_NONFINITE = -1, -2, -3, -4, -5
FULL, LOCAL, DD, RESID, DD_ADD = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
HOST, DEVICE = 0, 1
PC_JACOBI, PC_FRACTURE, PC_FRACTURE_COUPLED = 0, 1, 2
PSI = 6894.757293168


class FimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfim error {code}: {msg}")
        self.code = code


class NotConverged(RuntimeError):
    pass


class _Fluid(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p_ref", C.c_double),
                ("rho_ref", C.c_double), ("c", C.c_double), ("mu", C.c_double),
                ("rho_w", C.c_double), ("c_w", C.c_double), ("mu_w", C.c_double),
                ("rho_o", C.c_double), ("c_o", C.c_double), ("mu_o", C.c_double),
                ("swc", C.c_double), ("sor", C.c_double),
                ("rs_b", C.c_double), ("p_b", C.c_double), ("bo_slope", C.c_double),
                ("bg_c", C.c_double), ("rho_osc", C.c_double), ("rho_gsc", C.c_double),
                ("rho_wsc", C.c_double), ("mu_g", C.c_double), ("span", C.c_double)]


class _Desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_conn", C.c_int32), ("n_perf", C.c_int32),
                ("pv_ref", C.c_void_p), ("depth", C.c_void_p),
                ("always_active", C.c_void_p), ("conn_i", C.c_void_p),
                ("conn_j", C.c_void_p), ("conn_T", C.c_void_p),
                ("perf_cell", C.c_void_p), ("perf_wi", C.c_void_p),
                ("perf_bhp", C.c_void_p), ("c_r", C.c_double),
                ("p_ref_rock", C.c_double), ("gravity", C.c_double),
                ("fluid", _Fluid), ("frac_id", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("eps_conv", C.c_double), ("eps_loc", C.c_double), ("eps_s", C.c_double),
                ("tight", C.c_int32), ("m_layers", C.c_int32), ("m_layers_dd", C.c_int32),
                ("max_newton", C.c_int32), ("max_sweeps", C.c_int32),
                ("auto_cut", C.c_int32), ("max_cuts", C.c_int32), ("ds_max", C.c_double),
                ("precision", C.c_int32), ("lin_rtol", C.c_double),
                ("inner_rtol", C.c_double), ("krylov_maxit", C.c_int32),
                ("max_refine", C.c_int32), ("check_every", C.c_int32),
                ("precond", C.c_int32), ("eps_res", C.c_double),
                ("res_layers", C.c_int32), ("forcing_max", C.c_double)]


class IterStats(C.Structure):
    _fields_ = [("n_active", C.c_int32), ("n_boundary", C.c_int32),
                ("is_expand", C.c_int32), ("converged", C.c_int32),
                ("krylov_iters", C.c_int32), ("refine_passes", C.c_int32),
                ("n_switch", C.c_int32), ("nonfinite", C.c_int32),
                ("phase", C.c_int32), ("subdomain", C.c_int32),
                ("dp_max", C.c_double), ("ds_max", C.c_double),
                ("lin_relres", C.c_double), ("fp64_fallback", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelProfile(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64),
                ("total_ms", C.c_double), ("rows", C.c_double), ("nnzb", C.c_double),
                ("aux", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("cuts", C.c_int32), ("krylov_iters", C.c_int32),
                ("sum_active", C.c_double), ("max_active", C.c_int32),
                ("subdomains", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    # The library links libamdhip64.so.7 by soname.  PyTorch ships its own
    # HIP runtime under that soname; loading torch first makes the library
    # bind to the runtime torch uses, so one HIP runtime serves the process
    # (torch provides device memory and streams to the caller).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2008_01539_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, f64 = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "fim_default_options": (None, [vp]),
        "fim_create_model": (i32, [vp, vp, vp, vp]),
        "fim_set_state": (i32, [vp, vp, vp, i32]),
        "fim_get_state": (i32, [vp, vp, vp, i32]),
        "fim_checkpoint_bytes": (C.c_int64, [vp]),
        "fim_get_checkpoint": (i32, [vp, vp, C.c_int64]),
        "fim_set_checkpoint": (i32, [vp, vp, C.c_int64]),
        "fim_newton_step": (i32, [vp, f64, i32, vp]),
        "fim_newton_step_noalloc": (i32, [vp, f64, i32, vp]),
        "fim_solve_timestep": (i32, [vp, f64, i32, vp]),
        "fim_destroy_model": (i32, [vp]),
        "fim_last_error": (C.c_char_p, [vp]),
        "fim_num_cells": (i32, [vp]),
        "fim_block_size": (i32, [vp]),
        "fim_inspect_assemble": (i32, [vp, vp, vp, vp, f64, vp, vp, vp, vp, vp, vp, vp,
                                       C.c_int64]),
        "fim_inspect_sets": (i32, [vp, vp, vp, f64, i32, vp, vp, vp, vp, vp]),
        "fim_inspect_solve": (i32, [vp, vp, vp, vp]),
        "fim_inspect_pc_blocks": (i32, [vp, vp, vp, vp, vp, vp]),
        "fim_inspect_resid_error": (i32, [vp, vp, vp, vp, f64, vp]),
        "fim_inspect_resid_sets": (i32, [vp, vp, f64, i32, vp, vp, vp, vp]),
        "fim_inspect_dd_expand": (i32, [vp, vp, vp, vp, vp, f64, i32, vp, vp, vp, vp, vp,
                                        vp]),
        "fim_inspect_dd_pick": (i32, [vp, i32, vp, vp, vp, vp, vp, f64, i32, vp, vp, vp]),
        "fim_get_dd_total": (i32, [vp, vp, vp]),
        "fim_profile_enable": (i32, [vp, i32]),
        "fim_batch_create": (i32, [vp, i32, vp, vp]),
        "fim_model_bytes": (C.c_int64, [vp]),
        "fim_estimate_bytes": (C.c_int64, [vp, vp]),
        "fim_batch_set": (i32, [vp, vp, i32]),
        "fim_batch_newton_step": (i32, [vp, vp, vp, vp, vp]),
        "fim_batch_destroy": (i32, [vp]),
        "fim_batch_last_error": (C.c_char_p, [vp]),
        "fim_flags_enable": (i32, [vp, i32]),
        "fim_get_flags": (i32, [vp, vp]),
        "fim_profile_read": (i32, [vp, vp, i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


@dataclass
class Options:
    """Mirror of fim_options with its defaults: the paper's cutoffs and
    layers (Section 5); the linear-solve settings (tolerance, forcing term,
    precision, preconditioner) are readings where the paper is silent."""
    eps_conv: float = 0.3 * PSI
    eps_loc: float = 0.3 * PSI
    eps_s: float = 1e-10
    tight: int = 0
    m_layers: int = 2
    m_layers_dd: int = 4
    max_newton: int = 25
    max_sweeps: int = 40
    auto_cut: int = 0
    max_cuts: int = 8
    ds_max: float = 0.2
    precision: int = FP64
    lin_rtol: float = 1e-4
    inner_rtol: float = 1e-5
    krylov_maxit: int = 2000
    max_refine: int = 20
    check_every: int = 4
    precond: int = PC_FRACTURE
    eps_res: float = 1e-6
    res_layers: int = 1
    forcing_max: float = 0.1

    @staticmethod
    def tight_mode(**kw):
        o = Options(eps_conv=1e-7 * PSI, eps_loc=1e-7 * PSI, eps_s=1e-10, tight=1,
                    max_newton=40, lin_rtol=1e-12, forcing_max=0.0)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def _c(self):
        c = _Opts()
        for f in fields(self):
            setattr(c, f.name, getattr(self, f.name))
        return c


def _ptr(a):
    return a.ctypes.data if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(code, handle=None):
    if code < 0:
        msg = _lib.fim_last_error(handle).decode() if handle else "create failed"
        raise FimError(code, msg)
    return code


def _stream_handle(stream):
    if stream is not None:
        return stream
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _describe(model):
    """fim_model_desc for a model object (and the arrays it points to)."""
    fl = model.fluid
    f = _Fluid()
    f.kind = int(fl["kind"])
    for name, _ in _Fluid._fields_[1:]:
        if name in fl:
            setattr(f, name, float(fl[name]))
    keep = [_f64(model.pv_ref), _f64(model.depth),
            np.ascontiguousarray(model.always_active, dtype=np.uint8),
            _i32(model.conn_i), _i32(model.conn_j), _f64(model.conn_T),
            _i32(model.perf_cell), _f64(model.perf_wi), _f64(model.perf_bhp)]
    fid = (model.grid or {}).get("fid")
    frac = None
    if fid is not None and len(fid) == model.n - model.n_matrix:
        frac = np.full(model.n, -1, np.int32)
        frac[model.n_matrix:] = fid
    keep.append(frac)
    k = keep
    d = _Desc(n_cells=int(model.n), n_conn=int(k[3].size), n_perf=int(k[6].size),
              pv_ref=_ptr(k[0]), depth=_ptr(k[1]), always_active=_ptr(k[2]),
              conn_i=_ptr(k[3]), conn_j=_ptr(k[4]), conn_T=_ptr(k[5]),
              perf_cell=_ptr(k[6]), perf_wi=_ptr(k[7]), perf_bhp=_ptr(k[8]),
              c_r=float(model.rock["c_r"]), p_ref_rock=float(model.rock["p_ref"]),
              gravity=float(model.gravity), fluid=f, frac_id=_ptr(frac))
    return d, keep


def estimate_bytes(model, options: "Options | None" = None) -> int:
    """Device bytes FimModel(model) would allocate (no allocation)."""
    d, keep = _describe(model)
    o = (options or Options())._c()
    return int(_lib.fim_estimate_bytes(C.byref(d), C.byref(o)))


class FimModel:
    """One reservoir model resident on the GPU."""

    def __init__(self, model, options: Options | None = None, stream=None):
        self.options = options or Options()
        d, self._keep = _describe(model)
        opts = self.options._c()
        h = C.c_void_p()
        code = _lib.fim_create_model(C.byref(d), C.byref(opts), _stream_handle(stream),
                                     C.byref(h))
        if code != FIM_OK:
            raise FimError(code, "fim_create_model: " + _lib.fim_last_error(None).decode())
        self._h = h
        self.n = int(model.n)
        self.b = int(_lib.fim_block_size(h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.fim_destroy_model(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- state
    def set_state(self, u, status=None):
        """u: (b, n) numpy array (host) or a torch CUDA tensor (device)."""
        if hasattr(u, "data_ptr") and getattr(u, "is_cuda", False):
            st = status.data_ptr() if status is not None else None
            _check(_lib.fim_set_state(self._h, u.data_ptr(), st, DEVICE), self._h)
            return
        uu = _f64(u).reshape(self.b, self.n)
        st = np.ascontiguousarray(status, dtype=np.int8) if status is not None else None
        _check(_lib.fim_set_state(self._h, _ptr(uu), _ptr(st), HOST), self._h)

    def get_state(self):
        u = np.empty((self.b, self.n))
        st = np.empty(self.n, np.int8)
        _check(_lib.fim_get_state(self._h, _ptr(u), _ptr(st), HOST), self._h)
        return u, st

    def get_checkpoint(self):
        """The model's checkpoint between timesteps (state, phase status and
        the previous step's support set) as bytes."""
        nb = _lib.fim_checkpoint_bytes(self._h)
        buf = C.create_string_buffer(nb)
        _check(_lib.fim_get_checkpoint(self._h, buf, nb), self._h)
        return buf.raw

    def set_checkpoint(self, blob):
        """Restore a checkpoint written by get_checkpoint (same model)."""
        blob = bytes(blob)
        _check(_lib.fim_set_checkpoint(self._h, blob, len(blob)), self._h)

    def get_state_device(self, u_out, st_out=None):
        _check(_lib.fim_get_state(self._h, u_out.data_ptr(),
                                  st_out.data_ptr() if st_out is not None else None,
                                  DEVICE), self._h)

    # --------------------------------------------------------------- solving
    def newton_step(self, dt, mode=LOCAL):
        it = IterStats()
        code = _check(_lib.fim_newton_step(self._h, float(dt), int(mode), C.byref(it)), self._h)
        if code == FIM_NOT_CONVERGED:
            raise NotConverged(_lib.fim_last_error(self._h).decode())
        return it

    def newton_step_noalloc(self, dt, mode=LOCAL):
        """fim_newton_step without allocating (kernel scratch in the
        library's per-device static array)."""
        it = IterStats()
        code = _check(_lib.fim_newton_step_noalloc(self._h, float(dt), int(mode), C.byref(it)),
                      self._h)
        if code == FIM_NOT_CONVERGED:
            raise NotConverged(_lib.fim_last_error(self._h).decode())
        return it

    def solve_timestep(self, dt, mode=LOCAL, raise_on_fail=True):
        st = StepStats()
        code = _check(_lib.fim_solve_timestep(self._h, float(dt), int(mode), C.byref(st)),
                      self._h)
        if code == FIM_NOT_CONVERGED and raise_on_fail:
            raise NotConverged(_lib.fim_last_error(self._h).decode())
        return st

    def run(self, schedule, mode=LOCAL):
        """Advance through a schedule; returns the per-step statistics."""
        return [self.solve_timestep(dt, mode).as_dict() for dt in schedule]

    def device_bytes(self):
        return int(_lib.fim_model_bytes(self._h))

    # ---------------------------------------------------------- cell classes
    def record_flags(self, on=True):
        _check(_lib.fim_flags_enable(self._h, 1 if on else 0), self._h)

    def flags(self):
        out = np.empty(self.n, np.uint8)
        _check(_lib.fim_get_flags(self._h, _ptr(out)), self._h)
        return out

    # ------------------------------------------------------------ profiling
    def profile(self, on=True):
        _check(_lib.fim_profile_enable(self._h, 1 if on else 0), self._h)

    def profile_read(self):
        arr = (KernelProfile * 16)()
        k = _lib.fim_profile_read(self._h, arr, 16)
        return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                           rows=arr[i].rows, nnzb=arr[i].nnzb,
                                           aux=arr[i].aux)
                for i in range(k)}

    # ------------------------------------------------------------ inspection
    def inspect_assemble(self, u_old, u_iter, status, dt, act=None, cap_blocks=None):
        n, b = self.n, self.b
        cap = int(cap_blocks or 16 * n)
        uo, ui = _f64(u_old).reshape(b, n), _f64(u_iter).reshape(b, n)
        st = np.ascontiguousarray(status, np.int8) if status is not None else None
        ac = np.ascontiguousarray(act, np.uint8) if act is not None else None
        nA = C.c_int32()
        l2g = np.empty(n, np.int32)
        F = np.empty(n * b)
        rp = np.empty(n + 1, np.int32)
        col = np.empty(cap, np.int32)
        val = np.empty(cap * b * b)
        _check(_lib.fim_inspect_assemble(self._h, _ptr(uo), _ptr(ui), _ptr(st), float(dt),
                                         _ptr(ac), C.byref(nA), _ptr(l2g), _ptr(F), _ptr(rp),
                                         _ptr(col), _ptr(val), cap), self._h)
        na = nA.value
        nz = rp[na]
        return dict(n_active=na, l2g=l2g[:na].copy(), F=F[:na * b].reshape(na, b),
                    row_ptr=rp[:na + 1].copy(), col=col[:nz].copy(),
                    val=val[:nz * b * b].reshape(nz, b, b))

    def inspect_solve(self):
        x = np.empty(self.n * self.b)
        it = C.c_int32()
        rr = C.c_double()
        _check(_lib.fim_inspect_solve(self._h, _ptr(x), C.byref(it), C.byref(rr)), self._h)
        return x, it.value, rr.value

    def inspect_sets(self, act_in, dp_abs, eps, layers):
        n = self.n
        a = np.ascontiguousarray(act_in, np.uint8)
        dp = _f64(dp_abs)
        ao = np.empty(n, np.uint8)
        bo = np.empty(n, np.uint8)
        l2g = np.empty(n, np.int32)
        na = C.c_int32()
        ex = C.c_int32()
        _check(_lib.fim_inspect_sets(self._h, _ptr(a), _ptr(dp), float(eps), int(layers),
                                     _ptr(ao), _ptr(bo), _ptr(l2g), C.byref(na), C.byref(ex)),
               self._h)
        return dict(act=ao, bnd=bo, l2g=l2g[:na.value].copy(), n_active=na.value,
                    is_expand=bool(ex.value))

    def inspect_resid_error(self, u_old, u_iter, status, dt):
        n, b = self.n, self.b
        uo, ui = _f64(u_old).reshape(b, n), _f64(u_iter).reshape(b, n)
        st = np.ascontiguousarray(status, np.int8) if status is not None else None
        err = np.empty(n)
        _check(_lib.fim_inspect_resid_error(self._h, _ptr(uo), _ptr(ui), _ptr(st), float(dt),
                                            _ptr(err)), self._h)
        return err

    def inspect_pc_blocks(self, act=None):
        """Fracture-block layout for the active set act (None: all cells):
        n_active, l2g and per active row the first row of its block and its
        rows."""
        n = self.n
        a = None if act is None else np.ascontiguousarray(act, np.uint8).reshape(n)
        l2g = np.empty(n, np.int32)
        bs = np.empty(n, np.int32)
        br = np.empty(n, np.int32)
        na = C.c_int32()
        _check(_lib.fim_inspect_pc_blocks(self._h, _ptr(a), C.byref(na), _ptr(l2g), _ptr(bs),
                                          _ptr(br)), self._h)
        k = na.value
        return dict(n_active=k, l2g=l2g[:k].copy(), blk_start=bs[:k].copy(),
                    blk_rows=br[:k].copy())

    def inspect_resid_sets(self, err, tol, layers):
        n = self.n
        e = _f64(err)
        ao = np.empty(n, np.uint8)
        l2g = np.empty(n, np.int32)
        na = C.c_int32()
        nu = C.c_int32()
        _check(_lib.fim_inspect_resid_sets(self._h, _ptr(e), float(tol), int(layers), _ptr(ao),
                                           _ptr(l2g), C.byref(na), C.byref(nu)), self._h)
        return dict(act=ao, l2g=l2g[:na.value].copy(), n_active=na.value,
                    n_unconverged=nu.value)

    def inspect_dd_expand(self, vt, act, bnd, dp_abs, eps, layers):
        n = self.n
        vi, ai, bi = (np.ascontiguousarray(x, np.uint8).reshape(n) for x in (vt, act, bnd))
        dp = _f64(dp_abs)
        vo, ao, bo, oo = (np.empty(n, np.uint8) for _ in range(4))
        na = C.c_int32()
        ex = C.c_int32()
        _check(_lib.fim_inspect_dd_expand(self._h, _ptr(vi), _ptr(ai), _ptr(bi), _ptr(dp),
                                          float(eps), int(layers), _ptr(vo), _ptr(ao),
                                          _ptr(bo), _ptr(oo), C.byref(na), C.byref(ex)),
               self._h)
        return dict(vt=vo, act=ao, bnd=bo, outer=oo, n_active=na.value,
                    is_expand=bool(ex.value))

    def inspect_dd_pick(self, cells, outers, last_dp, eps, nxt):
        """cells, outers: lists of index arrays, one per subdomain."""
        k = len(cells)
        cp = np.zeros(k + 1, np.int32)
        op = np.zeros(k + 1, np.int32)
        cp[1:] = np.cumsum([len(c) for c in cells])
        op[1:] = np.cumsum([len(c) for c in outers])
        cc = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in cells])
                                  if cp[-1] else np.zeros(1, np.int32), np.int32)
        oc = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in outers])
                                  if op[-1] else np.zeros(1, np.int32), np.int32)
        ld = _f64(last_dp)
        smax = np.empty(k)
        pick = C.c_int32()
        nsw = C.c_int32()
        _check(_lib.fim_inspect_dd_pick(self._h, k, _ptr(cp), _ptr(cc), _ptr(op), _ptr(oc),
                                        _ptr(ld), float(eps), int(nxt), _ptr(smax),
                                        C.byref(pick), C.byref(nsw)), self._h)
        return smax, pick.value, bool(nsw.value)

    def dd_total(self):
        """V_T of the most recent Algorithm 2 timestep and its subdomain
        count."""
        vt = np.empty(self.n, np.uint8)
        ns = C.c_int32()
        _check(_lib.fim_get_dd_total(self._h, _ptr(vt), C.byref(ns)), self._h)
        return vt, ns.value


class FimBatch:
    """Several models advanced together: one Newton iteration of every
    member per call, with one batched Krylov solve over all of them.  A
    member's result is the same alone and in any batch."""

    @staticmethod
    def _handles(models):
        if any(m._h is None for m in models):
            raise FimError(FIM_E_ARG, "a batch member has been closed")
        return (C.c_void_p * len(models))(*[m._h.value for m in models])

    def __init__(self, models, stream=None):
        self._h = None
        self._models = list(models)
        arr = self._handles(self._models)
        h = C.c_void_p()
        code = _lib.fim_batch_create(arr, len(self._models), _stream_handle(stream), C.byref(h))
        if code != FIM_OK:
            raise FimError(code, "fim_batch_create: " + _lib.fim_batch_last_error(None).decode())
        self._h = h

    @property
    def models(self):
        return list(self._models)

    def set_models(self, models):
        """Replace the membership (between calls)."""
        arr = self._handles(list(models))
        self._models = list(models)
        code = _lib.fim_batch_set(self._h, arr, len(self._models))
        if code != FIM_OK:
            raise FimError(code, _lib.fim_batch_last_error(self._h).decode())

    def newton_step(self, dts, modes):
        """One Newton iteration of every member; returns (stats, codes)."""
        self._handles(self._models)
        k = len(self._models)
        d = np.ascontiguousarray(dts, dtype=np.float64).reshape(k)
        mo = np.ascontiguousarray(modes, dtype=np.int32).reshape(k)
        st = (IterStats * k)()
        codes = np.zeros(k, np.int32)
        code = _lib.fim_batch_newton_step(self._h, _ptr(d), _ptr(mo), st, _ptr(codes))
        if code != FIM_OK:
            raise FimError(code, _lib.fim_batch_last_error(self._h).decode())
        return [st[i].as_dict() for i in range(k)], codes

    def close(self):
        if self._h:
            _lib.fim_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols():
    """Names of the functions the C header declares (for load checks)."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "fim.h")
    with open(hdr) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(fim_[a-z_]+)\s*\(", txt)))
