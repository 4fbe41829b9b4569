"""stfdfd: MI355X (gfx950) overlapping-PML source-transfer FDFD solver.

Thin Python binding over the C ABI declared in include/stfdfd.h.  It only
marshals arguments (NumPy host arrays or torch device tensors -> pointers);
every step of the solver runs in the HIP library.  If libstfdfd.so is not built
the calls raise: there is no CPU fallback.

Arrays: complex128, node arrays shaped (ny, nx) (x fastest), cell maps
(ny+1, nx+1).  NumPy arrays are host buffers; torch CUDA tensors are device
buffers used in place on the context's stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

from . import _abi
from ._abi import (STF_C128, STF_C64, STF_X0_USER, STF_X0_ZERO, STF_X0_LEARNED,  # noqa: F401
                   KERNEL_CLASSES, STATUS_NAMES)

__all__ = ["Context", "Problem", "Network", "StfError", "plan_query", "debug_local_axes", "debug_level_shapes", "batch_solve",
           "make_params", "nn_param_count", "STF_C128", "STF_C64", "STF_X0_ZERO", "STF_X0_USER",
           "STF_X0_LEARNED", "KERNEL_CLASSES"]


class StfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def make_params(nx, ny, k0, dx=1.0, dy=1.0, pml=(0, 0, 0, 0), pml_order=3, pml_R=1e-8, px=1,
                py=1, overlap=0, local_pml=0, local_pml_order=3, local_pml_R=1e-8,
                front_prec=STF_C128, leaf_size=0):
    p = _abi.Params()
    p.nx, p.ny, p.dx, p.dy, p.k0 = int(nx), int(ny), float(dx), float(dy), float(k0)
    for i in range(4):
        p.pml[i] = int(pml[i])
    p.pml_order, p.pml_R = int(pml_order), float(pml_R)
    p.px, p.py, p.overlap, p.local_pml = int(px), int(py), int(overlap), int(local_pml)
    p.local_pml_order, p.local_pml_R = int(local_pml_order), float(local_pml_R)
    p.front_prec, p.leaf_size = int(front_prec), int(leaf_size)
    return p


def _params(prm):
    if isinstance(prm, _abi.Params):
        return prm
    return make_params(**prm)


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, n_complex, name):
    """(pointer, on_device, keepalive) for a complex128 array of n_complex entries."""
    if _is_torch(a):
        import torch
        if a.dtype != torch.complex128:
            raise TypeError("%s must be torch.complex128" % name)
        if not a.is_cuda or not a.is_contiguous():
            raise TypeError("%s must be a contiguous CUDA tensor" % name)
        if a.numel() != n_complex:
            raise ValueError("%s has %d entries, expected %d" % (name, a.numel(), n_complex))
        return C.c_void_p(a.data_ptr()), 1, a
    arr = np.ascontiguousarray(a, dtype=np.complex128)
    if arr.size != n_complex:
        raise ValueError("%s has %d entries, expected %d" % (name, arr.size, n_complex))
    return C.c_void_p(arr.ctypes.data), 0, arr


def _check(ctx_handle, status, allow=()):
    if status != 0 and status not in allow:
        msg = _abi.load().stf_last_error(ctx_handle)
        raise StfError(status, msg.decode() if msg else "")
    return status


def plan_query(prm):
    """Host-only plan statistics (partition and nested-dissection fronts)."""
    lib = _abi.load()
    info = _abi.PlanInfo()
    st = lib.stf_plan_query(C.byref(_params(prm)), C.byref(info))
    if st != 0:
        raise StfError(st, "invalid parameters")
    return {f: getattr(info, f) for f, _ in _abi.PlanInfo._fields_}


def debug_level_shapes(prm, nrhs=4):
    """Host-only: (levels, candidate shapes, invalid shapes) of the launch-shape
    rules on the plan of `prm`."""
    lib = _abi.load()
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    st = lib.stf_debug_level_shapes(C.byref(_params(prm)), int(nrhs), C.byref(a), C.byref(b), C.byref(c))
    if st != 0:
        raise StfError(st, "invalid parameters")
    return a.value, b.value, c.value


def debug_local_axes(prm, k):
    """Host-only: local coupling coefficients (cw, ce, cs, cn) of subdomain k and its boxes."""
    lib = _abi.load()
    p = _params(prm)
    dims = (C.c_int32 * 8)()
    st = lib.stf_debug_local_axes(C.byref(p), int(k), dims, None, None, None, None)
    if st != 0:
        raise StfError(st, "invalid parameters or subdomain")
    ox0, oy0, nxl, nyl, ix0, ix1, iy0, iy1 = list(dims)
    cw = np.zeros(nxl, np.complex128); ce = np.zeros(nxl, np.complex128)
    cs = np.zeros(nyl, np.complex128); cn = np.zeros(nyl, np.complex128)
    st = lib.stf_debug_local_axes(C.byref(p), int(k), dims, cw.ctypes.data, ce.ctypes.data,
                                  cs.ctypes.data, cn.ctypes.data)
    if st != 0:
        raise StfError(st, "invalid parameters or subdomain")
    return dict(ox=(ox0, ox0 + nxl), oy=(oy0, oy0 + nyl), ix=(ix0, ix1), iy=(iy0, iy1),
                cw=cw, ce=ce, cs=cs, cn=cn)


_live_contexts = weakref.WeakSet()


@atexit.register
def _close_all():
    # Release device state while the HIP runtime is still alive (Python's own
    # finalisation order of leftover objects is arbitrary).
    for c in list(_live_contexts):
        c.close()


def _what(factor, sweeps, orders):
    what = (1 if factor else 0) | (2 if sweeps else 0)
    for o in orders:
        if o not in _abi.ORDERS or o == "additive":
            raise ValueError("staged orders: rows, rows_cols, diagonal, checker")
        what |= 2 << _abi.ORDERS[o]
    return what


class Context:
    """Device context.  stream: a hipStream_t handle (int) or a torch stream; by
    default the current torch stream of `device` (so torch and library work are
    ordered), or the library's own stream when torch is unavailable."""

    def __init__(self, device=0, stream=None):
        self._lib = _abi.load()
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = 0
        elif hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        h = C.c_void_p()
        st = self._lib.stf_ctx_create(int(device), C.c_void_p(int(stream) or None), C.byref(h))
        if st != 0:
            msg = self._lib.stf_last_error(None)
            raise StfError(st, "stf_ctx_create: " + (msg.decode() if msg else ""))
        self.handle = h
        self.device = device
        self._problems = weakref.WeakSet()
        self._networks = weakref.WeakSet()
        _live_contexts.add(self)

    def close(self):
        """Destroy the context and every problem and network created on it (those first)."""
        if getattr(self, "handle", None):
            for pb in list(self._problems):
                pb.close()
            for nn in list(self._networks):
                nn.close()
            self._lib.stf_ctx_destroy(self.handle)
            self.handle = None

    def set_nn(self, net):
        """Network used by solves with x0="learned" (None detaches)."""
        _check(self.handle, self._lib.stf_ctx_set_nn(self.handle, net.handle if net else None))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on, classes=None):
        """Per-launch HIP event timing: on/off for all classes, or only for the
        named classes (KERNEL_CLASSES entries) when `classes` is given."""
        if classes is None:
            _check(self.handle, self._lib.stf_ctx_set_timing(self.handle, int(bool(on))))
            return
        mask = 0
        if on:
            for c in classes:
                mask |= 1 << (KERNEL_CLASSES.index(c) if isinstance(c, str) else int(c))
        _check(self.handle, self._lib.stf_ctx_set_timing_mask(self.handle, mask))

    def autotune(self, problems, nrhs=4, factor=True, sweeps=True, reps=3, orders=()):
        """Time every candidate launch shape of each tree level (factorisation
        and/or the round's sweeps with `nrhs` right-hand sides) of one problem, or
        of the set a batched solve builds for `problems`, and keep the fastest per
        level signature on this context; `orders` (names of staged orders) adds
        the subtree choice of their stages.  Leaves the problems factored.
        Returns the report as a dict."""
        if isinstance(problems, Problem):
            problems = [problems]
        what = _what(factor, sweeps, orders)
        arr = (C.c_void_p * len(problems))(*[p.handle.value for p in problems])
        rep = _abi.TuneReport()
        _check(self.handle, self._lib.stf_autotune(self.handle, len(problems), arr, int(nrhs), what,
                                                   int(reps), C.byref(rep)))
        return {f: getattr(rep, f) for f, _ in _abi.TuneReport._fields_}

    def tune_pick(self, problems, index, nrhs=4, factor=True, sweeps=True, orders=()):
        """Test hook: every level's shape (and the subtree choices of the
        additive round and of `orders`) set to candidate `index` (clamped);
        returns the largest candidate count."""
        if isinstance(problems, Problem):
            problems = [problems]
        what = _what(factor, sweeps, orders)
        arr = (C.c_void_p * len(problems))(*[p.handle.value for p in problems])
        most = C.c_int32()
        _check(self.handle, self._lib.stf_tune_pick(self.handle, len(problems), arr, int(nrhs), what,
                                                    int(index), C.byref(most)))
        return most.value

    def tune_save(self, path):
        _check(self.handle, self._lib.stf_tune_save(self.handle, os.fsencode(path)))

    def tune_load(self, path):
        _check(self.handle, self._lib.stf_tune_load(self.handle, os.fsencode(path)))

    def tune_clear(self):
        _check(self.handle, self._lib.stf_tune_clear(self.handle))

    def tune_entries(self):
        """The tuned shapes: list of (key, shape, (ms_chosen, ms_builtin)) with
        key = (op, elem, nrhs, fronts, max_m, max_p), shape = (kind, a, b, c)."""
        out = []
        for i in range(self._lib.stf_tune_count(self.handle)):
            key, shape, ms = (C.c_int32 * 6)(), (C.c_int32 * 4)(), (C.c_double * 2)()
            _check(self.handle, self._lib.stf_tune_entry(self.handle, i, key, shape, ms))
            out.append((tuple(key), tuple(shape), tuple(ms)))
        return out

    def kernel_stats(self, cls):
        if isinstance(cls, str):
            cls = KERNEL_CLASSES.index(cls)
        ms, n = C.c_double(), C.c_int64()
        _check(self.handle, self._lib.stf_ctx_kernel_stats(self.handle, int(cls), C.byref(ms),
                                                           C.byref(n)))
        return ms.value, n.value


class Problem:
    """An assembled problem: global operator, partition, symbolic plans, factors."""

    def __init__(self, ctx, prm, eps_cells):
        self.ctx = ctx
        self._lib = ctx._lib
        self.params = _params(prm)
        self.nx, self.ny = self.params.nx, self.params.ny
        ptr, dev, keep = _ptr(eps_cells, (self.nx + 1) * (self.ny + 1), "eps_cells")
        h = C.c_void_p()
        _check(ctx.handle, self._lib.stf_problem_create(ctx.handle, C.byref(self.params), ptr, dev,
                                                        C.byref(h)))
        self.handle = h
        ctx._problems.add(self)

    def close(self):
        # A problem must be destroyed before its context; closing the context
        # closes its problems, so a problem whose context is gone is already freed.
        if getattr(self, "handle", None) and getattr(self.ctx, "handle", None):
            self._lib.stf_problem_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ndof(self):
        return self.nx * self.ny

    def assemble(self, eps_cells):
        ptr, dev, keep = _ptr(eps_cells, (self.nx + 1) * (self.ny + 1), "eps_cells")
        _check(self.ctx.handle, self._lib.stf_assemble(self.handle, ptr, dev))

    def factor(self):
        """Returns True if a pivot was perturbed (STF_EPIVOT)."""
        st = _check(self.ctx.handle, self._lib.stf_factor(self.handle), allow=(_abi.STF_EPIVOT,))
        return st == _abi.STF_EPIVOT

    def _out_like(self, a, shape):
        if _is_torch(a):
            import torch
            return torch.empty(shape, dtype=torch.complex128, device=a.device)
        return np.empty(shape, dtype=np.complex128)

    def apply(self, x, y=None):
        n = self.ndof
        px, dev, kx = _ptr(x, n, "x")
        y = self._out_like(x, (self.ny, self.nx)) if y is None else y
        py_, dev2, ky = _ptr(y, n, "y")
        if dev != dev2:
            raise TypeError("x and y must both be host or both be device arrays")
        _check(self.ctx.handle, self._lib.stf_apply(self.handle, px, py_, dev))
        return y if dev else ky.reshape(self.ny, self.nx)

    def precond(self, v, z=None):
        """One source-transfer round; v shaped (ny, nx) or (nrhs, ny, nx) (swept together)."""
        shape = tuple(v.shape)
        nrhs = 1 if len(shape) == 2 else int(shape[0])
        n = self.ndof
        pv, dev, kv = _ptr(v, nrhs * n, "v")
        z = self._out_like(v, shape) if z is None else z
        pz, dev2, kz = _ptr(z, nrhs * n, "z")
        if dev != dev2:
            raise TypeError("v and z must both be host or both be device arrays")
        if len(shape) == 2:
            _check(self.ctx.handle, self._lib.stf_precond_apply(self.handle, pv, pz, dev))
        else:
            _check(self.ctx.handle, self._lib.stf_precond_apply_batch(self.handle, nrhs, pv, pz, dev))
        return z if dev else kz.reshape(shape)

    def sweep(self, v, order, z=None):
        """One preconditioner application in a staged order ("rows", "rows_cols",
        "diagonal", "checker"; "additive" is the round of precond())."""
        n = self.ndof
        pv, dev, kv = _ptr(v, n, "v")
        z = self._out_like(v, tuple(v.shape)) if z is None else z
        pz, dev2, kz = _ptr(z, n, "z")
        if dev != dev2:
            raise TypeError("v and z must both be host or both be device arrays")
        _check(self.ctx.handle, self._lib.stf_sweep_apply(self.handle, _order(order), pv, pz, dev))
        return z if dev else kz.reshape(tuple(v.shape))

    def precond_noalloc(self, v, z):
        """One source-transfer round into the preallocated z with the library's
        static workspace (no device allocation); v, z: complex128 CUDA tensors
        shaped (ny, nx).  Enqueued on the context stream, not synchronised."""
        n = self.ndof
        _check(self.ctx.handle, self._lib.stf_precond_apply_noalloc(
            self.handle, _cptr(v, n, "v"), _cptr(z, n, "z")))
        return z

    def line_flux(self, e, axis, index, lo, hi):
        """Power through the grid line between node rows (axis 1) or columns
        (axis 0) index and index + 1, nodes [lo, hi) along it: the line integral
        of Re(E x H*) / 2 (towards +y or +x)."""
        pe, dev, ke = _ptr(e, self.ndof, "e")
        out = C.c_double(0.0)
        _check(self.ctx.handle, self._lib.stf_line_flux(self.handle, pe, dev, int(axis), int(index),
                                                        int(lo), int(hi), C.byref(out)))
        return out.value

    def rcs(self, e, box, phis):
        """(sigma, F) of the scattered field e by the near-to-far-field transform
        over the contour around node box (i0, i1, j0, j1) at angles phis."""
        pe, dev, ke = _ptr(e, self.ndof, "e")
        ph = np.ascontiguousarray(phis, dtype=np.float64)
        bx = (C.c_int32 * 4)(*[int(v) for v in box])
        sig = np.zeros(ph.size, dtype=np.float64)
        F = np.zeros(ph.size, dtype=np.complex128)
        _check(self.ctx.handle, self._lib.stf_rcs(self.handle, pe, dev, bx, ph.size, ph.ctypes.data,
                                                  sig.ctypes.data, F.ctypes.data))
        return sig, F

    def stationary_solve(self, b, x=None, tol=1e-10, max_rounds=100, stop="residual"):
        """Algorithm 1 as a stationary iteration of source-transfer rounds:
        x_0 = B b, then x <- x + B (b - A x) until the stop rule holds ("residual":
        FP64 true relative residual <= tol; "overlap": Eq. (20), the summed
        overlap-field norms below tol times the initial ones) or max_rounds
        rounds.  Returns (x, info) with info = dict(rounds, status, relres_true,
        hist, energy) (hist / energy: relative residual / overlap energy of x_0
        and of every round)."""
        n = self.ndof
        pb_, dev, kb = _ptr(b, n, "b")
        x = self._out_like(b, tuple(b.shape)) if x is None else x
        px, dev2, kx = _ptr(x, n, "x")
        if dev != dev2:
            raise TypeError("b and x must both be host or both be device arrays")
        hist = np.zeros(int(max_rounds) + 1, dtype=np.float64)
        energy = np.zeros(int(max_rounds) + 1, dtype=np.float64)
        k = C.c_int32(0)
        rule = {"residual": 0, "overlap": 1}[stop]
        st = self._lib.stf_stationary_solve(self.handle, pb_, px, dev, float(tol), int(max_rounds),
                                            rule, hist.ctypes.data, energy.ctypes.data, C.byref(k))
        _check(self.ctx.handle, st, allow=(_abi.STF_ENOCONV,))
        h = hist[:k.value + 1].tolist()
        info = dict(rounds=k.value, status=st, relres_true=h[-1], hist=h,
                    energy=energy[:k.value + 1].tolist())
        return (x if dev else kx.reshape(tuple(b.shape))), info

    def solve(self, b, x=None, tol=1e-10, restart=30, max_iter=500, x0=None, history_cap=4096,
              raise_on_noconv=False, rounds=1, debug_fault=0, order="additive"):
        """Solve A x = b; b shaped (ny, nx) or (nrhs, ny, nx).  Returns (x, infos).
        x0: None (zero guess), an array (user guess) or "learned" (the context's network).
        debug_fault=1 re-factors with one planted zero pivot column first (test hook of the
        tiny-pivot path); the call then reports STF_EPIVOT as info["epivot"]."""
        return self._solve(self._lib.stf_solve, b, x, tol, restart, max_iter, x0, history_cap,
                           raise_on_noconv, rounds, debug_fault, order)

    def factor_solve(self, b, x=None, tol=1e-10, restart=30, max_iter=500, x0=None,
                     history_cap=4096, raise_on_noconv=False, rounds=1, order="additive"):
        """factor() then solve() in one call (stf_factor_solve); with x0="learned" and
        device arrays the network's guesses run during the factorisation."""
        return self._solve(self._lib.stf_factor_solve, b, x, tol, restart, max_iter, x0,
                           history_cap, raise_on_noconv, rounds, 0, order)

    def _solve(self, fn, b, x, tol, restart, max_iter, x0, history_cap, raise_on_noconv, rounds,
               debug_fault, order):
        shape = tuple(b.shape)
        nrhs = 1 if len(shape) == 2 else int(shape[0])
        n = self.ndof
        pb_, dev, kb = _ptr(b, nrhs * n, "b")
        mode = _abi.STF_X0_ZERO
        if isinstance(x0, str):
            if x0 != "learned":
                raise ValueError("x0 must be None, an array or 'learned'")
            mode = _abi.STF_X0_LEARNED
            x0 = None
            if x is None:
                x = self._out_like(b, shape)
        elif x0 is not None:
            mode = _abi.STF_X0_USER
            if _is_torch(x0):
                x = x0.clone()
            else:
                x = np.array(x0, dtype=np.complex128, copy=True)
        elif x is None:
            x = self._out_like(b, shape)
        pxx, dev2, kx = _ptr(x, nrhs * n, "x")
        if dev != dev2:
            raise TypeError("b and x must both be host or both be device arrays")
        opts = _abi.SolveOpts(float(tol), int(restart), int(max_iter), mode, int(rounds),
                              int(debug_fault), _order(order))
        infos = (_abi.SolveInfo * nrhs)()
        hist = [np.zeros(history_cap, dtype=np.float64) for _ in range(nrhs)]
        for i in range(nrhs):
            infos[i].history = hist[i].ctypes.data_as(C.POINTER(C.c_double))
            infos[i].history_cap = history_cap
        allow = (_abi.STF_EPIVOT,) if raise_on_noconv else (_abi.STF_ENOCONV, _abi.STF_EPIVOT)
        st = _check(self.ctx.handle, fn(self.handle, nrhs, pb_, pxx, dev, C.byref(opts), infos),
                    allow=allow)
        out = []
        for i in range(nrhs):
            inf = infos[i]
            out.append(dict(iters=inf.iters, restarts=inf.restarts, status=inf.status,
                            relres_true=inf.relres_true, relres_x0=inf.relres_x0,
                            used_learned=inf.used_learned, epivot=st == _abi.STF_EPIVOT,
                            t_factor_ms=inf.t_factor_ms, t_solve_ms=inf.t_solve_ms,
                            t_nn_ms=inf.t_nn_ms, history=hist[i][:inf.history_len].copy()))
        xo = x if dev else kx.reshape(shape)
        return xo, out

    def info(self):
        pi = _abi.PlanInfo()
        _check(self.ctx.handle, self._lib.stf_problem_info(self.handle, C.byref(pi)))
        return {f: getattr(pi, f) for f, _ in _abi.PlanInfo._fields_}

    def tile_data(self, net, b=None, x=None):
        """(features, fields) of this problem's tiles as float32 CUDA tensors
        (device b and x, either may be None)."""
        import torch
        nt = C.c_int32()
        _check(self.ctx.handle, self._lib.stf_nn_tile_data(self.handle, net.handle, None, None, None,
                                                           None, C.byref(nt)))
        n, N = net.cfg.n, self.ndof
        dev = b.device if b is not None else x.device
        f = torch.empty((nt.value, net.cfg.cin, n, n), dtype=torch.float32, device=dev) if b is not None else None
        t = torch.empty((nt.value, 2, n, n), dtype=torch.float32, device=dev) if x is not None else None
        _check(self.ctx.handle, self._lib.stf_nn_tile_data(
            self.handle, net.handle, _cptr(b, N, "b") if b is not None else None,
            _cptr(x, N, "x") if x is not None else None,
            C.c_void_p(f.data_ptr()) if f is not None else None,
            C.c_void_p(t.data_ptr()) if t is not None else None, C.byref(nt)))
        return f, t

    def initial_guess(self, net, b):
        """The network's blended initial guess for source b (same kind of array as b)."""
        n = self.ndof
        pb_, dev, kb = _ptr(b, n, "b")
        x = self._out_like(b, (self.ny, self.nx))
        px, dev2, kx = _ptr(x, n, "x0")
        _check(self.ctx.handle, self._lib.stf_nn_initial_guess(self.handle, net.handle, pb_, px, dev))
        return x if dev else kx.reshape(self.ny, self.nx)


def _order(order):
    if isinstance(order, str):
        if order not in _abi.ORDERS:
            raise ValueError("order must be one of %s" % list(_abi.ORDERS))
        return _abi.ORDERS[order]
    return int(order)


def batch_solve(ctx, problems, bs, xs=None, tol=1e-10, restart=10, max_iter=500, x0=None,
                history_cap=1024, raise_on_noconv=False, order="additive"):
    """Factor the problems together and solve all their right-hand sides in one
    lockstep batched FGMRES (stf_batch_solve).  bs[p]: (nrhs_p, ny, nx) or (ny, nx),
    all NumPy (host) or all complex128 CUDA tensors (device).  x0: None (zero),
    "learned", or a list of guesses shaped like bs.  Returns (xs, infos) with
    infos[p] a list of per-right-hand-side dicts as Problem.solve returns."""
    lib = ctx._lib
    n = len(problems)
    if n == 0 or len(bs) != n:
        raise ValueError("one right-hand side array per problem")
    shapes = [tuple(b.shape) for b in bs]
    nr = [1 if len(sh) == 2 else int(sh[0]) for sh in shapes]
    mode = _abi.STF_X0_ZERO
    if isinstance(x0, str):
        if x0 != "learned":
            raise ValueError("x0 must be None, a list of arrays or 'learned'")
        mode = _abi.STF_X0_LEARNED
    elif x0 is not None:
        mode = _abi.STF_X0_USER
        xs = [x.clone() if _is_torch(x) else np.array(x, dtype=np.complex128, copy=True) for x in x0]
    if xs is None:
        xs = [problems[p]._out_like(bs[p], shapes[p]) for p in range(n)]
    keep, bptr, xptr, dev = [], (C.c_void_p * n)(), (C.c_void_p * n)(), None
    for p in range(n):
        cnt = nr[p] * problems[p].ndof
        pb_, d1, kb = _ptr(bs[p], cnt, "b[%d]" % p)
        px_, d2, kx = _ptr(xs[p], cnt, "x[%d]" % p)
        if dev is None:
            dev = d1
        if d1 != dev or d2 != dev:
            raise TypeError("all right-hand sides and solutions must be host, or all device, arrays")
        keep += [kb, kx]
        bptr[p], xptr[p] = pb_.value, px_.value
    probs = (C.c_void_p * n)(*[pb.handle.value for pb in problems])
    nrhs = (C.c_int32 * n)(*nr)
    opts = _abi.SolveOpts(float(tol), int(restart), int(max_iter), mode, 1, 0, _order(order))
    infos = [(_abi.SolveInfo * nr[p])() for p in range(n)]
    hist = [[np.zeros(history_cap, dtype=np.float64) for _ in range(nr[p])] for p in range(n)]
    for p in range(n):
        for r in range(nr[p]):
            infos[p][r].history = hist[p][r].ctypes.data_as(C.POINTER(C.c_double))
            infos[p][r].history_cap = history_cap
    iptr = (C.c_void_p * n)(*[C.cast(infos[p], C.c_void_p).value for p in range(n)])
    allow = (_abi.STF_EPIVOT,) if raise_on_noconv else (_abi.STF_ENOCONV, _abi.STF_EPIVOT)
    st = _check(ctx.handle, lib.stf_batch_solve(ctx.handle, n, probs, nrhs, bptr, xptr, dev,
                                                C.byref(opts), iptr), allow=allow)
    out = []
    for p in range(n):
        lst = []
        for r in range(nr[p]):
            inf = infos[p][r]
            lst.append(dict(iters=inf.iters, restarts=inf.restarts, status=inf.status,
                            relres_true=inf.relres_true, relres_x0=inf.relres_x0,
                            used_learned=inf.used_learned, epivot=st == _abi.STF_EPIVOT,
                            t_factor_ms=inf.t_factor_ms, t_solve_ms=inf.t_solve_ms,
                            t_nn_ms=inf.t_nn_ms, history=hist[p][r][:inf.history_len].copy()))
        out.append(lst)
    res = [xs[p] if dev else keep[2 * p + 1].reshape(shapes[p]) for p in range(n)]
    return res, out


def _cptr(a, count, name):
    """Device pointer of a contiguous complex128 CUDA tensor with `count` entries."""
    import torch
    if not (_is_torch(a) and a.is_cuda and a.dtype == torch.complex128 and a.is_contiguous()):
        raise TypeError("%s must be a contiguous complex128 CUDA tensor" % name)
    if a.numel() != count:
        raise ValueError("%s has %d entries, expected %d" % (name, a.numel(), count))
    return C.c_void_p(a.data_ptr())


def _nn_config(n, width, modes, layers, cin=3, max_batch=16):
    c = _abi.NNConfig()
    c.n, c.width, c.modes, c.layers, c.cin, c.max_batch = (int(n), int(width), int(modes),
                                                            int(layers), int(cin), int(max_batch))
    return c


def nn_param_count(n, width, modes, layers, cin=3):
    return int(_abi.load().stf_nn_param_count(C.byref(_nn_config(n, width, modes, layers, cin))))


def _fptr(a, count, name):
    """Device pointer of a contiguous float32 CUDA tensor with `count` entries."""
    import torch
    if not (_is_torch(a) and a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()):
        raise TypeError("%s must be a contiguous float32 CUDA tensor" % name)
    if a.numel() != count:
        raise ValueError("%s has %d entries, expected %d" % (name, a.numel(), count))
    return C.c_void_p(a.data_ptr())


class Network:
    """The learned warm start's spectral neural operator (see include/stfdfd.h).
    params: flat float64/float32 host array in the documented layout."""

    def __init__(self, ctx, params, n=256, width=16, modes=16, layers=4, cin=3, max_batch=16):
        self.ctx = ctx
        self._lib = ctx._lib
        self.cfg = _nn_config(n, width, modes, layers, cin, max_batch)
        self.nparams = int(self._lib.stf_nn_param_count(C.byref(self.cfg)))
        if self.nparams < 0:
            raise StfError(_abi.STF_EINVAL, "invalid network configuration")
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.nparams:
            raise ValueError("params has %d entries, expected %d" % (p.size, self.nparams))
        h = C.c_void_p()
        _check(ctx.handle, self._lib.stf_nn_create(ctx.handle, C.byref(self.cfg),
                                                   C.c_void_p(p.ctypes.data), C.byref(h)))
        self.handle = h
        ctx._networks.add(self)

    def close(self):
        if getattr(self, "handle", None) and getattr(self.ctx, "handle", None):
            self._lib.stf_nn_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _per(self, ch):
        return ch * self.cfg.n * self.cfg.n

    def get_params(self):
        out = np.empty(self.nparams, dtype=np.float32)
        _check(self.ctx.handle, self._lib.stf_nn_get_params(self.handle, C.c_void_p(out.ctypes.data)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.nparams:
            raise ValueError("params has %d entries, expected %d" % (p.size, self.nparams))
        _check(self.ctx.handle, self._lib.stf_nn_set_params(self.handle, C.c_void_p(p.ctypes.data)))

    def forward(self, f, y=None):
        """f: float32 CUDA tensor (B, cin, n, n) -> y (B, 2, n, n)."""
        import torch
        B = int(f.shape[0])
        if y is None:
            y = torch.empty((B, 2, self.cfg.n, self.cfg.n), dtype=torch.float32, device=f.device)
        _check(self.ctx.handle, self._lib.stf_nn_forward(self.handle, B,
                                                         _fptr(f, B * self._per(self.cfg.cin), "f"),
                                                         _fptr(y, B * self._per(2), "y")))
        return y

    def loss_grad(self, f, t):
        """(loss, gradient as a host float32 array) for one batch."""
        B = int(f.shape[0])
        loss = C.c_double()
        g = np.empty(self.nparams, dtype=np.float32)
        _check(self.ctx.handle, self._lib.stf_nn_loss_grad(
            self.handle, B, _fptr(f, B * self._per(self.cfg.cin), "f"),
            _fptr(t, B * self._per(2), "t"), C.byref(loss), C.c_void_p(g.ctypes.data)))
        return loss.value, g

    def train_step(self, f, t, lr, step):
        B = int(f.shape[0])
        loss = C.c_double()
        _check(self.ctx.handle, self._lib.stf_nn_train_step(
            self.handle, B, _fptr(f, B * self._per(self.cfg.cin), "f"),
            _fptr(t, B * self._per(2), "t"), float(lr), int(step), C.byref(loss)))
        return loss.value
