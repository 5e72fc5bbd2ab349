"""MI355X (gfx950) randomized rank-1 lattice QMC for sector integrals and amplitudes.

Thin ctypes binding of ``libqmcamp.so`` (C ABI in ``include/qmcamp.h``).  This module
only marshals arguments: every step of the integration runs in the library's HIP
kernels.  PyTorch provides device memory (the plan workspace and output tensors) and
the stream.  There is no CPU fallback: importing fails loudly when the library is
missing, and every call requires a HIP device.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import flow  # noqa: F401  (learned flow transform)
from ._abi import (QMC_MAX_DIM, QMC_MAX_LOG, QMC_MAX_ORDERS, QMC_PREC_FP32, QMC_PREC_FP64,
                   QMC_SPEC_COMPILE_ONLY, QMC_SPEC_OFF, QMC_SPEC_PERSISTENT, TRANSFORMS, AmpOptions, AmpStats, Amplitude, LaunchShape, QmcError, lib,
                   options_struct,
                   problem_struct)

QMC_AMP_HOST = 0
QMC_AMP_DEVICE = 1

__all__ = ["Plan", "QmcError", "lib", "korobov_search", "lattice_points", "TRANSFORMS",
           "QMC_PREC_FP64", "QMC_PREC_FP32"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2305_19768_amd needs a HIP device (torch.cuda.is_available() "
                           "is False); the library has no CPU path")
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    st = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(st.cuda_stream)


def _check(rc: int, what: str):
    if rc != 0:
        raise QmcError(rc, f"{what}: {lib().qmc_last_error().decode(errors='replace')}")


class Plan:
    """A packed problem bound to a device workspace.

    ``problem`` is a ``workloads.Problem``-like object (sectors with monomial tables,
    exponents, log coefficients, lattice size n and Korobov parameter a).
    """

    def __init__(self, problem, m: Optional[int] = None, precision: int = QMC_PREC_FP64,
                 seed: int = 0, n_max: int = 0, block: int = 0, shift_tile: int = 0,
                 shifts_per_pass: int = 0, use_problem_shifts: bool = True, device=None,
                 bind_workspace: bool = True):
        torch = _torch()
        self.problem = problem
        self.m = int(problem.m if m is None else m)
        self.S = len(problem.sectors)
        self.K = problem.K
        self._keep, prob = problem_struct(problem)
        opt = options_struct(self.m, precision, seed, n_max, block, shift_tile, shifts_per_pass)
        h = ctypes.c_void_p()
        _check(lib().qmc_plan(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h)), "qmc_plan")
        self._h = h
        self.complex = bool(lib().qmc_plan_complex(h))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.workspace = None
        if bind_workspace:   # without one, only integrate_static runs (static device scratch)
            nbytes = int(lib().qmc_workspace_bytes(h))
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _check(lib().qmc_bind_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()),
                                            ctypes.c_size_t(nbytes), _stream_ptr()),
                   "qmc_bind_workspace")
        if use_problem_shifts and getattr(problem, "shifts", None) is not None:
            self.set_shifts(problem.shifts)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().qmc_plan_free(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def set_shifts(self, shifts: Sequence[np.ndarray]):
        arr = np.zeros((self.S, self.m, QMC_MAX_DIM), dtype=np.float64)
        for s, sh in enumerate(shifts):
            sh = np.asarray(sh, dtype=np.float64)
            arr[s, :, :sh.shape[1]] = sh[:self.m]
        _check(lib().qmc_set_shifts(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _stream_ptr()), "qmc_set_shifts")
        self._shift_host = arr   # keep alive until the copy is issued

    def integrate(self, n: Optional[Sequence[int]] = None, a: Optional[Sequence[int]] = None,
                  out=None, stream=None, check: bool = True, z=None):
        """Runs the lattice rule on every sector.  Returns (q [S, m, K], mean [S, K],
        err [S, K]) as float64 device tensors; a complex plan appends a (re, im) axis of
        length 2 to each.  With check=True the stream is synchronised and a non-finite sum
        (or, in a complex plan, a sign-check violation) raises QmcError."""
        torch = _torch()
        tail = (2,) if self.complex else ()
        if out is None:
            q = torch.empty((self.S, self.m, self.K) + tail, dtype=torch.float64,
                            device=self.device)
            mean = torch.empty((self.S, self.K) + tail, dtype=torch.float64, device=self.device)
            err = torch.empty((self.S, self.K) + tail, dtype=torch.float64, device=self.device)
        else:
            q, mean, err = out
        n_arr = None if n is None else np.ascontiguousarray(n, dtype=np.uint64)
        a_arr = None if a is None else np.ascontiguousarray(a, dtype=np.uint64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.c_void_p
        st = _stream_ptr(stream)
        if z is not None:   # general generating vectors [S][QMC_MAX_DIM]
            z_arr = np.ascontiguousarray(z, dtype=np.uint64).reshape(self.S, QMC_MAX_DIM)
            _check(lib().qmc_integrate_vec(self._h,
                                           None if n_arr is None else n_arr.ctypes.data_as(u64p),
                                           z_arr.ctypes.data_as(u64p), st,
                                           dp(q.data_ptr()) if q is not None else None,
                                           dp(mean.data_ptr()), dp(err.data_ptr())),
                   "qmc_integrate_vec")
        else:
            _check(lib().qmc_integrate(self._h,
                                       None if n_arr is None else n_arr.ctypes.data_as(u64p),
                                       None if a_arr is None else a_arr.ctypes.data_as(u64p), st,
                                       dp(q.data_ptr()) if q is not None else None,
                                       dp(mean.data_ptr()), dp(err.data_ptr())), "qmc_integrate")
        if check:
            self.check_status(stream)
        return q, mean, err

    def integrate_static(self, n: Optional[Sequence[int]] = None,
                         a: Optional[Sequence[int]] = None, out=None, stream=None,
                         check: bool = True):
        """integrate() through qmc_integrate_static: the call's device state lives in the
        library's static scratch, so it needs no workspace.  Same outputs."""
        torch = _torch()
        tail = (2,) if self.complex else ()
        if out is None:
            q = torch.empty((self.S, self.m, self.K) + tail, dtype=torch.float64,
                            device=self.device)
            mean = torch.empty((self.S, self.K) + tail, dtype=torch.float64, device=self.device)
            err = torch.empty((self.S, self.K) + tail, dtype=torch.float64, device=self.device)
        else:
            q, mean, err = out
        n_arr = None if n is None else np.ascontiguousarray(n, dtype=np.uint64)
        a_arr = None if a is None else np.ascontiguousarray(a, dtype=np.uint64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.c_void_p
        _check(lib().qmc_integrate_static(self._h,
                                          None if n_arr is None else n_arr.ctypes.data_as(u64p),
                                          None if a_arr is None else a_arr.ctypes.data_as(u64p),
                                          _stream_ptr(stream),
                                          dp(q.data_ptr()) if q is not None else None,
                                          dp(mean.data_ptr()), dp(err.data_ptr())),
               "qmc_integrate_static")
        if check:
            self.check_status(stream)
        return q, mean, err

    def flow_samples(self, sector: int, n: int, a: int, shift: int = 0, stream=None):
        """Training samples of a sector for a flow transform: (x [n, d], w [n]) device
        float64 tensors (see qmc_flow_samples)."""
        torch = _torch()
        d = int(self.problem.sectors[sector].d)
        x = torch.empty((int(n), d), dtype=torch.float64, device=self.device)
        w = torch.empty(int(n), dtype=torch.float64, device=self.device)
        _check(lib().qmc_flow_samples(self._h, int(sector), ctypes.c_uint64(int(n)),
                                      ctypes.c_uint64(int(a)), int(shift), _stream_ptr(stream),
                                      ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr())),
               "qmc_flow_samples")
        return x, w

    def attach_flow(self, sector: int, flow, cond=None, stream=None):
        """Integrate `sector` through `flow` (a paper_2305_19768_amd.flow.Flow; for a
        conditional flow, cond holds the sector's n_cond conditioning features), or detach
        with None.  The plan keeps a reference to the flow while attached."""
        if not hasattr(self, "_flows"):
            self._flows = {}
        ptr = None if flow is None else ctypes.c_void_p(flow.ptr)
        nc = 0 if flow is None else flow.n_cond
        cv = np.ascontiguousarray([] if cond is None else cond, dtype=np.float64).reshape(-1)
        if flow is not None and cv.size != nc:
            raise ValueError(f"flow takes {nc} conditioning features, got {cv.size}")
        _check(lib().qmc_flow_attach(self._h, int(sector), ptr, nc,
                                     cv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                     if nc else None, _stream_ptr(stream)),
               "qmc_flow_attach")
        if flow is None:
            self._flows.pop(int(sector), None)
        else:
            self._flows[int(sector)] = flow

    def median_lattice(self, r: int = 11, n=None, candidates=None, seed: int = 0,
                       order: int = -1, stream=None):
        """Median QMC rule per sector (see qmc_median_lattice).  candidates: [S][r][d or 8]
        generating vectors; None draws them (seeded) uniformly from U_n.  Returns
        (z [S][QMC_MAX_DIM], estimates [S][r], candidates [S][r][QMC_MAX_DIM])."""
        import math
        torch = _torch()
        ns = [int(x) for x in (n if n is not None else [s.n for s in self.problem.sectors])]
        c = np.zeros((self.S, r, QMC_MAX_DIM), dtype=np.uint64)
        if candidates is None:
            rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 23])))
            for s, sec in enumerate(self.problem.sectors):
                for k in range(r):
                    for j in range(sec.d):
                        while True:
                            v = int(rng.integers(1, ns[s]))
                            if math.gcd(v, ns[s]) == 1:
                                c[s, k, j] = v
                                break
        else:
            cc = np.asarray(candidates, dtype=np.uint64)
            c[:, :, :cc.shape[2]] = cc
        nb = int(lib().qmc_median_workspace_bytes(self._h, r))
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        ptr = scratch.data_ptr() + (-scratch.data_ptr()) % 256
        n_arr = np.ascontiguousarray(ns, dtype=np.uint64)
        z = np.zeros((self.S, QMC_MAX_DIM), dtype=np.uint64)
        q = np.zeros((self.S, r))
        u64p = ctypes.POINTER(ctypes.c_uint64)
        _check(lib().qmc_median_lattice(self._h, n_arr.ctypes.data_as(u64p), int(r),
                                        c.ctypes.data_as(u64p), int(order), ctypes.c_void_p(ptr),
                                        ctypes.c_size_t(nb), _stream_ptr(stream),
                                        z.ctypes.data_as(u64p),
                                        q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "qmc_median_lattice")
        return z, q, c

    def launch_shape(self) -> dict:
        sh = LaunchShape()
        _check(lib().qmc_get_launch_shape(self._h, ctypes.byref(sh)), "qmc_get_launch_shape")
        return {f: getattr(sh, f) for f, _ in LaunchShape._fields_}

    def set_launch_shape(self, block: int, shift_tile: int, shifts_per_pass: int,
                         target_blocks: int = 16384):
        sh = LaunchShape(block, shift_tile, shifts_per_pass, target_blocks, 0.0)
        _check(lib().qmc_set_launch_shape(self._h, ctypes.byref(sh)), "qmc_set_launch_shape")

    def specialize(self, off: bool = False, persistent: bool = False) -> float:
        """Compiles and loads plan-specialised integrand kernels for the launch classes of
        the real-contour sectors without a flow (see qmc_specialize); persistent=True
        compiles the batched amplitude form's persistent kernel instead; off=True unloads
        them.  Returns the seconds taken."""
        sec = ctypes.c_double()
        flags = QMC_SPEC_OFF if off else (QMC_SPEC_PERSISTENT if persistent else 0)
        _check(lib().qmc_specialize(self._h, flags, ctypes.byref(sec)), "qmc_specialize")
        return sec.value

    def gen_source(self, d: int, f32: bool = False) -> str:
        """Generated source of launch class (d, f32) as qmc_specialize would compile it."""
        return gen_source(self._h, d, f32)

    def autotune(self, n=None, a=None, reps: int = 3, use_cache: bool = True, stream=None) -> dict:
        """Times the launch shapes of the integrand kernels on lattices n, a and keeps the
        fastest (see qmc_autotune); returns it with its time in ms."""
        n_arr = None if n is None else np.ascontiguousarray(n, dtype=np.uint64)
        a_arr = None if a is None else np.ascontiguousarray(a, dtype=np.uint64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        sh = LaunchShape()
        _check(lib().qmc_autotune(self._h, None if n_arr is None else n_arr.ctypes.data_as(u64p),
                                  None if a_arr is None else a_arr.ctypes.data_as(u64p),
                                  int(reps), 1 if use_cache else 0, _stream_ptr(stream),
                                  ctypes.byref(sh)), "qmc_autotune")
        return {f: getattr(sh, f) for f, _ in LaunchShape._fields_}

    def sign_violations(self, stream=None) -> np.ndarray:
        """Per-sector sign-check violation counts of the last integrate() (complex plans)."""
        out = np.zeros(self.S, dtype=np.uint64)
        _check(lib().qmc_sign_violations(self._h, _stream_ptr(stream),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
               "qmc_sign_violations")
        return out

    def set_deformation(self, lam, stream=None):
        arr = np.ascontiguousarray(lam, dtype=np.float64)
        _check(lib().qmc_set_deformation(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         _stream_ptr(stream)), "qmc_set_deformation")
        torch = _torch()
        torch.cuda.current_stream().synchronize()

    def choose_deformation(self, n_pre: int, a_pre=None, max_halvings: int = 16, stream=None):
        """Presample choice of the deformation parameters (halve lambda while a sample
        violates the sign check).  Returns (lambda [S], halvings [S], status) with status
        0 or QMC_E_SIGNCHECK (-6) if some sector could not be fixed."""
        lam = np.zeros(self.S, dtype=np.float64)
        halv = np.zeros(self.S, dtype=np.int32)
        a_arr = None if a_pre is None else np.ascontiguousarray(a_pre, dtype=np.uint64)
        rc = lib().qmc_choose_deformation(
            self._h, ctypes.c_uint64(int(n_pre)),
            None if a_arr is None else a_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            ctypes.c_int32(max_halvings), _stream_ptr(stream),
            lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            halv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if rc not in (0, -6):
            _check(rc, "qmc_choose_deformation")
        return lam, halv, rc

    def integrate_deformed(self, n: Optional[Sequence[int]] = None,
                           a: Optional[Sequence[int]] = None, max_halvings: int = 16, out=None,
                           stream=None):
        """integrate() of a complex plan with the sign-check fallback (qmc_integrate_deformed):
        sectors with a violating sample are re-integrated with lambda halved.  Returns
        (q, mean, err, lambda [S], halvings [S], status) with status 0 or QMC_E_SIGNCHECK
        (-6) if some sector could not be fixed (its results are still written)."""
        torch = _torch()
        if out is None:
            q = torch.empty((self.S, self.m, self.K, 2), dtype=torch.float64, device=self.device)
            mean = torch.empty((self.S, self.K, 2), dtype=torch.float64, device=self.device)
            err = torch.empty((self.S, self.K, 2), dtype=torch.float64, device=self.device)
        else:
            q, mean, err = out
        n_arr = None if n is None else np.ascontiguousarray(n, dtype=np.uint64)
        a_arr = None if a is None else np.ascontiguousarray(a, dtype=np.uint64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.c_void_p
        lam = np.zeros(self.S, dtype=np.float64)
        halv = np.zeros(self.S, dtype=np.int32)
        rc = lib().qmc_integrate_deformed(
            self._h, None if n_arr is None else n_arr.ctypes.data_as(u64p),
            None if a_arr is None else a_arr.ctypes.data_as(u64p), ctypes.c_int32(max_halvings),
            _stream_ptr(stream), dp(q.data_ptr()) if q is not None else None,
            dp(mean.data_ptr()), dp(err.data_ptr()),
            lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            halv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if rc not in (0, -6):
            _check(rc, "qmc_integrate_deformed")
        return q, mean, err, lam, halv, rc

    def check_status(self, stream=None):
        sec, sh, order = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qmc_query_status(self._h, _stream_ptr(stream), ctypes.byref(sec),
                                      ctypes.byref(sh), ctypes.byref(order)), "qmc_query_status")

    def enable_timing(self, on: bool = True):
        """Record HIP events around the integrand kernel of each integrate() call."""
        _check(lib().qmc_enable_timing(self._h, ctypes.c_int32(1 if on else 0)),
               "qmc_enable_timing")

    def read_timing(self):
        """(summed kernel milliseconds, number of timed launches) since enable_timing."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int32()
        _check(lib().qmc_read_timing(self._h, ctypes.byref(ms), ctypes.byref(cnt)),
               "qmc_read_timing")
        return float(ms.value), int(cnt.value)

    def korobov_p2(self, n: int, d: int, candidates: Sequence[int], stream=None):
        """P_2 figure of merit of the Korobov vectors (1, a, ..., a^(d-1)) mod n (device)."""
        torch = _torch()
        c = np.ascontiguousarray(candidates, dtype=np.uint64)
        out = torch.empty(len(c), dtype=torch.float64, device=self.device)
        _check(lib().qmc_korobov_p2(self._h, ctypes.c_uint64(n), ctypes.c_int32(d),
                                    c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    ctypes.c_int32(len(c)), _stream_ptr(stream),
                                    ctypes.c_void_p(out.data_ptr())), "qmc_korobov_p2")
        return out

    def korobov_search(self, n: int, d: int, candidates: Sequence[int], stream=None):
        """Korobov parameter minimising P_2 over the candidates (ties: smallest a)."""
        c = np.ascontiguousarray(candidates, dtype=np.uint64)
        a = ctypes.c_uint64()
        p2 = ctypes.c_double()
        _check(lib().qmc_korobov_search(self._h, ctypes.c_uint64(n), ctypes.c_int32(d),
                                        c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                        ctypes.c_int32(len(c)), _stream_ptr(stream),
                                        ctypes.byref(a), ctypes.byref(p2)), "qmc_korobov_search")
        return int(a.value), float(p2.value)


    def lattice_table(self, sizes, candidates, dims=None):
        """Korobov parameter per (size, dimension): the P_2-minimising candidate, chosen on
        the device.  candidates: [L, QMC_MAX_DIM, R] (row d-1 for dimension d).  Returns
        uint64 [L, QMC_MAX_DIM]; dimensions not in `dims` (default: the plan's) get 1."""
        sizes = np.asarray(sizes, dtype=np.uint64)
        cands = np.asarray(candidates, dtype=np.uint64)
        dims = sorted({s.d for s in self.problem.sectors}) if dims is None else sorted(dims)
        out = np.ones((len(sizes), QMC_MAX_DIM), dtype=np.uint64)
        for l, n in enumerate(sizes):
            for d in dims:
                out[l, d - 1] = self.korobov_search(int(n), d, [int(c) for c in cands[l, d - 1]])[0]
        return out

    def amp_evaluate(self, coef, epsrel: float, epsabs: float = 0.0, lattice_n=None,
                     lattice_a=None, tau=None, alpha: float = 2.0, n_presample: int = 10000,
                     max_rounds: int = 50, timeout_s: float = 0.0, mode: int = QMC_AMP_HOST,
                     stream=None, coef_order_lo: int = 0, return_tau: bool = False):
        """Adaptive evaluation of weighted sums A_t = sum_i C_ti I_i (see amp_evaluate in
        include/qmcamp.h).  coef: complex [n_sums, n_integrals] (or [n_integrals] for one
        sum), or [n_sums, n_integrals, P] Laurent terms of eps^(coef_order_lo + p).
        Returns (value complex [n_sums, K], error complex [n_sums, K] as
        (err_re + 1j err_im), n_final [S], stats dict); order j of the values is
        eps^(order_lo + coef_order_lo + j).  tau=None measures the costs while the
        evaluation runs; return_tau=True adds stats["tau_used"] [allocations, S], the
        costs each allocation used."""
        C = np.asarray(coef, dtype=np.complex128)
        if C.ndim == 1:
            C = C[None, :]
        if C.ndim == 2:
            C = C[:, :, None]
        T, NI, P = C.shape
        rows, cols, cre, cim = [0], [], [], []
        for t in range(T):
            nz = np.nonzero(np.any(C[t] != 0, axis=1))[0]
            cols.extend(int(i) for i in nz)
            for i in nz:
                cre.extend(float(v) for v in C[t, i].real)
                cim.extend(float(v) for v in C[t, i].imag)
            rows.append(len(cols))
        row_ptr = np.array(rows, dtype=np.int64)
        col = np.array(cols, dtype=np.int32)
        cr = np.array(cre, dtype=np.float64)
        ci = np.array(cim, dtype=np.float64)
        A = Amplitude()
        A.n_sums = T
        A.n_terms = P
        A.coef_order_lo = int(coef_order_lo)
        A.row_ptr = row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        A.col = col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        A.coef_re = cr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        A.coef_im = ci.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ln = np.ascontiguousarray(lattice_n, dtype=np.uint64)
        la = np.ascontiguousarray(lattice_a, dtype=np.uint64).reshape(len(ln), QMC_MAX_DIM)
        O = AmpOptions()
        O.epsrel, O.epsabs, O.timeout_s, O.alpha = epsrel, epsabs, timeout_s, alpha
        O.n_presample, O.max_rounds, O.mode, O.n_lattice = n_presample, max_rounds, mode, len(ln)
        O.lattice_n = ln.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        O.lattice_a = la.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        tau_arr = None
        if tau is not None:
            tau_arr = np.ascontiguousarray(tau, dtype=np.float64)
            O.tau = tau_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        tau_used = None
        if return_tau:
            tau_used = np.full((max_rounds, self.S), np.nan)
            O.tau_used = tau_used.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        val = np.zeros((T, self.K, 2))
        err = np.zeros((T, self.K, 2))
        nfin = np.zeros(self.S, dtype=np.uint64)
        st = AmpStats()
        rc = lib().amp_evaluate(self._h, ctypes.byref(A), ctypes.byref(O), _stream_ptr(stream),
                                val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                err.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                nfin.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                ctypes.byref(st))
        if rc not in (0, -5):
            _check(rc, "amp_evaluate")
        stats = {f: getattr(st, f) for f, _ in AmpStats._fields_}
        stats["status"] = rc
        if tau_used is not None:   # the rows the allocations wrote
            rows = 0
            while rows < len(tau_used) and not np.isnan(tau_used[rows]).any():
                rows += 1
            stats["tau_used"] = tau_used[:rows].copy()
        return (val[..., 0] + 1j * val[..., 1], err[..., 0] + 1j * err[..., 1], nfin, stats)

    def amp_evaluate_expressions(self, sums, symbols=None, regulator: str = "eps", **kw):
        """Named weighted sums with coefficients given as expressions (Sec. 2.4).
        sums: {name: row} (or a list of rows, named 0, 1, ...); a row is a list with one
        entry per integral or a dict {integral index: entry}; entries are expression
        strings or numbers, "0" or 0 for absent integrals.  The coefficients are expanded
        exactly in the regulator (qmc_coef_series) from the lowest leading order of all
        entries over the plan's K orders, then evaluated by amp_evaluate (keyword
        arguments passed on).  Returns ({name: {"orders": [eps powers], "value": complex
        [K], "error": complex [K]}}, n_final, stats)."""
        named = dict(sums) if isinstance(sums, dict) else dict(enumerate(sums))
        NI = self.problem.n_integrals
        rows = {}
        for name, row in named.items():
            items = row.items() if isinstance(row, dict) else enumerate(row)
            ent = {}
            for i, e in items:
                if not 0 <= int(i) < NI:
                    raise ValueError(f"sum {name!r}: integral {i} outside [0, {NI})")
                e = e if isinstance(e, str) else repr(e)
                lead, _ = coef_series(e, regulator, symbols, 0, 0)
                if lead is not None:
                    ent[int(i)] = (e, lead)
            rows[name] = ent
        leads = [lead for ent in rows.values() for _, lead in ent.values()]
        lo = min(leads) if leads else 0
        C = np.zeros((len(rows), NI, self.K), dtype=np.complex128)
        for t, ent in enumerate(rows.values()):
            for i, (e, _) in ent.items():
                C[t, i] = coef_series(e, regulator, symbols, lo, self.K)[1]
        val, err, nfin, stats = self.amp_evaluate(C, coef_order_lo=lo, **kw)
        orders = [self.problem.order_lo + lo + j for j in range(self.K)]
        out = {name: {"orders": orders, "value": val[t], "error": err[t]}
               for t, name in enumerate(rows)}
        return out, nfin, stats


def coef_series(expr: str, regulator: str = "eps", symbols=None, order_lo: int = 0,
                n_terms: int = 1):
    """Laurent series of a coefficient expression in the regulator, evaluated exactly
    with the symbol values `symbols` ({name: value expression or number}) and rounded
    to doubles (qmc_coef_series).  Returns (leading order or None for an identically zero
    expression, complex coefficients [n_terms] of regulator^(order_lo + j))."""
    names = list((symbols or {}).keys())
    vals = [str(v) if not isinstance(v, str) else v for v in (symbols or {}).values()]
    cn = (ctypes.c_char_p * max(1, len(names)))(*[n.encode() for n in names])
    cv = (ctypes.c_char_p * max(1, len(vals)))(*[v.encode() for v in vals])
    re = np.zeros(max(1, n_terms))
    im = np.zeros(max(1, n_terms))
    lead = ctypes.c_int32(0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().qmc_coef_series(expr.encode(), regulator.encode(), len(names), cn, cv,
                                 int(order_lo), int(n_terms), ctypes.byref(lead),
                                 re.ctypes.data_as(dp), im.ctypes.data_as(dp)),
           "qmc_coef_series")
    lo = None if lead.value == 2 ** 31 - 1 else int(lead.value)
    return lo, (re + 1j * im)[:n_terms]


def host_plan(problem, m: Optional[int] = None, precision: int = QMC_PREC_FP64, seed: int = 0,
              shifts_per_pass: int = 0):
    """A plan handle without a workspace (host-only calls such as qmc_gen_source and
    qmc_specialize(QMC_SPEC_COMPILE_ONLY)); free with lib().qmc_plan_free."""
    keep, prob = problem_struct(problem)
    opt = options_struct(problem.m if m is None else m, precision, seed, 0, 0, 0, shifts_per_pass)
    h = ctypes.c_void_p()
    _check(lib().qmc_plan(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h)), "qmc_plan")
    return h


def gen_source(handle, d: int, f32: bool = False) -> str:
    """Generated source of launch class (d, f32) of a plan (see qmc_gen_source)."""
    n = ctypes.c_size_t()
    _check(lib().qmc_gen_source(handle, int(d), 1 if f32 else 0, None, 0, ctypes.byref(n)),
           "qmc_gen_source")
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().qmc_gen_source(handle, int(d), 1 if f32 else 0, buf, n.value + 1, None),
           "qmc_gen_source")
    return buf.value.decode()


def specialize_compile_only(handle) -> float:
    """qmc_specialize(QMC_SPEC_COMPILE_ONLY): generates and compiles every class kernel of
    a plan without loading it (no GPU needed); returns the seconds taken."""
    sec = ctypes.c_double()
    _check(lib().qmc_specialize(handle, QMC_SPEC_COMPILE_ONLY, ctypes.byref(sec)), "qmc_specialize")
    return sec.value


def korobov_search(plan: Plan, n: int, d: int, candidates: Sequence[int]):
    return plan.korobov_search(n, d, candidates)


def lattice_points(n: int, a: int, shift: Sequence[float], i0: int = 0,
                   count: Optional[int] = None, stream=None):
    """Shifted rank-1 lattice points computed on the device, float64 [count, d]."""
    torch = _torch()
    sh = np.ascontiguousarray(shift, dtype=np.float64)
    d = len(sh)
    count = n - i0 if count is None else count
    out = torch.empty((count, d), dtype=torch.float64, device="cuda")
    _check(lib().qmc_lattice_points(ctypes.c_uint64(n), ctypes.c_int32(d), ctypes.c_uint64(a),
                                    sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.c_uint64(i0), ctypes.c_uint64(count),
                                    _stream_ptr(stream), ctypes.c_void_p(out.data_ptr())),
           "qmc_lattice_points")
    return out
