"""Python binding of libdgsn: argument marshalling only.

Every step of the transport path runs in the HIP library; torch tensors are
used for device memory and the current HIP stream.  Array layouts follow
include/dgsn.h: per-cell fields [G][nz][ny][nx], nodal fields
[G][nz][ny][nx][8] (node n = ix + 2 iy + 4 iz fastest).
"""
import ctypes
import warnings

import numpy as np
import torch

from . import _lib
from ._lib import DgsnError, ProblemDesc  # noqa: F401

FP32 = _lib.DGSN_FP32
FP64 = _lib.DGSN_FP64
GE = _lib.DGSN_GE
ANN = _lib.DGSN_ANN
GE_DENSE = _lib.DGSN_GE_DENSE

_PREC = {"fp32": FP32, "fp64": FP64, FP32: FP32, FP64: FP64}
_SOLVER = {"ge": GE, "ann": ANN, "ge_dense": GE_DENSE, GE: GE, ANN: ANN, GE_DENSE: GE_DENSE}
_DTYPE = {FP32: torch.float32, FP64: torch.float64}


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def version():
    return _lib.load().dgsn_version()


def quadrature_ls(order):
    """Level-symmetric LQ_N set from the library: (omega [D,3], weight [D])."""
    lib = _lib.load()
    n = ctypes.c_int(0)
    _lib.check(lib.dgsn_quadrature_ls(int(order), None, None, ctypes.byref(n)))
    om = np.zeros((n.value, 3))
    w = np.zeros(n.value)
    _lib.check(lib.dgsn_quadrature_ls(int(order), om.ctypes.data_as(_lib._PD),
                                      w.ctypes.data_as(_lib._PD), ctypes.byref(n)))
    return om, w


def _desc(n, length, groups, omega, weight, precision, solver, store_psi):
    omega = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(-1, 3))
    weight = np.ascontiguousarray(np.asarray(weight, np.float64).reshape(-1))
    d = ProblemDesc(int(n[0]), int(n[1]), int(n[2]), float(length[0]), float(length[1]),
                    float(length[2]), int(groups), int(omega.shape[0]),
                    omega.ctypes.data_as(_lib._PD), weight.ctypes.data_as(_lib._PD),
                    _PREC[precision], _SOLVER[solver], int(bool(store_psi)))
    return d, (omega, weight)   # keep the arrays alive with the descriptor


def validate(n, length, groups, omega, weight, precision="fp32", solver="ge", store_psi=False):
    """Host-side descriptor validation (no device needed)."""
    d, keep = _desc(n, length, groups, omega, weight, precision, solver, store_psi)
    _lib.check(_lib.load().dgsn_problem_validate(ctypes.byref(d)))


class Context:
    def __init__(self, device=0):
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().dgsn_ctx_create(int(device), ctypes.byref(self._h)))
        self.device = torch.device("cuda", int(device))

    def close(self):
        if self._h:
            _lib.load().dgsn_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ann:
    """A loaded shallow-ANN artifact (device-resident operand images)."""

    def __init__(self, ctx, path):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().dgsn_ann_load(ctx._h, str(path).encode(), ctypes.byref(self._h)))

    def info(self):
        """(version, n_in, n_hidden, n_nets) of the artifact."""
        v = [ctypes.c_int() for _ in range(4)]
        _lib.check(_lib.load().dgsn_ann_info(self._h, *[ctypes.byref(a) for a in v]))
        return tuple(a.value for a in v)

    @property
    def version(self):
        return self.info()[0]

    def set_mode(self, mode):
        """'bf16' (default) or 'bf16x2' (split-BF16 activations) for the
        matrix-core network."""
        m = {"bf16": _lib.DGSN_ANN_BF16, "bf16x2": _lib.DGSN_ANN_BF16X2}[mode]
        _lib.check(_lib.load().dgsn_ann_set_mode(self._h, m))

    def infer_octant(self, octant, x, out=None):
        """Paper-form network `octant` on raw inputs x [n,26] float32 -> [n,8]
        (per-direction artifacts: the index of the direction's network)."""
        x = x.contiguous()
        if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != 26:
            raise ValueError("x must be a float32 [n, 26] tensor")
        y = out if out is not None else torch.empty((x.shape[0], 8), dtype=torch.float32,
                                                    device=x.device)
        _lib.check(_lib.load().dgsn_ann_infer_octant(self._h, int(octant), _ptr(x), _ptr(y),
                                                     x.shape[0], _stream(x.device)))
        return y

    def infer(self, x, out=None):
        """y = W2 relu(W1 x + b1) + b2 on the BF16 matrix cores; x [n,24] float32."""
        x = x.contiguous()
        if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != 24:
            raise ValueError("x must be a float32 [n, 24] tensor")
        y = out if out is not None else torch.empty((x.shape[0], 8), dtype=torch.float32,
                                                    device=x.device)
        _lib.check(_lib.load().dgsn_ann_infer(self._h, _ptr(x), _ptr(y), x.shape[0],
                                              _stream(x.device)))
        return y

    def close(self):
        if self._h:
            _lib.load().dgsn_ann_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def local_solve(ctx, x):
    """Batched canonical one-cell GE; x [n,24] (float32 or float64) -> psi [n,8]."""
    x = x.contiguous()
    prec = FP64 if x.dtype == torch.float64 else FP32
    if x.dtype not in (torch.float32, torch.float64) or x.dim() != 2 or x.shape[1] != 24:
        raise ValueError("x must be a float32/float64 [n, 24] tensor")
    y = torch.empty((x.shape[0], 8), dtype=x.dtype, device=x.device)
    _lib.check(_lib.load().dgsn_local_solve(ctx._h, _ptr(x), _ptr(y), x.shape[0], prec,
                                            _stream(x.device)))
    return y


def real_ylm(order, omega):
    """The library's real orthonormal spherical harmonics [n, (order+1)^2]
    at unit directions omega [n, 3] (host computation)."""
    om = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(-1, 3))
    nm = (order + 1) ** 2
    out = np.zeros((om.shape[0], nm))
    _lib.check(_lib.load().dgsn_real_ylm(int(order), om.ctypes.data_as(_lib._PD), om.shape[0],
                                         out.ctypes.data_as(_lib._PD)))
    return out


def autotune_cache_clear():
    """Forget every autotuner choice of this process."""
    _lib.check(_lib.load().dgsn_autotune_cache_clear())


def autotune_cache_size():
    n = ctypes.c_int(0)
    _lib.check(_lib.load().dgsn_autotune_cache_size(ctypes.byref(n)))
    return n.value


def autotune_cache_save(path):
    """Write the autotuner's choices of this process to path (JSON)."""
    _lib.check(_lib.load().dgsn_autotune_cache_save(str(path).encode()))


def autotune_cache_load(path):
    """Merge choices saved by autotune_cache_save; later Problem.autotune
    calls for those shapes apply them without timing."""
    _lib.check(_lib.load().dgsn_autotune_cache_load(str(path).encode()))


def spectral_radius(resid, tail=0.5):
    """Effective spectral radius of a source iteration from its residual
    history: the geometric mean ratio of successive residuals over the last
    `tail` fraction of the iterations (at least 2 steps), or None when fewer
    than 4 iterations were run or a residual is zero."""
    r = np.asarray(resid, dtype=np.float64)
    n = r.size
    if n < 4:
        return None
    m = min(n - 3, int(n * (1.0 - tail)))
    if r[m] <= 0.0 or r[-1] <= 0.0:
        return None
    return float((r[-1] / r[m]) ** (1.0 / (n - 1 - m)))


class Problem:
    """One DGFEM S_n problem on the GPU (uniform hex mesh, one quadrature)."""

    def __init__(self, ctx, n, length, groups, omega, weight, precision="fp32", solver="ge",
                 store_psi=False):
        self.ctx = ctx
        self.n = tuple(int(v) for v in n)
        self.length = tuple(float(v) for v in length)
        self.groups = int(groups)
        self.precision = _PREC[precision]
        self.dtype = _DTYPE[self.precision]
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        d, keep = _desc(self.n, self.length, groups, omega, weight, precision, solver, store_psi)
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().dgsn_problem_create(ctx._h, ctypes.byref(d), ctypes.byref(self._h)))
        self.n_dirs = int(d.n_dirs)
        self._ann = None

    # -- setup --------------------------------------------------------------
    def _dev(self, a, shape):
        if a is None:
            return None
        t = torch.as_tensor(a).to(device=self.ctx.device, dtype=self.dtype).contiguous()
        return t.reshape(shape)

    def set_materials(self, sigma_t, sigma_s=None, q=None):
        shape = (self.groups, self.ncell)
        st, ss, qq = self._dev(sigma_t, shape), self._dev(sigma_s, shape), self._dev(q, shape)
        _lib.check(_lib.load().dgsn_problem_set_materials(self._h, _ptr(st), _ptr(ss), _ptr(qq),
                                                          _stream(self.ctx.device)))
        torch.cuda.current_stream(self.ctx.device).synchronize()

    def set_scattering(self, sigma_gg):
        """Multigroup isotropic scattering [G, G, ncell] (from g' into g at
        [g', g]); None removes it."""
        if sigma_gg is None:
            _lib.check(_lib.load().dgsn_problem_set_scattering(self._h, None,
                                                               _stream(self.ctx.device)))
            return
        m = self._dev(sigma_gg, (self.groups, self.groups, self.ncell))
        _lib.check(_lib.load().dgsn_problem_set_scattering(self._h, _ptr(m),
                                                           _stream(self.ctx.device)))
        torch.cuda.current_stream(self.ctx.device).synchronize()

    def set_anisotropy(self, sigma_sn):
        """In-group anisotropic scattering: sigma_sn [L, G, ncell], the Legendre
        moments of orders 1..L (L <= 3); None removes them."""
        lib = _lib.load()
        if sigma_sn is None:
            _lib.check(lib.dgsn_problem_set_anisotropy(self._h, 0, None,
                                                       _stream(self.ctx.device)))
            self.pl_order = 0
            return
        size = int(np.prod(tuple(sigma_sn.shape)))
        L = size // (self.groups * self.ncell)
        if L < 1 or L * self.groups * self.ncell != size:
            raise ValueError("sigma_sn must hold [L, G, ncell] values")
        m = self._dev(sigma_sn, (L, self.groups, self.ncell))
        self._set_orders(lib.dgsn_problem_set_anisotropy(self._h, L, _ptr(m),
                                                         _stream(self.ctx.device)), L)

    def _set_orders(self, rc, L):
        # a setter that fails after its argument checks leaves no orders
        if rc in (_lib.DGSN_ENOMEM, _lib.DGSN_EHIP):
            self.pl_order = 0
        _lib.check(rc)
        torch.cuda.current_stream(self.ctx.device).synchronize()
        self.pl_order = L

    def set_anisotropy_gg(self, sigma_sn_gg):
        """Anisotropic scattering with a group-to-group matrix per Legendre
        order: sigma_sn_gg [L+1, G, G, ncell], order 0 first, from g' into g
        at [n, g', g] (1 <= L <= 3).  Clear with set_anisotropy(None)."""
        size = int(np.prod(tuple(sigma_sn_gg.shape)))
        per = self.groups * self.groups * self.ncell
        L = size // per - 1
        if L < 1 or (L + 1) * per != size:
            raise ValueError("sigma_sn_gg must hold [L+1, G, G, ncell] values with L >= 1")
        m = self._dev(sigma_sn_gg, (L + 1, self.groups, self.groups, self.ncell))
        self._set_orders(_lib.load().dgsn_problem_set_anisotropy_gg(self._h, L, _ptr(m),
                                                                    _stream(self.ctx.device)), L)

    def moments(self):
        """Flux moments k = 1 .. (L+1)^2 - 1 of the last source iteration,
        [(L+1)^2 - 1, G, ncell, 8] on the device."""
        nm = (getattr(self, "pl_order", 0) + 1) ** 2
        out = torch.empty((max(nm - 1, 1), self.groups, self.ncell, 8), dtype=self.dtype,
                          device=self.ctx.device)
        _lib.check(_lib.load().dgsn_problem_get_moments(self._h, _ptr(out),
                                                        _stream(self.ctx.device)))
        return out

    def set_inflow(self, psi_inc):
        arr = np.ascontiguousarray(np.asarray(psi_inc, np.float64).reshape(6))
        _lib.check(_lib.load().dgsn_problem_set_inflow(self._h, arr.ctypes.data_as(_lib._PD)))

    def set_ann(self, ann):
        self._ann = ann
        _lib.check(_lib.load().dgsn_problem_set_ann(self._h, ann._h if ann else None))

    def set_solver(self, solver):
        _lib.check(_lib.load().dgsn_problem_set_solver(self._h, _SOLVER[solver]))

    def stats(self):
        s = ctypes.c_longlong(0)
        p = ctypes.c_int(0)
        b = ctypes.c_double(0)
        _lib.check(_lib.load().dgsn_problem_stats(self._h, ctypes.byref(s), ctypes.byref(p),
                                                  ctypes.byref(b)))
        return dict(solves_per_sweep=s.value, n_planes=p.value, algo_bytes_per_sweep=b.value)

    def set_si_criterion(self, criterion):
        """'maxnorm' (FP64 max-norm relative change), 'eps_s' (Eq. (Test:Eq3)) or
        'fixed' (exactly max_iter iterations)."""
        c = {"maxnorm": _lib.DGSN_SI_MAXNORM, "eps_s": _lib.DGSN_SI_EPS_S,
             "fixed": _lib.DGSN_SI_FIXED}[criterion]
        _lib.check(_lib.load().dgsn_problem_set_si_criterion(self._h, c))

    def set_tile(self, b):
        _lib.check(_lib.load().dgsn_problem_set_tile(self._h, int(b)))

    def tile(self):
        b = ctypes.c_int(0)
        _lib.check(_lib.load().dgsn_problem_get_tile(self._h, ctypes.byref(b)))
        return b.value

    def set_debug(self, poison_fronts=False):
        """poison_fronts: fill the face fronts with NaN before every sweep,
        so that an out-of-order front read shows up as NaN."""
        flags = _lib.DGSN_DEBUG_POISON_FRONTS if poison_fronts else 0
        _lib.check(_lib.load().dgsn_problem_set_debug(self._h, flags))

    def set_schedule(self, schedule, poll_limit=0):
        """'planes' (one launch per hyperplane) or 'dataflow' (one launch per
        sweep, device counters between hyperplanes; every solver)."""
        sc = {"planes": _lib.DGSN_SCHED_PLANES, "dataflow": _lib.DGSN_SCHED_DATAFLOW}[schedule]
        _lib.check(_lib.load().dgsn_problem_set_schedule(self._h, sc, int(poll_limit)))

    def schedule(self):
        s = ctypes.c_int(0)
        _lib.check(_lib.load().dgsn_problem_get_schedule(self._h, ctypes.byref(s)))
        return ("planes", "dataflow")[s.value]

    def check(self):
        """Synchronize and raise if a dataflow wait expired since the last check."""
        _lib.check(_lib.load().dgsn_problem_check(self._h, _stream(self.ctx.device)))

    def autotune(self):
        """Time one sweep with each tile edge 1..3 and schedule and keep the
        fastest; returns (tile, schedule, {(schedule, tile): ms})."""
        t = ctypes.c_int(0)
        s = ctypes.c_int(0)
        ms = np.zeros(6)
        _lib.check(_lib.load().dgsn_problem_autotune(self._h, _stream(self.ctx.device),
                                                     ctypes.byref(t), ctypes.byref(s),
                                                     ms.ctypes.data_as(_lib._PD)))
        names = ("planes", "dataflow")
        times = {(names[k // 3], k % 3 + 1): float(ms[k]) for k in range(6) if np.isfinite(ms[k])}
        return t.value, names[s.value], times

    def set_balance(self, enable=True):
        """Tally the FP64 particle balance of later forward sweeps."""
        _lib.check(_lib.load().dgsn_problem_set_balance(self._h, int(bool(enable))))

    def balance(self):
        """Balance terms of the last tallied sweep: dict with the boundary
        outflow, boundary inflow, absorption, source and their balance
        outflow - inflow + absorption - source."""
        t = np.zeros(5)
        _lib.check(_lib.load().dgsn_problem_balance(self._h, t.ctypes.data_as(_lib._PD),
                                                    _stream(self.ctx.device)))
        return dict(outflow=float(t[0]), inflow=float(t[1]), absorption=float(t[2]),
                    source=float(t[3]), balance=float(t[4]))

    def generation(self):
        """Counter that changes with every change of the problem's inputs or
        of its stored angular flux."""
        g = ctypes.c_ulonglong(0)
        _lib.check(_lib.load().dgsn_problem_generation(self._h, ctypes.byref(g)))
        return g.value

    def set_timing(self, enable=True):
        _lib.check(_lib.load().dgsn_problem_set_timing(self._h, int(bool(enable))))

    def kernel_time(self):
        """(sum of sweep-kernel durations in ms, launches) of the last sweep."""
        ms = ctypes.c_double(0)
        n = ctypes.c_int(0)
        _lib.check(_lib.load().dgsn_problem_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # -- solves -------------------------------------------------------------
    def nodal_empty(self):
        return torch.empty((self.groups, self.ncell, 8), dtype=self.dtype,
                           device=self.ctx.device)

    def sweep(self, src, phi=None):
        """phi = sum_d w_d psi_d of one sweep with total nodal source src."""
        src = self._dev(src, (self.groups, self.ncell, 8))
        phi = phi if phi is not None else self.nodal_empty()
        _lib.check(_lib.load().dgsn_sweep(self._h, _ptr(src), _ptr(phi), _stream(self.ctx.device)))
        return phi

    def source_iterate(self, phi0=None, tol=1e-8, max_iter=1000, allow_notconv=False,
                       phi=None, noalloc=False):
        """Source iteration from phi0 (zero if None) into a new tensor, or in
        place into phi (a [G, ncell, 8] device tensor holding the initial
        guess).  noalloc=True calls dgsn_source_iterate_noalloc, whose scratch
        is the library's static device array (pass phi to keep the call free
        of allocations on the torch side as well)."""
        if phi is None:
            phi = (self._dev(phi0, (self.groups, self.ncell, 8)).clone() if phi0 is not None
                   else torch.zeros((self.groups, self.ncell, 8), dtype=self.dtype,
                                    device=self.ctx.device))
        it = ctypes.c_int(0)
        r = ctypes.c_double(0)
        es = ctypes.c_double(0)
        fn = (_lib.load().dgsn_source_iterate_noalloc if noalloc
              else _lib.load().dgsn_source_iterate)
        rc = fn(self._h, _ptr(phi), float(tol), int(max_iter), ctypes.byref(it),
                ctypes.byref(r), ctypes.byref(es), _stream(self.ctx.device))
        _lib.check(rc, allow=(_lib.DGSN_ENOTCONV,) if allow_notconv else ())
        return phi, dict(iters=it.value, resid=r.value, eps_s=es.value,
                         converged=(rc == _lib.DGSN_OK))

    def si_history(self):
        """Per-iteration residual (max-norm relative change) and eps_S of the
        last source_iterate call, as two float64 arrays."""
        n = ctypes.c_int(0)
        lib = _lib.load()
        _lib.check(lib.dgsn_problem_si_history(self._h, None, None, 0, ctypes.byref(n)))
        r = np.zeros(max(n.value, 1))
        e = np.zeros(max(n.value, 1))
        _lib.check(lib.dgsn_problem_si_history(
            self._h, r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value, ctypes.byref(n)))
        return r[:n.value], e[:n.value]

    def si_step(self, phi):
        """One source iteration in place on phi (source build, sweep, octant
        reduction, FP64 residual); returns the residual."""
        it = ctypes.c_int(0)
        r = ctypes.c_double(0)
        es = ctypes.c_double(0)
        rc = _lib.load().dgsn_source_iterate(self._h, _ptr(phi), 0.0, 1, ctypes.byref(it),
                                             ctypes.byref(r), ctypes.byref(es),
                                             _stream(self.ctx.device))
        _lib.check(rc, allow=(_lib.DGSN_ENOTCONV,))
        return r.value

    def adjoint(self, dj_dphi, tol=1e-8, max_iter=1000, allow_notconv=False):
        g = self._dev(dj_dphi, (self.groups, self.ncell, 8))
        gst = torch.empty((self.groups, self.ncell), dtype=self.dtype, device=self.ctx.device)
        gq = torch.empty_like(gst)
        it = ctypes.c_int(0)
        rc = _lib.load().dgsn_adjoint_solve(self._h, _ptr(g), _ptr(gst), _ptr(gq), float(tol),
                                            int(max_iter), ctypes.byref(it),
                                            _stream(self.ctx.device))
        _lib.check(rc, allow=(_lib.DGSN_ENOTCONV,) if allow_notconv else ())
        return gst, gq, dict(iters=it.value, converged=(rc == _lib.DGSN_OK))

    def close(self):
        if self._h:
            _lib.load().dgsn_problem_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TransportSolve(torch.autograd.Function):
    """phi = SI-solution(sigma_t, q) with sigma_s held fixed; backward by the
    library's adjoint sweep (reversed directions, transposed cell systems).

    forward(problem, sigma_t [G,ncell], q [G,ncell], sigma_s [G,ncell], tol,
    max_iter) -> phi [G,ncell,8].  The problem must be created with
    store_psi=True.  The backward pass uses the angular flux and materials the
    problem holds, so it raises if the problem changed after this forward
    (another forward, a sweep or a setter on the same problem); use one
    problem per pending backward.  A forward or adjoint iteration that stops
    before tol warns.
    """

    @staticmethod
    def forward(ctx, problem, sigma_t, q, sigma_s, tol, max_iter):
        problem.set_materials(sigma_t.detach(), sigma_s.detach(), q.detach())
        phi, info = problem.source_iterate(tol=tol, max_iter=max_iter, allow_notconv=True)
        if not info["converged"]:
            warnings.warn(f"TransportSolve forward stopped after {info['iters']} iterations at "
                          f"residual {info['resid']:.3e} (tol {tol:g}); gradients are those of "
                          "the last iterate", RuntimeWarning, stacklevel=2)
        ctx.problem = problem
        ctx.generation = problem.generation()
        ctx.tol = tol
        ctx.max_iter = max_iter
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        if ctx.problem.generation() != ctx.generation:
            raise RuntimeError("TransportSolve.backward: the problem changed after this forward "
                               "(another forward, sweep or setter); its stored angular flux no "
                               "longer belongs to this graph")
        gst, gq, info = ctx.problem.adjoint(grad_phi.contiguous(), tol=ctx.tol,
                                            max_iter=ctx.max_iter, allow_notconv=True)
        if not info["converged"]:
            warnings.warn(f"TransportSolve adjoint stopped after {info['iters']} iterations "
                          f"(tol {ctx.tol:g})", RuntimeWarning, stacklevel=2)
        return None, gst, gq, None, None, None


class Batch:
    """One sweep of many independent FP32 problems in one HIP-graph launch."""

    def __init__(self, ctx, problems):
        self.ctx = ctx
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().dgsn_batch_create(ctx._h, arr, len(self.problems),
                                                 ctypes.byref(self._h)))
        self._io = [None] * len(self.problems)

    def set_io(self, index, src, phi):
        self._io[index] = (src, phi)   # keep the tensors alive
        _lib.check(_lib.load().dgsn_batch_set_io(self._h, int(index), _ptr(src), _ptr(phi)))

    def set_tiles(self, tiles):
        arr = (ctypes.c_int * len(self.problems))(*[int(t) for t in tiles])
        _lib.check(_lib.load().dgsn_batch_set_tiles(self._h, arr))

    def set_schedule(self, schedule):
        """'planes' (one batched kernel per step) or 'dataflow' (one launch)."""
        sc = {"planes": _lib.DGSN_SCHED_PLANES, "dataflow": _lib.DGSN_SCHED_DATAFLOW}[schedule]
        _lib.check(_lib.load().dgsn_batch_set_schedule(self._h, sc))

    def schedule(self):
        s = ctypes.c_int(0)
        _lib.check(_lib.load().dgsn_batch_get_schedule(self._h, ctypes.byref(s)))
        return ("planes", "dataflow")[s.value]

    def autotune(self):
        ms = ctypes.c_double(0)
        _lib.check(_lib.load().dgsn_batch_autotune(self._h, _stream(self.ctx.device),
                                                   ctypes.byref(ms)))
        return ms.value

    def run(self):
        _lib.check(_lib.load().dgsn_batch_run(self._h, _stream(self.ctx.device)))

    def latencies_us(self):
        out = np.zeros(len(self.problems))
        _lib.check(_lib.load().dgsn_batch_latencies_us(self._h, out.ctypes.data_as(_lib._PD)))
        return out

    def close(self):
        if self._h:
            _lib.load().dgsn_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
