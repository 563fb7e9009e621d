"""FP64 CPU oracle for the DGFEM S_n sweep of Tano & Ragusa (arXiv 1906.04017).

TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It is a plain, slow, obviously-correct implementation written
from the paper: element matrices by Gauss quadrature, cell systems assembled
term by term, Gaussian elimination with partial pivoting, sweeps by nested
loops in upwind order, source iteration, the exact discrete adjoint, and the
FP64 forward passes of the two shallow networks (the canonical 24-input one
and the paper's 26-input tanh/ELU form, per octant or per quadrature
direction).  It shares no code with the HIP library.

Array conventions (identical to the library's public layout, but implemented
separately): cell index c = i + nx (j + ny k); nodal fields are
[G][ncell][8] with local node n = ix + 2 iy + 4 iz fastest; per-cell fields are
[G][ncell]; faces f = 2 axis + side (side 1 = high face).

Parity status of each function is recorded in its docstring; every function
here is pinned by the ``-m "not gpu"`` tests (closed forms, brute force,
invariants, finite differences), except where a docstring says
"parity unpinned".
"""
import ctypes
import os

import numpy as np

from .quadrature import lq_n  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "dgfem.c")
    if (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        from .build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_element_matrices.argtypes = [_D, _D, _D, _D]
    lib.orc_ge_solve.argtypes = [ctypes.c_int, _D, _D, _D]
    lib.orc_sweep.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [ctypes.c_int] * 2 + \
        [_D] * 5 + [_D, _D, ctypes.c_int]
    lib.orc_source_iterate.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 6 + [_D, ctypes.c_double, ctypes.c_int, _I, _D, _D, _D,
                                          ctypes.c_int]
    lib.orc_adjoint.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [ctypes.c_int] * 2 + \
        [_D] * 7 + [ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _I, ctypes.c_int]
    lib.orc_source_iterate_gg.argtypes = lib.orc_source_iterate.argtypes
    lib.orc_source_iterate_eps.argtypes = lib.orc_source_iterate.argtypes
    lib.orc_adjoint_gg.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 7 + [ctypes.c_double, ctypes.c_int, _D, _D, _D, _I,
                                         ctypes.c_int]
    lib.orc_cell_balance.argtypes = [_D, _D, ctypes.c_double, _D, _D, _D]
    lib.orc_cell_balance.restype = ctypes.c_double
    lib.orc_cell_solve_batch.argtypes = [ctypes.c_long, _D, _D, _D, _D, _D, _D, ctypes.c_int]
    lib.orc_ann_features.argtypes = [_D, _D, ctypes.c_double, _D, _D, _D, _D]
    lib.orc_ann_forward.argtypes = [ctypes.c_int] * 4 + [_D] * 6
    lib.orc_ann_cell_batch.argtypes = [ctypes.c_long, _D, _D, _D, _D, _D, ctypes.c_int,
                                       ctypes.c_int, _D, _D, _D, _D, _D]
    lib.orc_ann_sweep.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 5 + [ctypes.c_int, ctypes.c_int] + [_D] * 5 + [ctypes.c_int]
    lib.orc_ann_source_iterate.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 6 + [ctypes.c_int, ctypes.c_int] + [_D] * 5 + \
        [ctypes.c_double, ctypes.c_int, _I, _D, _D, ctypes.c_int]
    lib.orc_pann_octant.argtypes = [_D]
    lib.orc_pann_inputs.argtypes = [_D, _D, ctypes.c_double, _D, _D, _D]
    _pann = [ctypes.c_int, ctypes.c_double, ctypes.c_double] + [_D] * 6 + [ctypes.c_int, _D]
    lib.orc_pann_forward.argtypes = _pann + [ctypes.c_int, _D, _D]
    lib.orc_pann_cell_batch.argtypes = [ctypes.c_long] + [_D] * 5 + _pann + [_D]
    lib.orc_pann_sweep.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 5 + _pann + [_D, _D, ctypes.c_int]
    lib.orc_pann_source_iterate.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 6 + _pann + [_D, ctypes.c_double, ctypes.c_int, _I, _D, _D,
                                                 ctypes.c_int]
    lib.orc_real_ylm.argtypes = [ctypes.c_int, _D, _D]
    lib.orc_si_metrics.argtypes = [ctypes.c_long, _D, _D, _D, _D]
    lib.orc_sweep_balance.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 7
    lib.orc_source_iterate_pl.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 3 + [ctypes.c_int] + [_D] * 5 + \
        [ctypes.c_double, ctypes.c_int, _I, _D, _D, _D, ctypes.c_int]
    lib.orc_adjoint_pl.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + \
        [ctypes.c_int] * 2 + [_D] * 3 + [ctypes.c_int] + [_D] * 4 + \
        [ctypes.c_double, ctypes.c_int, _D, _D, _D, _I, ctypes.c_int]
    lib.orc_source_iterate_pl_gg.argtypes = lib.orc_source_iterate_pl.argtypes
    lib.orc_adjoint_pl_gg.argtypes = lib.orc_adjoint_pl.argtypes
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


ORC_ENOTCONV = -4


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc not in (0, ORC_ENOTCONV):
        raise OracleError(f"{what} failed with code {rc}")
    return rc


# ---------------------------------------------------------------------------
# element level
# ---------------------------------------------------------------------------

def element_matrices(h):
    """Mass M, gradient G[a] (test-function derivative) and face masses Mf[f]
    of one hexahedron with edge lengths h, by 2-point Gauss quadrature
    (weak form under Eq. (T9)).  Pinned by the Kronecker closed form."""
    lib = _load()
    h = _f64(h, (3,))
    M = np.zeros(64)
    G = np.zeros(3 * 64)
    Mf = np.zeros(6 * 64)
    lib.orc_element_matrices(_p(h), _p(M), _p(G), _p(Mf))
    return M.reshape(8, 8), G.reshape(3, 8, 8), Mf.reshape(6, 8, 8)


def ge_solve(A, b):
    """Gaussian elimination with partial pivoting (Eq. (T12) solve)."""
    lib = _load()
    A = _f64(A)
    n = A.shape[0]
    b = _f64(b, (n,))
    x = np.zeros(n)
    rc = lib.orc_ge_solve(n, _p(A), _p(b), _p(x))
    if rc:
        raise OracleError(f"ge_solve failed ({rc})")
    return x


def cell_balance(h, omega, sigma_t, S, psi_up, psi):
    """1^T (A psi - b) of one cell system (particle balance residual)."""
    lib = _load()
    return lib.orc_cell_balance(_p(_f64(h, (3,))), _p(_f64(omega, (3,))), float(sigma_t),
                                _p(_f64(S, (8,))), _p(_f64(psi_up, (6, 8))), _p(_f64(psi, (8,))))


def cell_solve_batch(h, omega, sigma_t, S, psi_up, nthreads=0):
    """Batched one-cell assemble + GE in physical orientation.
    h, omega [n,3]; sigma_t [n]; S [n,8]; psi_up [n,6,8] (inflow faces only)."""
    lib = _load()
    omega = _f64(omega)
    n = omega.shape[0]
    h = _f64(np.broadcast_to(np.asarray(h, np.float64), (n, 3)))
    out = np.zeros((n, 8))
    rc = lib.orc_cell_solve_batch(n, _p(h), _p(omega), _p(_f64(sigma_t, (n,))), _p(_f64(S, (n, 8))),
                                  _p(_f64(psi_up, (n, 6, 8))), _p(out), int(nthreads))
    _check(rc, "cell_solve_batch")
    return out


# ---------------------------------------------------------------------------
# sweep / source iteration / adjoint
# ---------------------------------------------------------------------------

def _mesh_args(mesh):
    nx, ny, nz, lx, ly, lz = mesh
    return int(nx), int(ny), int(nz), float(lx), float(ly), float(lz)


def sweep(mesh, omega, weight, sigma_t, src, psi_inc=None, store_psi=False, nthreads=0):
    """One full sweep (all directions, all groups).

    mesh = (nx, ny, nz, lx, ly, lz); omega [D,3]; weight [D];
    sigma_t [G, ncell]; src [G, ncell, 8] total nodal source per steradian;
    psi_inc [6] per domain face.  Returns phi [G, ncell, 8] (and psi
    [D, G, ncell, 8] with store_psi).  Pinned by brute force and invariants.
    """
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    src = _f64(src, (ng, ncell, 8))
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    phi = np.zeros((ng, ncell, 8))
    psi = np.zeros((nd, ng, ncell, 8)) if store_psi else None
    rc = lib.orc_sweep(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))),
                       _p(sigma_t), _p(src), _p(inc), _p(phi), _p(psi), int(nthreads))
    _check(rc, "sweep")
    return (phi, psi) if store_psi else phi


def si_metrics(phi_new, phi_old):
    """(r, eps_s) of one source-iteration step: the max-norm relative change
    and Eq. (Test:Eq3) on cell averages (orc_si_metrics).  phi_* [..., 8]
    nodal fluxes of the same shape (the last axis the cell's 8 nodes)."""
    lib = _load()
    a = _f64(phi_new).reshape(-1, 8)
    b = _f64(phi_old).reshape(-1, 8)
    if a.shape != b.shape:
        raise ValueError("phi_new and phi_old must have the same shape")
    r = ctypes.c_double(0)
    e = ctypes.c_double(0)
    lib.orc_si_metrics(a.shape[0], _p(a), _p(b), ctypes.byref(r), ctypes.byref(e))
    return r.value, e.value


def sweep_balance(mesh, omega, weight, sigma_t, src, psi_inc, psi):
    """Particle balance of one sweep from its stored angular flux psi
    [D, G, ncell, 8] (orc_sweep_balance): dict with the weighted outflow and
    inflow over all cell faces and over the domain boundary, absorption and
    source."""
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    out = np.zeros(6)
    rc = lib.orc_sweep_balance(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))),
                               _p(sigma_t), _p(_f64(src, (ng, ncell, 8))),
                               _p(_f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))),
                               _p(_f64(psi, (nd, ng, ncell, 8))), _p(out))
    _check(rc, "sweep_balance")
    return dict(outflow_all=out[0], inflow_all=out[1], outflow=out[2], inflow=out[3],
                absorption=out[4], source=out[5])


def source_iterate(mesh, omega, weight, sigma_t, sigma_s, q, psi_inc=None, tol=1e-8,
                   max_iter=1000, phi0=None, store_psi=False, nthreads=0, sigma_gg=None,
                   criterion="maxnorm"):
    """Scattering source iteration to max-norm relative change < tol, or with
    criterion="eps_s" to Eq. (Test:Eq3) < tol (in-group scattering only).
    sigma_gg [G, G, ncell] (from g' into g at [g', g]) replaces the in-group
    sigma_s with multigroup scattering when given.
    Returns dict(phi, iters, resid, eps_s, converged[, psi])."""
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    sigma_s = _f64(sigma_s, (ng, ncell))
    q = _f64(q, (ng, ncell))
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    phi = np.zeros((ng, ncell, 8)) if phi0 is None else _f64(phi0, (ng, ncell, 8)).copy()
    psi = np.zeros((nd, ng, ncell, 8)) if store_psi else None
    it = ctypes.c_int(0)
    resid = ctypes.c_double(0)
    eps = ctypes.c_double(0)
    if criterion not in ("maxnorm", "eps_s") or (criterion == "eps_s" and sigma_gg is not None):
        raise ValueError("criterion must be 'maxnorm', or 'eps_s' without sigma_gg")
    if sigma_gg is None:
        fn = lib.orc_source_iterate if criterion == "maxnorm" else lib.orc_source_iterate_eps
        rc = fn(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))),
                _p(sigma_t), _p(sigma_s), _p(q), _p(inc), _p(phi), float(tol), int(max_iter),
                ctypes.byref(it), ctypes.byref(resid), ctypes.byref(eps), _p(psi),
                int(nthreads))
    else:
        rc = lib.orc_source_iterate_gg(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega),
                                       _p(_f64(weight, (nd,))), _p(sigma_t),
                                       _p(_f64(sigma_gg, (ng, ng, ncell))), _p(q), _p(inc),
                                       _p(phi), float(tol), int(max_iter), ctypes.byref(it),
                                       ctypes.byref(resid), ctypes.byref(eps), _p(psi),
                                       int(nthreads))
    _check(rc, "source_iterate")
    out = dict(phi=phi, iters=it.value, resid=resid.value, eps_s=eps.value, converged=(rc == 0))
    if store_psi:
        out["psi"] = psi
    return out


def adjoint(mesh, omega, weight, sigma_t, sigma_s, psi, phi, gphi, tol=1e-13, max_iter=2000,
            nthreads=0, sigma_gg=None, sigma_sn=None, pl_gg=False):
    """Exact discrete adjoint of the converged source iteration.
    gphi = dJ/dphi [G, ncell, 8].  Returns dict(grad_sigma_t, grad_q,
    grad_sigma_s [G, ncell], phi_dag [G, ncell, 8], iters); direct partial
    derivatives of J are not included.  With sigma_gg (multigroup scattering,
    the transposed coupling in the adjoint) grad_sigma_s is not computed;
    with sigma_sn [L+1, G, ncell] (in-group P_L, order 0 first; sigma_s is
    then ignored), or with pl_gg a matrix per order [L+1, G, G, ncell]
    (from g' into g at [n, g', g]; sigma_s and sigma_gg are then ignored),
    neither.  Pinned by duality, the dense transpose and central finite
    differences."""
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    gst = np.zeros((ng, ncell))
    gq = np.zeros((ng, ncell))
    gss = np.zeros((ng, ncell))
    pd = np.zeros((ng, ncell, 8))
    it = ctypes.c_int(0)
    if sigma_sn is not None:
        gss = None
        sn = _f64(sigma_sn).reshape((-1, ng, ng, ncell) if pl_gg else (-1, ng, ncell))
        fn = lib.orc_adjoint_pl_gg if pl_gg else lib.orc_adjoint_pl
        rc = fn(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega),
                _p(_f64(weight, (nd,))), _p(sigma_t), int(sn.shape[0] - 1),
                _p(sn), _p(_f64(psi, (nd, ng, ncell, 8))),
                _p(_f64(phi, (ng, ncell, 8))), _p(_f64(gphi, (ng, ncell, 8))),
                float(tol), int(max_iter), _p(gst), _p(gq), _p(pd),
                ctypes.byref(it), int(nthreads))
    elif sigma_gg is None:
        rc = lib.orc_adjoint(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))),
                             _p(sigma_t), _p(_f64(sigma_s, (ng, ncell))),
                             _p(_f64(psi, (nd, ng, ncell, 8))), _p(_f64(phi, (ng, ncell, 8))),
                             _p(_f64(gphi, (ng, ncell, 8))), float(tol), int(max_iter), _p(gst),
                             _p(gq), _p(gss), _p(pd), ctypes.byref(it), int(nthreads))
    else:
        gss = None
        rc = lib.orc_adjoint_gg(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega),
                                _p(_f64(weight, (nd,))), _p(sigma_t),
                                _p(_f64(sigma_gg, (ng, ng, ncell))),
                                _p(_f64(psi, (nd, ng, ncell, 8))), _p(_f64(phi, (ng, ncell, 8))),
                                _p(_f64(gphi, (ng, ncell, 8))), float(tol), int(max_iter),
                                _p(gst), _p(gq), _p(pd), ctypes.byref(it), int(nthreads))
    _check(rc, "adjoint")
    return dict(grad_sigma_t=gst, grad_q=gq, grad_sigma_s=gss, phi_dag=pd, iters=it.value,
                converged=(rc == 0))


# ---------------------------------------------------------------------------
# shallow ANN (Sec. 3)
# ---------------------------------------------------------------------------

ACT_RELU = 0
ACT_TANH = 1


def ann_features(h, omega, sigma_t, S, psi_up):
    """Canonical 24-feature input and homogeneity scale m of one cell."""
    lib = _load()
    x = np.zeros(24)
    m = np.zeros(1)
    lib.orc_ann_features(_p(_f64(h, (3,))), _p(_f64(omega, (3,))), float(sigma_t), _p(_f64(S, (8,))),
                         _p(_f64(psi_up, (6, 8))), _p(x), _p(m))
    return x, float(m[0])


def ann_forward(net, x):
    """FP64 forward pass, Eq. (ANN:Eq1) with a linear output layer."""
    lib = _load()
    W1, b1, W2, b2 = (_f64(net[k]) for k in ("W1", "b1", "W2", "b2"))
    nh, nin = W1.shape
    nout = W2.shape[0]
    x = _f64(x, (nin,))
    y = np.zeros(nout)
    lib.orc_ann_forward(nin, nh, nout, int(net.get("act", ACT_RELU)), _p(W1), _p(b1), _p(W2),
                        _p(b2), _p(x), _p(y))
    return y


def _net_args(net):
    W1, b1, W2, b2 = (_f64(net[k]) for k in ("W1", "b1", "W2", "b2"))
    return W1.shape[0], int(net.get("act", ACT_RELU)), W1, b1, W2, b2


def ann_cell_batch(net, h, omega, sigma_t, S, psi_up):
    lib = _load()
    omega = _f64(omega)
    n = omega.shape[0]
    h = _f64(np.broadcast_to(np.asarray(h, np.float64), (n, 3)))
    nh, act, W1, b1, W2, b2 = _net_args(net)
    out = np.zeros((n, 8))
    rc = lib.orc_ann_cell_batch(n, _p(h), _p(omega), _p(_f64(sigma_t, (n,))), _p(_f64(S, (n, 8))),
                                _p(_f64(psi_up, (n, 6, 8))), nh, act, _p(W1), _p(b1), _p(W2),
                                _p(b2), _p(out))
    _check(rc, "ann_cell_batch")
    return out


def ann_sweep(net, mesh, omega, weight, sigma_t, src, psi_inc=None, nthreads=0):
    """Sweep with the ANN forward pass in place of assembly + GE."""
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    nh, act, W1, b1, W2, b2 = _net_args(net)
    phi = np.zeros((ng, ncell, 8))
    rc = lib.orc_ann_sweep(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))),
                           _p(sigma_t), _p(_f64(src, (ng, ncell, 8))), _p(inc), nh, act, _p(W1),
                           _p(b1), _p(W2), _p(b2), _p(phi), int(nthreads))
    _check(rc, "ann_sweep")
    return phi


def ann_source_iterate(net, mesh, omega, weight, sigma_t, sigma_s, q, psi_inc=None, tol=1e-4,
                       max_iter=1000, nthreads=0):
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    nh, act, W1, b1, W2, b2 = _net_args(net)
    phi = np.zeros((ng, ncell, 8))
    it = ctypes.c_int(0)
    resid = ctypes.c_double(0)
    eps = ctypes.c_double(0)
    rc = lib.orc_ann_source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega),
                                    _p(_f64(weight, (nd,))), _p(sigma_t),
                                    _p(_f64(sigma_s, (ng, ncell))), _p(_f64(q, (ng, ncell))),
                                    _p(inc), nh, act, _p(W1), _p(b1), _p(W2), _p(b2), _p(phi),
                                    float(tol), int(max_iter), ctypes.byref(it),
                                    ctypes.byref(resid), ctypes.byref(eps), int(nthreads))
    _check(rc, "ann_source_iterate")
    return dict(phi=phi, iters=it.value, resid=resid.value, eps_s=eps.value, converged=(rc == 0))


# ---------------------------------------------------------------------------
# paper-form per-octant network (Sec. 3, Eq. (ANN:Eq1)-(ANN:Eq4))
# ---------------------------------------------------------------------------
# net = dict(kind="paper", W1 [K][nh][26], b1 [K][nh], W2 [K][8][nh], b2 [K][8],
#            imin [26], imax [26], alpha, beta_scale[, omega [K][3]]):
# K = 8 networks, one per octant, or with omega one network per quadrature
# direction (net k serves the direction omega[k])

def pann_octant(omega):
    """Octant o = [omega_x < 0] + 2 [omega_y < 0] + 4 [omega_z < 0]."""
    return int(_load().orc_pann_octant(_p(_f64(omega, (3,)))))


def pann_inputs(h, omega, sigma_t, S, psi_up):
    """The 26 physical-frame inputs of one cell (see orc_pann_inputs)."""
    I = np.zeros(26)
    _load().orc_pann_inputs(_p(_f64(h, (3,))), _p(_f64(omega, (3,))), float(sigma_t),
                            _p(_f64(S, (8,))), _p(_f64(psi_up, (6, 8))), _p(I))
    return I


def _pann_args(net):
    W1 = _f64(net["W1"])
    nh = W1.shape[1]
    om = net.get("omega")
    k = 8 if om is None else _f64(om).shape[0]
    if W1.shape != (k, nh, 26):
        raise ValueError(f"paper network W1 must be [{k}][nh][26]")
    om = np.zeros((1, 3)) if om is None else _f64(om, (k, 3))
    return (nh, float(net["alpha"]), float(net["beta_scale"]), _f64(net["imin"], (26,)),
            _f64(net["imax"], (26,)), W1, _f64(net["b1"], (k, nh)), _f64(net["W2"], (k, 8, nh)),
            _f64(net["b2"], (k, 8)), 0 if net.get("omega") is None else k, om)


def _pann_ptrs(a):
    nh, alpha, bs, imin, imax, W1, b1, W2, b2, ndir, om = a
    return [nh, alpha, bs] + [_p(x) for x in (imin, imax, W1, b1, W2, b2)] + [ndir, _p(om)]


def pann_forward(net, octant, I):
    """FP64 forward pass of net `octant` (the octant's network, or with
    per-direction networks the direction's index) on raw inputs I[26] -> psi[8]."""
    a = _pann_args(net)
    psi = np.zeros(8)
    rc = _load().orc_pann_forward(*_pann_ptrs(a), int(octant), _p(_f64(I, (26,))), _p(psi))
    _check(rc, "pann_forward")
    return psi


def pann_cell_batch(net, h, omega, sigma_t, S, psi_up):
    """Batched one-cell solves by the paper-form network (physical orientation)."""
    omega = _f64(omega)
    n = omega.shape[0]
    h = _f64(np.broadcast_to(np.asarray(h, np.float64), (n, 3)))
    a = _pann_args(net)
    out = np.zeros((n, 8))
    rc = _load().orc_pann_cell_batch(n, _p(h), _p(omega), _p(_f64(sigma_t, (n,))),
                                     _p(_f64(S, (n, 8))), _p(_f64(psi_up, (n, 6, 8))),
                                     *_pann_ptrs(a), _p(out))
    _check(rc, "pann_cell_batch")
    return out


def pann_sweep(net, mesh, omega, weight, sigma_t, src, psi_inc=None, nthreads=0,
               store_psi=False):
    """Sweep with the paper-form network in place of assembly + GE (and
    the angular flux [D, G, ncell, 8] with store_psi)."""
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    phi = np.zeros((ng, ncell, 8))
    psi = np.zeros((nd, ng, ncell, 8)) if store_psi else None
    rc = lib.orc_pann_sweep(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))),
                            _p(sigma_t), _p(_f64(src, (ng, ncell, 8))), _p(inc),
                            *_pann_ptrs(_pann_args(net)), _p(phi), _p(psi), int(nthreads))
    _check(rc, "pann_sweep")
    return (phi, psi) if store_psi else phi


def pann_source_iterate(net, mesh, omega, weight, sigma_t, sigma_s, q, psi_inc=None, tol=1e-4,
                        max_iter=1000, nthreads=0):
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    phi = np.zeros((ng, ncell, 8))
    it = ctypes.c_int(0)
    resid = ctypes.c_double(0)
    eps = ctypes.c_double(0)
    rc = lib.orc_pann_source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega),
                                     _p(_f64(weight, (nd,))), _p(sigma_t),
                                     _p(_f64(sigma_s, (ng, ncell))), _p(_f64(q, (ng, ncell))),
                                     _p(inc), *_pann_ptrs(_pann_args(net)), _p(phi), float(tol),
                                     int(max_iter), ctypes.byref(it), ctypes.byref(resid),
                                     ctypes.byref(eps), int(nthreads))
    _check(rc, "pann_source_iterate")
    return dict(phi=phi, iters=it.value, resid=resid.value, eps_s=eps.value, converged=(rc == 0))


# ---------------------------------------------------------------------------
# error metrics (Sec. 4)
# ---------------------------------------------------------------------------

def real_ylm(L, omega):
    """Real orthonormal spherical harmonics Y[d][k], k = n^2 + n + m, n <= L,
    at the unit directions omega [D, 3] (polar axis z, no (-1)^m phase)."""
    lib = _load()
    om = _f64(omega).reshape(-1, 3)
    nm = (L + 1) ** 2
    out = np.zeros((om.shape[0], nm))
    for d in range(om.shape[0]):
        row = np.zeros(nm)
        _check(lib.orc_real_ylm(int(L), _p(np.ascontiguousarray(om[d])), _p(row)), "real_ylm")
        out[d] = row
    return out


def source_iterate_pl(mesh, omega, weight, sigma_t, sigma_sn, q, psi_inc=None, tol=1e-8,
                      max_iter=1000, phi0=None, mom0=None, nthreads=0, store_psi=False,
                      gg=False):
    """P_L scattering source iteration (Eq. (T3)-(T8)).
    sigma_sn [L+1, G, ncell] in-group, or with gg a group-to-group matrix
    per order [L+1, G, G, ncell] (from g' into g at [n, g', g]), order 0
    first; returns dict(phi [G, ncell, 8], mom [(L+1)^2 - 1, G, ncell, 8]
    (the moments k = n^2 + n + m >= 1), iters, resid, eps_s, converged)."""
    lib = _load()
    nx, ny, nz, lx, ly, lz = _mesh_args(mesh)
    ncell = nx * ny * nz
    omega = _f64(omega)
    nd = omega.shape[0]
    sigma_t = _f64(sigma_t).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    sigma_sn = _f64(sigma_sn).reshape((-1, ng, ng, ncell) if gg else (-1, ng, ncell))
    L = sigma_sn.shape[0] - 1
    q = _f64(q, (ng, ncell))
    inc = _f64(np.zeros(6) if psi_inc is None else psi_inc, (6,))
    phi = np.zeros((ng, ncell, 8)) if phi0 is None else _f64(phi0, (ng, ncell, 8)).copy()
    nm = (L + 1) ** 2
    mom = np.zeros((nm - 1, ng, ncell, 8)) if mom0 is None else \
        _f64(mom0, (nm - 1, ng, ncell, 8)).copy()
    it = ctypes.c_int(0)
    resid = ctypes.c_double(0)
    eps = ctypes.c_double(0)
    psi = np.zeros((nd, ng, ncell, 8)) if store_psi else None
    fn = lib.orc_source_iterate_pl_gg if gg else lib.orc_source_iterate_pl
    rc = fn(nx, ny, nz, lx, ly, lz, ng, nd, _p(omega), _p(_f64(weight, (nd,))), _p(sigma_t),
            int(L), _p(sigma_sn), _p(q), _p(inc), _p(phi), _p(mom), float(tol), int(max_iter),
            ctypes.byref(it), ctypes.byref(resid), ctypes.byref(eps), _p(psi), int(nthreads))
    if rc not in (0, ORC_ENOTCONV):
        _check(rc, "source_iterate_pl")
    out = dict(phi=phi, mom=mom, iters=it.value, resid=resid.value, eps_s=eps.value,
               converged=(rc == 0))
    if store_psi:
        out["psi"] = psi
    return out


def cell_average(phi):
    """Cell average of a nodal trilinear field [G, ncell, 8] -> [G, ncell]."""
    return np.asarray(phi, np.float64).mean(axis=-1)


def eps_p(phi_ref, phi, m=1e-8):
    """Eq. (Test:Eq2): mean over cells of |phi - phi_ann| / (|phi| + m), on
    cell averages, per group."""
    a = cell_average(phi_ref)
    b = cell_average(phi)
    return (np.abs(a - b) / (np.abs(a) + m)).mean(axis=-1)


def rel_err(phi_ref, phi):
    """Norm-wise relative error max|phi - ref| / max|ref| per group."""
    a = np.asarray(phi_ref, np.float64)
    b = np.asarray(phi, np.float64)
    ax = tuple(range(1, a.ndim))
    return np.abs(a - b).max(axis=ax) / np.abs(a).max(axis=ax)
