"""Seeded synthetic inputs for the DGFEM S_n sweep workloads.

This module only draws material fields, sources and boundary data with
``numpy.random.default_rng(seed)`` (PCG64).  It holds none of the method's
arithmetic (no quadrature, no element matrices, no solves), so that both the
HIP library path and the independent FP64 oracle can be fed the very same
arrays.

Array conventions: per-cell fields are float64 [G][Nz][Ny][Nx] flattened to
[G][ncell] with c = i + Nx (j + Ny k); boundary inflow is one value per domain
face in the order x-, x+, y-, y+, z-, z+.

Workloads (the paper's own problems are cubes of 10 cm with uniform hex cells,
Tables P1-P4 of Sec. 4; the other recipes are synthetic stand-ins of the same
structure):

* ``absorber_cube``   8^3 unit cube, S4, 1 group, sigma_t ~ U[1, 10] per cell,
                      pure absorber, q = 1 per steradian, vacuum.
* ``blocky_scatter``  64^3 unit cube, S8, 8 groups; 8x8x8 material blocks, per
                      (group, block) sigma_t = clip(exp(N(0,1)), 0.1, 50),
                      c ~ U[0, 0.9], sigma_s = c sigma_t; q = 1; vacuum.
* ``paper_problems``  10 cm cube, 128^3, S8, 4 groups where group g carries the
                      materials of the paper's Problem g+1 (sigma_t 10 / 0.001 /
                      10 / 10, sigma_s 0 / 0 / 0 / 9.9, q 0 / 0 / 1 / 1);
                      psi_inc = 1 on the x-, y-, z- faces, vacuum elsewhere.
* ``adjoint_box``     32^3 unit cube, S4, 2 groups, sigma_t ~ U[1, 10] per
                      (group, cell), sigma_s = 0.5 sigma_t, q = 1, vacuum;
                      response box = cells 12..19 on every axis.
* ``uneven_batch``    64 independent cubes, N in {16, 24, ..., 96}, S_N in
                      {4, ..., 12}, 1..8 groups, GE or ANN with p = 1/2,
                      blocky materials as above (8 blocks per axis), q = 1,
                      vacuum.
"""
import numpy as np


def _ncell(n):
    return int(n[0]) * int(n[1]) * int(n[2])


def blocky_materials(n, groups, seed, blocks=8, c_max=0.9, lognormal=True):
    """Block-constant random materials on an n = (nx, ny, nz) grid.

    Per (group, block): sigma_t = clip(exp(N(0, 1)), 0.1, 50), scattering ratio
    c ~ U[0, c_max], sigma_s = c sigma_t.  Returns (sigma_t, sigma_s) [G, ncell].
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in n)
    bx, by, bz = (min(blocks, nx), min(blocks, ny), min(blocks, nz))
    if lognormal:
        st_b = np.clip(np.exp(rng.normal(0.0, 1.0, size=(groups, bz, by, bx))), 0.1, 50.0)
    else:
        st_b = rng.uniform(1.0, 10.0, size=(groups, bz, by, bx))
    c_b = rng.uniform(0.0, c_max, size=(groups, bz, by, bx))
    ix = (np.arange(nx) * bx) // nx
    iy = (np.arange(ny) * by) // ny
    iz = (np.arange(nz) * bz) // nz
    st = st_b[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]]
    cc = c_b[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]]
    return st.reshape(groups, -1).copy(), (cc * st).reshape(groups, -1).copy()


def problem(n, length, order, groups, sigma_t, sigma_s, q, psi_inc, name):
    n = tuple(int(v) for v in n)
    length = tuple(float(v) for v in length)
    ncell = _ncell(n)
    return dict(
        name=name, n=n, length=length, order=int(order), groups=int(groups),
        sigma_t=np.ascontiguousarray(np.asarray(sigma_t, np.float64).reshape(groups, ncell)),
        sigma_s=np.ascontiguousarray(np.asarray(sigma_s, np.float64).reshape(groups, ncell)),
        q=np.ascontiguousarray(np.asarray(q, np.float64).reshape(groups, ncell)),
        psi_inc=np.asarray(psi_inc, np.float64).reshape(6).copy(),
    )


def absorber_cube(n=8, seed=1, order=4):
    rng = np.random.default_rng(seed)
    ncell = n ** 3
    st = rng.uniform(1.0, 10.0, size=(1, ncell))
    return problem((n, n, n), (1.0, 1.0, 1.0), order, 1, st, np.zeros((1, ncell)),
                   np.ones((1, ncell)), np.zeros(6), f"absorber_cube_{n}^3_S{order}_G1")


def blocky_scatter(n=64, groups=8, seed=2, order=8, blocks=8):
    st, ss = blocky_materials((n, n, n), groups, seed, blocks=blocks)
    ncell = n ** 3
    return problem((n, n, n), (1.0, 1.0, 1.0), order, groups, st, ss, np.ones((groups, ncell)),
                   np.zeros(6), f"blocky_scatter_{n}^3_S{order}_G{groups}")


# materials of the paper's four test problems (Tables P1-P4 of Sec. 4)
PAPER_PROBLEMS = (
    dict(sigma_t=10.0, sigma_s=0.0, q=0.0),    # Problem 1: thick pure absorber
    dict(sigma_t=0.001, sigma_s=0.0, q=0.0),   # Problem 2: quasi-transparent
    dict(sigma_t=10.0, sigma_s=0.0, q=1.0),    # Problem 3: absorber with source
    dict(sigma_t=10.0, sigma_s=9.9, q=1.0),    # Problem 4: scattering, c = 0.99
)


def paper_problems(n=128, groups=4, order=8, length=10.0):
    ncell = n ** 3
    st = np.zeros((groups, ncell))
    ss = np.zeros((groups, ncell))
    q = np.zeros((groups, ncell))
    for g in range(groups):
        p = PAPER_PROBLEMS[g % 4]
        st[g] = p["sigma_t"]
        ss[g] = p["sigma_s"]
        q[g] = p["q"]
    inc = np.array([1.0, 0.0, 1.0, 0.0, 1.0, 0.0])
    return problem((n, n, n), (length,) * 3, order, groups, st, ss, q, inc,
                   f"paper_problems_{n}^3_S{order}_G{groups}")


def adjoint_box(n=32, groups=2, seed=4, order=4, c=0.5, box=(12, 20)):
    rng = np.random.default_rng(seed)
    ncell = n ** 3
    st = rng.uniform(1.0, 10.0, size=(groups, ncell))
    p = problem((n, n, n), (1.0, 1.0, 1.0), order, groups, st, c * st, np.ones((groups, ncell)),
                np.zeros(6), f"adjoint_box_{n}^3_S{order}_G{groups}")
    lo, hi = box
    lo = max(0, min(lo, n))
    hi = max(lo, min(hi, n))
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    inside = (i >= lo) & (i < hi) & (j >= lo) & (j < hi) & (k >= lo) & (k < hi)
    p["box_mask"] = inside.reshape(-1).copy()
    return p


def uneven_batch(count=64, seed=5, sizes=tuple(range(16, 97, 8)), orders=(4, 6, 8, 10, 12),
                 max_groups=8):
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        n = int(rng.choice(sizes))
        order = int(rng.choice(orders))
        groups = int(rng.integers(1, max_groups + 1))
        solver = "ann" if rng.uniform() < 0.5 else "ge"
        mseed = int(rng.integers(0, 2 ** 31 - 1))
        st, ss = blocky_materials((n, n, n), groups, mseed)
        p = problem((n, n, n), (1.0, 1.0, 1.0), order, groups, st, ss, np.ones((groups, n ** 3)),
                    np.zeros(6), f"batch{b}_{n}^3_S{order}_G{groups}_{solver}")
        p["solver"] = solver
        probs.append(p)
    return probs


def random_problem(n, order, groups, seed, length=(1.0, 1.0, 1.0), c_max=0.0, inflow=True,
                   sigma_range=(0.5, 5.0)):
    """Small random problem for parity tests: per-cell sigma_t ~ U[sigma_range],
    sigma_s = c sigma_t with c ~ U[0, c_max], q ~ U[0, 1], inflow ~ U[0, 1]."""
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in n)
    ncell = _ncell(n)
    st = rng.uniform(*sigma_range, size=(groups, ncell))
    ss = rng.uniform(0.0, c_max, size=(groups, ncell)) * st if c_max > 0 else np.zeros_like(st)
    q = rng.uniform(0.0, 1.0, size=(groups, ncell))
    inc = rng.uniform(0.0, 1.0, size=6) if inflow else np.zeros(6)
    return problem(n, length, order, groups, st, ss, q, inc,
                   f"random_{n[0]}x{n[1]}x{n[2]}_S{order}_G{groups}_seed{seed}")


def anisotropic_orders(sigma_s, L, seed, ratios=(0.5, 0.25, 0.12)):
    """Legendre moments of orders 1..L of the scattering cross section
    [L, G, ncell]: sigma_{s,n} = r_n u sigma_s with u ~ U[0.8, 1] per cell
    (a forward-peaked kernel, |sigma_{s,n}| < sigma_s)."""
    rng = np.random.default_rng(seed)
    ss = np.asarray(sigma_s, np.float64)
    return np.stack([ratios[n] * rng.uniform(0.8, 1.0, size=ss.shape) * ss for n in range(L)])


def multigroup_orders(sigma_s, L, seed, up=0.05, ratios=(0.5, 0.25, 0.12)):
    """Group-to-group scattering moments of orders 0..L [L+1, G, G, ncell]
    (from g' into g at [n, g', g]): order 0 spreads sigma_s[g'] over the
    destination groups, in-group and downscatter with U[0, 1] weights and
    upscatter damped by `up`, normalised so that the total out of g' is
    sigma_s[g']; order n >= 1 is r_n u times order 0 with u ~ U[0.8, 1]
    per entry (forward-peaked)."""
    rng = np.random.default_rng(seed)
    ss = np.asarray(sigma_s, np.float64)
    G = ss.shape[0]
    f = rng.uniform(0.0, 1.0, (G, G) + ss.shape[1:])
    for g2 in range(G):
        f[g2, :g2] *= up
    m0 = f / f.sum(axis=1, keepdims=True) * ss[:, None]
    out = [m0] + [ratios[n] * rng.uniform(0.8, 1.0, m0.shape) * m0 for n in range(L)]
    return np.stack(out)


def random_nodal(shape_cells, groups, seed, lo=0.0, hi=1.0):
    """Random nodal field [G, ncell, 8] ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(groups, int(shape_cells), 8))
