"""Brute-force dense global solves on tiny meshes (FP64, NumPy).

TEST INFRASTRUCTURE: part of the CPU oracle, used only by the tests.

The whole discrete problem -- every (direction, group, cell) block of the
DGFEM S_n system of Sec. 2 (Eq. (T10)-(T12) with full upwinding and
Eq. (TBC)), plus the isotropic scattering coupling -- is assembled as one dense
matrix and solved with numpy.linalg.solve.  No sweep ordering is involved.
The element matrices are built here from exact 1D integrals combined by
Kronecker products (a construction independent of the Gauss-quadrature build
of the C oracle):

  1D on [0, h]: mass  m = h [[1/3, 1/6], [1/6, 1/3]]
                deriv g[k][j] = int l_k' l_j = [[-1/2, -1/2], [1/2, 1/2]]
                traces e_lo = [[1, 0], [0, 0]], e_hi = [[0, 0], [0, 1]]
  3D (node = ix + 2 iy + 4 iz, x fastest): kron(z, kron(y, x)).
"""
import numpy as np


def kron3(ax, ay, az):
    return np.kron(az, np.kron(ay, ax))


def element_matrices_kron(h):
    m = [hh * np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]]) for hh in h]
    g = np.array([[-0.5, -0.5], [0.5, 0.5]])
    e = [np.array([[1.0, 0.0], [0.0, 0.0]]), np.array([[0.0, 0.0], [0.0, 1.0]])]
    M = kron3(m[0], m[1], m[2])
    G = np.stack([kron3(g, m[1], m[2]), kron3(m[0], g, m[2]), kron3(m[0], m[1], g)])
    # face masses: the axis factor is the trace, the other two are 1D masses
    Mf = []
    for axis in range(3):
        for side in range(2):
            f = [m[0], m[1], m[2]]
            f[axis] = e[side]
            Mf.append(kron3(*f))
    return M, G, np.stack(Mf)


def _cell_id(c, n):
    return c[0] + n[0] * (c[1] + n[1] * c[2])


def assemble(mesh, omega, weight, sigma_t, sigma_s, q, psi_inc, extra_src=None, sigma_gg=None,
             sigma_sn=None, sigma_sn_gg=None):
    """Dense (L - K) and right-hand side Q for unknowns psi[d][g][c][8].

    sigma_t, sigma_s, q: [G, ncell]; psi_inc [6]; extra_src [G, ncell, 8]
    optional nodal source (per steradian) added to q; sigma_gg [G, G, ncell]
    optional group-to-group scattering (from g' to g at [g', g]), which then
    replaces the in-group sigma_s; sigma_sn [L, G, ncell] optional in-group
    anisotropic Legendre moments of orders 1..L, coupling directions d and d'
    through the kernel of Eq. (T3), sum_n (2n+1)/(4 pi) sigma_{s,n}
    P_n(Omega_d . Omega_d') (Legendre polynomials of the scattering cosine,
    not the spherical harmonics of the sweep's moments); sigma_sn_gg
    [L, G, G, ncell] optional group-to-group anisotropic moments of orders
    1..L (from g' to g at [n-1, g', g]) in place of sigma_sn.  Returns (A, Q)."""
    nx, ny, nz, lx, ly, lz = mesh
    n = (nx, ny, nz)
    h = (lx / nx, ly / ny, lz / nz)
    M, G, Mf = element_matrices_kron(h)
    ncell = nx * ny * nz
    omega = np.asarray(omega, np.float64)
    nd = omega.shape[0]
    sigma_t = np.asarray(sigma_t, np.float64).reshape(-1, ncell)
    ng = sigma_t.shape[0]
    sigma_s = np.asarray(sigma_s, np.float64).reshape(ng, ncell)
    q = np.asarray(q, np.float64).reshape(ng, ncell)
    if sigma_gg is not None:
        sigma_gg = np.asarray(sigma_gg, np.float64).reshape(ng, ng, ncell)
    aniso = None
    if sigma_sn is not None or sigma_sn_gg is not None:
        if sigma_sn_gg is not None:
            sn_gg = np.asarray(sigma_sn_gg, np.float64).reshape(-1, ng, ng, ncell)
        else:
            # in-group: the matrix of each order is diagonal in the groups
            sn = np.asarray(sigma_sn, np.float64).reshape(-1, ng, ncell)
            sn_gg = np.zeros((sn.shape[0], ng, ng, ncell))
            for g in range(ng):
                sn_gg[:, g, g, :] = sn[:, g, :]
        cosines = np.clip(omega @ omega.T, -1.0, 1.0)
        # aniso[n-1][d][d'] = (2n+1)/(4 pi) P_n(Omega_d . Omega_d')
        aniso = np.stack([(2 * o + 1) / (4 * np.pi) *
                          np.polynomial.legendre.legval(cosines, [0.0] * o + [1.0])
                          for o in range(1, sn_gg.shape[0] + 1)])
    N = nd * ng * ncell * 8
    A = np.zeros((N, N))
    Q = np.zeros(N)

    def blk(d, g, c):
        return ((d * ng + g) * ncell + c) * 8

    cells = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    for d in range(nd):
        om = omega[d]
        for g in range(ng):
            for c in cells:
                ci = _cell_id(c, n)
                r = blk(d, g, ci)
                Ac = sigma_t[g, ci] * M - np.einsum("a,akj->kj", om, G)
                S = np.full(8, q[g, ci])
                if extra_src is not None:
                    S = S + np.asarray(extra_src, np.float64).reshape(ng, ncell, 8)[g, ci]
                Q[r:r + 8] += M @ S
                for f in range(6):
                    axis, side = divmod(f, 2)
                    on = om[axis] * (1.0 if side else -1.0)
                    if on > 0:
                        Ac = Ac + on * Mf[f]
                    elif on < 0:
                        nb = list(c)
                        nb[axis] += 1 if side else -1
                        if 0 <= nb[axis] < n[axis]:
                            nbi = _cell_id(nb, n)
                            # upwind trace: neighbour node with the axis bit flipped
                            P = np.zeros((8, 8))
                            for nn in range(8):
                                P[nn, nn ^ (1 << axis)] = 1.0
                            cb = blk(d, g, nbi)
                            A[r:r + 8, cb:cb + 8] -= (-on) * Mf[f] @ P
                        else:
                            Q[r:r + 8] += (-on) * Mf[f] @ np.full(8, psi_inc[f])
                A[r:r + 8, r:r + 8] += Ac
                # isotropic scattering: - sigma_s/(4 pi) M sum_d' w_d' psi_d' (from
                # every group g2 with the matrix, from g itself without)
                src_groups = [(g, sigma_s[g, ci])] if sigma_gg is None else \
                    [(g2, sigma_gg[g2, g, ci]) for g2 in range(ng)]
                for g2, sig in src_groups:
                    if sig == 0.0:
                        continue
                    for d2 in range(nd):
                        cb = blk(d2, g2, ci)
                        A[r:r + 8, cb:cb + 8] -= sig / (4 * np.pi) * weight[d2] * M
                if aniso is not None:
                    for g2 in range(ng):
                        for d2 in range(nd):
                            k = float(np.dot(sn_gg[:, g2, g, ci], aniso[:, d, d2]))
                            if k != 0.0:
                                cb = blk(d2, g2, ci)
                                A[r:r + 8, cb:cb + 8] -= k * weight[d2] * M
    return A, Q


def solve(mesh, omega, weight, sigma_t, sigma_s, q, psi_inc, extra_src=None, sigma_gg=None,
          sigma_sn=None, sigma_sn_gg=None):
    """Returns (psi [D,G,ncell,8], phi [G,ncell,8]) of the dense global system."""
    A, Q = assemble(mesh, omega, weight, sigma_t, sigma_s, q, psi_inc, extra_src, sigma_gg,
                    sigma_sn, sigma_sn_gg)
    x = np.linalg.solve(A, Q)
    nx, ny, nz = mesh[:3]
    ncell = nx * ny * nz
    nd = len(weight)
    ng = np.asarray(sigma_t).reshape(-1, ncell).shape[0]
    psi = x.reshape(nd, ng, ncell, 8)
    phi = np.einsum("d,dgcn->gcn", np.asarray(weight, np.float64), psi)
    return psi, phi


def adjoint_solve(mesh, omega, weight, sigma_t, sigma_s, gphi, sigma_gg=None, sigma_sn=None,
                  sigma_sn_gg=None):
    """Dense transpose solve (L - K)^T lambda = W^T g for a response with
    dJ/dphi = gphi [G, ncell, 8]; returns lambda [D, G, ncell, 8]."""
    nd = len(weight)
    ncell = mesh[0] * mesh[1] * mesh[2]
    ng = np.asarray(sigma_t).reshape(-1, ncell).shape[0]
    A, _ = assemble(mesh, omega, weight, sigma_t, sigma_s, np.zeros((ng, ncell)), np.zeros(6),
                    sigma_gg=sigma_gg, sigma_sn=sigma_sn, sigma_sn_gg=sigma_sn_gg)
    gphi = np.asarray(gphi, np.float64).reshape(ng, ncell, 8)
    r = np.concatenate([weight[d] * gphi.reshape(-1) for d in range(nd)])
    lam = np.linalg.solve(A.T, r)
    return lam.reshape(nd, ng, ncell, 8)
