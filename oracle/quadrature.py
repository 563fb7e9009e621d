"""Level-symmetric LQ_N angular quadrature, FP64 (oracle side).

TEST INFRASTRUCTURE: part of the CPU oracle.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may use it; the product library has
its own, independently written construction.

The paper uses an S_N angular discretisation with directions Omega_d and
weights Delta Omega_d (Sec. 2, Eq. (T7)-(T8)) but does not name the family.
Level-symmetric sets are the standard choice of the transport text it cites for
the formulation (Lewis & Miller).  Construction:

* mu_i^2 = mu_1^2 + (i - 1) * 2 (1 - 3 mu_1^2) / (N - 2),  i = 1 .. N/2;
* the points of one octant are the triples (mu_i, mu_j, mu_k) with
  i + j + k = N/2 + 2;
* points that are permutations of each other share one weight;
* mu_1 and the n_w class weights satisfy the even-moment conditions
  sum_octant w mu_x^(2k) = 1/(2k+1) for k = 0, 2, 3, ..., n_w + 1 (k = 1
  follows from the permutation symmetry); the smallest admissible root mu_1 is
  taken;
* the weights are scaled so that the full sphere sums to 4 pi.

Directions are ordered octant-major, octant o = [Ox<0] + 2[Oy<0] + 4[Oz<0],
points inside an octant by (i, j, k) lexicographically.
"""
import itertools

import numpy as np


def _octant_points(N):
    n2 = N // 2
    return [t for t in itertools.product(range(1, n2 + 1), repeat=3) if sum(t) == n2 + 2]


def _levels(mu1, N):
    n2 = N // 2
    if N == 2:
        return np.array([np.sqrt(1.0 / 3.0)])
    d = 2.0 * (1.0 - 3.0 * mu1 * mu1) / (N - 2)
    return np.sqrt(mu1 * mu1 + d * np.arange(n2))


def _class_weights(mu1, N, pts, classes):
    """Solve the n_w linear moment conditions k = 0, 2, ..., n_w for the weights."""
    mu = _levels(mu1, N)
    nw = len(classes)
    ks = [0] + list(range(2, nw + 1))
    A = np.zeros((nw, nw))
    rhs = np.zeros(nw)
    for r, k in enumerate(ks):
        for c, cl in enumerate(classes):
            A[r, c] = sum(mu[p[0] - 1] ** (2 * k) for p in pts if tuple(sorted(p)) == cl)
        rhs[r] = 1.0 / (2 * k + 1)
    w = np.linalg.solve(A, rhs)
    return w, mu


def _extra_moment_residual(mu1, N, pts, classes):
    nw = len(classes)
    k = nw + 1
    w, mu = _class_weights(mu1, N, pts, classes)
    s = 0.0
    for c, cl in enumerate(classes):
        s += w[c] * sum(mu[p[0] - 1] ** (2 * k) for p in pts if tuple(sorted(p)) == cl)
    return s - 1.0 / (2 * k + 1)


def lq_mu1(N):
    """Smallest root mu_1 of the extra even-moment condition (N >= 4)."""
    pts = _octant_points(N)
    classes = sorted({tuple(sorted(p)) for p in pts})
    # Above ~0.5 the levels crowd together (all equal at 1/sqrt(3)) and the
    # weight system degenerates; every tabulated set has mu_1 < 0.36.
    grid = np.linspace(1e-3, 0.5, 2000)
    vals = [_extra_moment_residual(m, N, pts, classes) for m in grid]
    for a, b, fa, fb in zip(grid[:-1], grid[1:], vals[:-1], vals[1:]):
        if fa == 0.0:
            return a
        if fa * fb < 0.0:
            lo, hi = a, b
            flo = fa
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                fm = _extra_moment_residual(mid, N, pts, classes)
                if flo * fm <= 0.0:
                    hi = mid
                else:
                    lo, flo = mid, fm
            return 0.5 * (lo + hi)
    raise ValueError(f"no admissible mu_1 for S{N}")


def lq_n(N):
    """Return (omega [D,3], weight [D]) of the LQ_N set, sum(weight) = 4 pi."""
    if N < 2 or N % 2 or N > 12:
        # above S12 the even-moment conditions alone no longer fix the class
        # weights (the system becomes singular); no workload here needs them
        raise ValueError("LQ_N is built for even N in 2..12")
    pts = _octant_points(N)
    if N == 2:
        mu = _levels(0.0, 2)
        w_pt = np.array([1.0])
    else:
        classes = sorted({tuple(sorted(p)) for p in pts})
        mu1 = lq_mu1(N)
        w, mu = _class_weights(mu1, N, pts, classes)
        w_pt = np.array([w[classes.index(tuple(sorted(p)))] for p in pts])
    om = np.array([[mu[i - 1], mu[j - 1], mu[k - 1]] for (i, j, k) in pts])
    omegas, weights = [], []
    for o in range(8):
        sgn = np.array([-1.0 if (o >> a) & 1 else 1.0 for a in range(3)])
        omegas.append(om * sgn)
        weights.append(w_pt * (np.pi / 2.0))
    return np.concatenate(omegas), np.concatenate(weights)
