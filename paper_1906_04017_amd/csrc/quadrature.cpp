// Level-symmetric LQ_N angular quadrature (host).
//
// The paper discretises angle with S_N directions and weights (Sec. 2,
// Eq. (T7)-(T8)) without naming the set; the level-symmetric family of the
// transport literature it cites is used.  Construction: direction cosines on
// N/2 levels with mu_i^2 = mu_1^2 + (i-1) * 2(1 - 3 mu_1^2)/(N - 2); octant
// points are the level triples whose indices sum to N/2 + 2; permutations of a
// triple share a weight; mu_1 and the class weights make the even moments of
// one direction cosine exact (orders 0, 4, 6, ..., 2(n_classes + 1)); the
// smallest admissible mu_1 is taken; the sphere total is 4 pi.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "common.hpp"

namespace dgsn {
namespace {

struct Octant {
    std::vector<std::array<int, 3>> pts;   // level indices (1-based)
    std::vector<int> cls;                  // weight class of each point
    int ncls = 0;
};

Octant octant_points(int order)
{
    Octant o;
    const int half = order / 2;
    std::map<std::array<int, 3>, int> class_of;
    for (int i = 1; i <= half; ++i)
        for (int j = 1; j <= half; ++j) {
            const int k = half + 2 - i - j;
            if (k < 1 || k > half) continue;
            std::array<int, 3> p{i, j, k};
            std::array<int, 3> key = p;
            std::sort(key.begin(), key.end());
            auto it = class_of.find(key);
            if (it == class_of.end()) it = class_of.emplace(key, (int)class_of.size()).first;
            o.pts.push_back(p);
        }
    // class ids in sorted-key order (deterministic, independent of visit order)
    int id = 0;
    for (auto &kv : class_of) kv.second = id++;
    o.ncls = id;
    for (auto &p : o.pts) {
        std::array<int, 3> key = p;
        std::sort(key.begin(), key.end());
        o.cls.push_back(class_of[key]);
    }
    return o;
}

std::vector<double> levels(double mu1, int order)
{
    const int half = order / 2;
    std::vector<double> mu(half);
    if (order == 2) {
        mu[0] = std::sqrt(1.0 / 3.0);
        return mu;
    }
    const double step = 2.0 * (1.0 - 3.0 * mu1 * mu1) / (order - 2);
    for (int i = 0; i < half; ++i) mu[i] = std::sqrt(mu1 * mu1 + i * step);
    return mu;
}

// Dense solve with partial pivoting; false if singular.
bool dense_solve(std::vector<double> A, std::vector<double> b, int n, std::vector<double> &x)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
        if (std::fabs(A[p * n + k]) < 1e-300) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
            std::swap(b[k], b[p]);
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    x.assign(n, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
        x[i] = s / A[i * n + i];
    }
    return true;
}

// sum over the points of class c of mu_x^(2k)
double class_moment(const Octant &o, const std::vector<double> &mu, int c, int k)
{
    double s = 0.0;
    for (size_t p = 0; p < o.pts.size(); ++p)
        if (o.cls[p] == c) s += std::pow(mu[o.pts[p][0] - 1], 2 * k);
    return s;
}

bool class_weights(const Octant &o, double mu1, int order, std::vector<double> &w)
{
    const std::vector<double> mu = levels(mu1, order);
    const int n = o.ncls;
    std::vector<double> A(n * n), b(n);
    for (int r = 0; r < n; ++r) {
        const int k = (r == 0) ? 0 : r + 1;   // moment orders 0, 2, 3, ..., n
        for (int c = 0; c < n; ++c) A[r * n + c] = class_moment(o, mu, c, k);
        b[r] = 1.0 / (2 * k + 1);
    }
    return dense_solve(A, b, n, w);
}

bool extra_residual(const Octant &o, double mu1, int order, double &res)
{
    std::vector<double> w;
    if (!class_weights(o, mu1, order, w)) return false;
    const std::vector<double> mu = levels(mu1, order);
    const int k = o.ncls + 1;
    double s = 0.0;
    for (int c = 0; c < o.ncls; ++c) s += w[c] * class_moment(o, mu, c, k);
    res = s - 1.0 / (2 * k + 1);
    return true;
}

}  // namespace

int level_symmetric(int order, std::vector<double> &omega, std::vector<double> &weight)
{
    if (order < 2 || order > 12 || (order & 1))
        return set_error(DGSN_EINVAL, "LQ_N order must be even and in 2..12 (got %d)", order);
    const Octant o = octant_points(order);
    std::vector<double> w(1, 1.0);
    double mu1 = std::sqrt(1.0 / 3.0);
    if (order > 2) {
        // scan for the first sign change of the extra-moment residual, then bisect
        const int nscan = 2000;
        const double lo_lim = 1e-3, hi_lim = 0.5;
        double a = lo_lim, fa = 0.0;
        bool have_a = extra_residual(o, a, order, fa), found = false;
        for (int s = 1; s <= nscan && !found; ++s) {
            const double bpt = lo_lim + (hi_lim - lo_lim) * s / nscan;
            double fb;
            if (!extra_residual(o, bpt, order, fb)) { have_a = false; continue; }
            if (have_a && fa * fb <= 0.0) {
                double lo = a, hi = bpt, flo = fa;
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    double fm;
                    extra_residual(o, mid, order, fm);
                    if (flo * fm <= 0.0) hi = mid;
                    else { lo = mid; flo = fm; }
                }
                mu1 = 0.5 * (lo + hi);
                found = true;
            }
            a = bpt; fa = fb; have_a = true;
        }
        if (!found) return set_error(DGSN_EUNSUPPORTED, "no admissible mu_1 for S%d", order);
        if (!class_weights(o, mu1, order, w))
            return set_error(DGSN_EUNSUPPORTED, "singular weight system for S%d", order);
    }
    const std::vector<double> mu = levels(mu1, order);
    const int per = (int)o.pts.size();
    omega.resize(8 * per * 3);
    weight.resize(8 * per);
    for (int oct = 0; oct < 8; ++oct)
        for (int p = 0; p < per; ++p) {
            const int d = oct * per + p;
            for (int a = 0; a < 3; ++a) {
                const double sgn = ((oct >> a) & 1) ? -1.0 : 1.0;
                omega[3 * d + a] = sgn * mu[o.pts[p][a] - 1];
            }
            weight[d] = w[o.cls[p]] * (M_PI / 2.0);
        }
    return DGSN_OK;
}

}  // namespace dgsn

namespace dgsn {

// Real orthonormal spherical harmonics through order 3 in Cartesian form:
// the normalised harmonic polynomials of degree n restricted to the unit
// sphere, ordered k = n^2 + n + m (m < 0: the sine-type harmonics).
void real_ylm(int L, const double om[3], double *Y)
{
    const double x = om[0], y = om[1], z = om[2];
    const double pi = 3.14159265358979323846;
    Y[0] = std::sqrt(1.0 / (4.0 * pi));
    if (L < 1) return;
    const double c1 = std::sqrt(3.0 / (4.0 * pi));
    Y[1] = c1 * y;
    Y[2] = c1 * z;
    Y[3] = c1 * x;
    if (L < 2) return;
    const double c2 = std::sqrt(15.0 / (4.0 * pi));
    Y[4] = c2 * x * y;
    Y[5] = c2 * y * z;
    Y[6] = std::sqrt(5.0 / (16.0 * pi)) * (3.0 * z * z - 1.0);
    Y[7] = c2 * x * z;
    Y[8] = std::sqrt(15.0 / (16.0 * pi)) * (x * x - y * y);
    if (L < 3) return;
    const double c33 = std::sqrt(35.0 / (32.0 * pi));
    const double c31 = std::sqrt(21.0 / (32.0 * pi));
    Y[9] = c33 * y * (3.0 * x * x - y * y);
    Y[10] = std::sqrt(105.0 / (4.0 * pi)) * x * y * z;
    Y[11] = c31 * y * (5.0 * z * z - 1.0);
    Y[12] = std::sqrt(7.0 / (16.0 * pi)) * z * (5.0 * z * z - 3.0);
    Y[13] = c31 * x * (5.0 * z * z - 1.0);
    Y[14] = std::sqrt(105.0 / (16.0 * pi)) * z * (x * x - y * y);
    Y[15] = c33 * x * (x * x - 3.0 * y * y);
}

}  // namespace dgsn
