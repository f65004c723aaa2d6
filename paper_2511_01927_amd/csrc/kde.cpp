// KDE contour construction (paper Sec. 4.2 "Adaptive Contour Design for CI
// Solver", interval sparsity function G_k(t) and Alg. "Adaptive Contour
// Construction via KDE").  Host code: it works on at most a few thousand
// predicted eigenvalues.
//
// Readings of points the paper leaves open:
//  * I_0 = [min - eps, max + eps], eps = beta (max - min) (Sec. 4.2), or the
//    caller's target window when one is given;
//  * the split point is the minimiser of G_k over the midpoints between
//    consecutive predicted eigenvalues inside I_k (never an interval end,
//    where G_k also decays) that leave at least N_min predictions on each
//    side when such midpoints exist; ties go to the lowest G, then to the
//    point nearest the interval centre;
//  * an interval with N_k > N_max whose predictions are all equal is kept;
//  * merging: an interval with N_k < N_min joins the neighbour with the
//    smaller count (left on ties); a merged interval above N_max is split
//    again; at most 4 * #intervals merge steps;
//  * circle: centre (s + e)/2, radius (1 + alpha)(e - s)/2 (Sec. 4.2, with
//    the local inflation alpha), keep window [s, e).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gep_ci.h"

namespace gep {
void set_error(const std::string& msg);
}

namespace {

struct Iv {
    double s, e;
};

int count_in(const std::vector<double>& lam, double s, double e, bool last) {
    auto lo = std::lower_bound(lam.begin(), lam.end(), s);
    auto hi = last ? std::upper_bound(lam.begin(), lam.end(), e) : std::lower_bound(lam.begin(), lam.end(), e);
    return (int)(hi - lo);
}

// split point of [s, e] by the minimum of the sparsity function, or NaN.
// Candidates leave at least nmin predictions on each side when possible.
double kde_cut(const std::vector<double>& lam, double s, double e, bool last, double w, int nmin) {
    auto lo = std::lower_bound(lam.begin(), lam.end(), s);
    auto hi = last ? std::upper_bound(lam.begin(), lam.end(), e) : std::lower_bound(lam.begin(), lam.end(), e);
    const int n = (int)(hi - lo);
    bool balanced = false;
    for (int i = 0; i + 1 < n; ++i)
        if (*(lo + i + 1) > *(lo + i) && i + 1 >= nmin && n - i - 1 >= nmin) balanced = true;
    const double width = e - s;
    double best = NAN, bestg = INFINITY, bestd = INFINITY;
    const double mid = 0.5 * (s + e);
    for (int i = 0; i + 1 < n; ++i) {
        auto it = lo + i;
        if (!(*(it + 1) > *it)) continue;
        if (balanced && !(i + 1 >= nmin && n - i - 1 >= nmin)) continue;
        const double t = 0.5 * (*it + *(it + 1));
        double g = 0.0;
        for (auto jt = lo; jt < hi; ++jt) {
            const double d = (t - *jt) / width;
            g += std::exp(-w * d * d);
        }
        const double dc = std::fabs(t - mid);
        if (g < bestg || (g == bestg && dc < bestd)) {
            bestg = g;
            bestd = dc;
            best = t;
        }
    }
    return best;
}

void split_until(const std::vector<double>& lam, Iv iv, bool last_of_all, int nmax, double w,
                 int nmin, std::vector<Iv>& out) {
    std::vector<std::pair<Iv, bool>> todo{{iv, last_of_all}};
    while (!todo.empty()) {
        auto [cur, last] = todo.back();
        todo.pop_back();
        const int nk = count_in(lam, cur.s, cur.e, last);
        double t = NAN;
        if (nk > nmax) t = kde_cut(lam, cur.s, cur.e, last, w, nmin);
        if (nk <= nmax || !std::isfinite(t)) {
            out.push_back(cur);
            continue;
        }
        todo.push_back({{t, cur.e}, last});
        todo.push_back({{cur.s, t}, false});
    }
}

}  // namespace

extern "C" int gep_kde_contours(const double* lam_hat, int64_t m, int nmin, int nmax, double w,
                                double alpha, double beta, double window_lo, double window_hi,
                                gep_contour* out, int cap, int* count) {
    if (!count || (m > 0 && !lam_hat) || nmin < 0 || nmax < 1 || nmin > nmax || !(w > 0) ||
        alpha < 0 || beta < 0) {
        gep::set_error("bad KDE arguments");
        return GEP_EINVAL;
    }
    std::vector<double> lam(lam_hat, lam_hat + m);
    for (double x : lam)
        if (!std::isfinite(x)) {
            gep::set_error("non-finite predicted eigenvalue");
            return GEP_EINVAL;
        }
    std::sort(lam.begin(), lam.end());
    double s0, e0;
    if (std::isfinite(window_lo) && std::isfinite(window_hi) && window_lo < window_hi) {
        s0 = window_lo;
        e0 = window_hi;
    } else {
        if (m == 0) {
            *count = 0;
            return GEP_OK;
        }
        const double eps = beta * (lam.back() - lam.front());
        s0 = lam.front() - eps;
        e0 = lam.back() + eps;
        if (!(e0 > s0)) {
            const double pad = std::max(1e-12, 1e-8 * std::fabs(s0));
            s0 -= pad;
            e0 += pad;
        }
    }
    std::vector<Iv> ivs;
    split_until(lam, {s0, e0}, true, nmax, w, nmin, ivs);
    std::sort(ivs.begin(), ivs.end(), [](const Iv& a, const Iv& b) { return a.s < b.s; });
    // merge intervals with fewer than nmin predicted eigenvalues
    for (int guard = 0; guard < 4 * (int)ivs.size() + 8 && ivs.size() > 1; ++guard) {
        int bad = -1;
        for (size_t i = 0; i < ivs.size(); ++i)
            if (count_in(lam, ivs[i].s, ivs[i].e, i + 1 == ivs.size()) < nmin) {
                bad = (int)i;
                break;
            }
        if (bad < 0) break;
        const int nl = bad > 0 ? count_in(lam, ivs[bad - 1].s, ivs[bad - 1].e, false) : INT32_MAX;
        const int nr = bad + 1 < (int)ivs.size()
                           ? count_in(lam, ivs[bad + 1].s, ivs[bad + 1].e, bad + 2 == (int)ivs.size())
                           : INT32_MAX;
        const int a = (nl <= nr) ? bad - 1 : bad;   // merge ivs[a] and ivs[a + 1]
        Iv merged{ivs[a].s, ivs[a + 1].e};
        const bool last = a + 2 == (int)ivs.size();
        ivs.erase(ivs.begin() + a, ivs.begin() + a + 2);
        std::vector<Iv> parts;
        split_until(lam, merged, last, nmax, w, nmin, parts);
        std::sort(parts.begin(), parts.end(), [](const Iv& x, const Iv& y) { return x.s < y.s; });
        ivs.insert(ivs.begin() + a, parts.begin(), parts.end());
        if (parts.size() > 1) {
            // the merged interval had to be split again: stop if nothing changes
            bool any_small = false;
            for (size_t i = 0; i < ivs.size(); ++i)
                any_small |= count_in(lam, ivs[i].s, ivs[i].e, i + 1 == ivs.size()) < nmin;
            if (!any_small) break;
        }
    }
    *count = (int)ivs.size();
    if (!out) return GEP_OK;
    if (cap < (int)ivs.size()) {
        gep::set_error("contour buffer too small");
        return GEP_EINVAL;
    }
    for (size_t i = 0; i < ivs.size(); ++i) {
        const double s = ivs[i].s, e = ivs[i].e;
        out[i].center = 0.5 * (s + e);
        out[i].radius = (1.0 + alpha) * 0.5 * (e - s);
        out[i].keep_lo = s;
        out[i].keep_hi = e;
    }
    return GEP_OK;
}
