// Host-side construction of the multi-resolution partition (Sec. 1.2).
// Compiled with -ffp-contract=off so that midpoints and knot bars are the
// plain IEEE results of the expressions below; the knot-coincidence test
// compares observations with knots bit for bit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "../../include/mra.h"
#include "mra_internal.h"

namespace mra {

namespace {

int64_t ipow(int64_t b, int e) {
    int64_t v = 1;
    while (e-- > 0) v *= b;
    return v;
}

// Bar position p of nb bars over [lo, hi): offset*length in from lo, then
// equal steps of length*(1 - 2*offset)/(nb - 1) (Appendix A form).
double bar(double lo, double hi, int nb, double f, int p) {
    const double L = hi - lo;
    if (nb == 1) return lo + f * L;
    return (lo + f * L) + ((static_cast<double>(p) * L) * (1.0 - 2.0 * f)) / static_cast<double>(nb - 1);
}

struct Box {
    double xlo, xhi, ylo, yhi;
};

// Quadtree (J = 4): both sides halved, child index = [x >= mid] + 2 [y >= mid].
// Binary (J = 2): the longer side halved (x on a tie), child = [coord >= mid].
int which_child(const Box& b, int J, double px, double py) {
    const double mx = 0.5 * (b.xlo + b.xhi), my = 0.5 * (b.ylo + b.yhi);
    if (J == 4) return (px >= mx ? 1 : 0) + (py >= my ? 2 : 0);
    const bool sx = (b.xhi - b.xlo) >= (b.yhi - b.ylo);
    return sx ? (px >= mx ? 1 : 0) : (py >= my ? 1 : 0);
}

Box child(const Box& b, int J, int j) {
    const double mx = 0.5 * (b.xlo + b.xhi), my = 0.5 * (b.ylo + b.yhi);
    Box c = b;
    if (J == 4) {
        if (j & 1) c.xlo = mx; else c.xhi = mx;
        if (j & 2) c.ylo = my; else c.yhi = my;
        return c;
    }
    const bool sx = (b.xhi - b.xlo) >= (b.yhi - b.ylo);
    if (sx) { if (j) c.xlo = mx; else c.xhi = mx; }
    else    { if (j) c.ylo = my; else c.yhi = my; }
    return c;
}

}  // namespace

int build_host_tree(const double* x, const double* y, const double* z, int64_t n, int J, int r,
                    int M, double offset, uint32_t flags, const double* domain4, HostTree& t, std::string& err) {
    if (n < 0 || (J != 2 && J != 4) || r < 1 || M < 1 || M > 16) {
        err = "invalid n, J (2 or 4), r (>= 1) or M (1..16)";
        return MRA_EINVAL;
    }
    int nx = 1;
    while (static_cast<int64_t>(nx) * nx < r) ++nx;
    const int ny = r / nx;
    t.J = J; t.M = M; t.r = r; t.nx = nx; t.ny = ny; t.rhat = nx * ny;
    if (t.rhat > 64) {
        err = "r_hat > 64 is not supported (the kernel tiles hold at most 64 knots)";
        return MRA_EINVAL;
    }
    t.P = t.rhat <= 16 ? 16 : (t.rhat <= 32 ? 32 : 64);
    t.offset = offset > 0.0 ? offset : std::exp(1.0) / 100.0;
    t.n_in = n;
    // guard the region count (J^(M-1) leaves)
    if (static_cast<double>(M - 1) * std::log(static_cast<double>(J)) > std::log(4.0e7)) {
        err = "too many regions (J^(M-1) > 4e7)";
        return MRA_EINVAL;
    }
    t.nleaf = ipow(J, M - 1);
    t.lvl_start.assign(M + 1, 0);
    t.nreg = 0;
    for (int m = 0; m < M; ++m) { t.lvl_start[m] = t.nreg; t.nreg += ipow(J, m); }
    t.lvl_start[M] = t.nreg;

    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i])) {
            err = "non-finite location at index " + std::to_string(i);
            return MRA_EINVAL;
        }

    Box root;
    if (domain4) {
        root = {domain4[0], domain4[1], domain4[2], domain4[3]};
        if (!(root.xhi > root.xlo) || !(root.yhi > root.ylo)) {
            err = "domain4 must have xmax > xmin and ymax > ymin";
            return MRA_EINVAL;
        }
    } else {
        double xmin = std::numeric_limits<double>::infinity(), xmax = -xmin, ymin = xmin, ymax = -xmin;
        for (int64_t i = 0; i < n; ++i) {
            xmin = std::fmin(xmin, x[i]); xmax = std::fmax(xmax, x[i]);
            ymin = std::fmin(ymin, y[i]); ymax = std::fmax(ymax, y[i]);
        }
        if (n == 0) { xmin = ymin = 0.0; xmax = ymax = 1.0; }
        const double lx = xmax - xmin, ly = ymax - ymin;
        // top and right sides pushed out by one percent of the side (of 1.0 if degenerate)
        root = {xmin, xmax + 0.01 * (lx > 0.0 ? lx : 1.0), ymin, ymax + 0.01 * (ly > 0.0 ? ly : 1.0)};
    }
    t.box.assign(4 * t.nreg, 0.0);
    auto put = [&](int64_t g, const Box& b) {
        t.box[4 * g] = b.xlo; t.box[4 * g + 1] = b.xhi; t.box[4 * g + 2] = b.ylo; t.box[4 * g + 3] = b.yhi;
    };
    auto get = [&](int64_t g) { return Box{t.box[4 * g], t.box[4 * g + 1], t.box[4 * g + 2], t.box[4 * g + 3]}; };
    put(0, root);
    for (int m = 0; m + 1 < M; ++m)
        for (int64_t k = 0; k < ipow(J, m); ++k) {
            const Box b = get(t.lvl_start[m] + k);
            for (int j = 0; j < J; ++j) put(t.lvl_start[m + 1] + J * k + j, child(b, J, j));
        }

    // repeated locations: observations (with a value) sorted by location, then
    // input index; every later member of a run of equal locations is a repeat
    std::vector<char> rep(n, 0);
    if (flags & MRA_ELIM_DUPLICATES) {
        std::vector<int64_t> ord;
        ord.reserve(n);
        for (int64_t i = 0; i < n; ++i)
            if (!std::isnan(z[i])) ord.push_back(i);
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
            if (x[a] != x[b]) return x[a] < x[b];
            if (y[a] != y[b]) return y[a] < y[b];
            return a < b;
        });
        for (size_t s = 1; s < ord.size(); ++s)
            if (x[ord[s]] == x[ord[s - 1]] && y[ord[s]] == y[ord[s - 1]]) rep[ord[s]] = 1;
    }

    // leaf of every observation; drop NaN values, repeats and knot coincidences
    std::vector<int64_t> leaf(n, -1);
    std::vector<double> xb(nx), yb(ny);
    int64_t used = 0;
    t.n_nan = t.n_elim = t.n_dup = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (std::isnan(z[i])) { ++t.n_nan; continue; }
        if (x[i] < root.xlo || x[i] >= root.xhi || y[i] < root.ylo || y[i] >= root.yhi) {
            err = "observation " + std::to_string(i) + " lies outside the root region";
            return MRA_EDOMAIN;
        }
        if (rep[i]) { ++t.n_dup; continue; }
        int64_t k = 0;
        bool on_knot = false;
        for (int m = 0; m + 1 < M; ++m) {
            const Box b = get(t.lvl_start[m] + k);
            bool hx = false, hy = false;
            for (int p = 0; p < nx && !hx; ++p) hx = (x[i] == bar(b.xlo, b.xhi, nx, t.offset, p));
            for (int q = 0; q < ny && !hy; ++q) hy = (y[i] == bar(b.ylo, b.yhi, ny, t.offset, q));
            on_knot = on_knot || (hx && hy);
            k = J * k + which_child(b, J, x[i], y[i]);
        }
        if (on_knot) { ++t.n_elim; continue; }
        leaf[i] = k;
        ++used;
    }
    t.n_used = used;
    // stable grouping by leaf
    std::vector<int64_t> cnt(t.nleaf + 1, 0);
    for (int64_t i = 0; i < n; ++i) if (leaf[i] >= 0) ++cnt[leaf[i] + 1];
    for (int64_t k = 0; k < t.nleaf; ++k) cnt[k + 1] += cnt[k];
    t.x.resize(used); t.y.resize(used); t.z.resize(used); t.orig.resize(used);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i) {
        if (leaf[i] < 0) continue;
        const int64_t d = fill[leaf[i]]++;
        t.x[d] = x[i]; t.y[d] = y[i]; t.z[d] = z[i]; t.orig[d] = i;
    }
    // observation range of every region's subtree
    t.obs_lo.assign(t.nreg, 0);
    t.obs_hi.assign(t.nreg, 0);
    for (int m = 0; m < M; ++m) {
        const int64_t span = ipow(J, M - 1 - m);
        for (int64_t k = 0; k < ipow(J, m); ++k) {
            t.obs_lo[t.lvl_start[m] + k] = cnt[k * span];
            t.obs_hi[t.lvl_start[m] + k] = cnt[(k + 1) * span];
        }
    }
    return MRA_OK;
}

int locate_leaves(const HostTree& t, const double* x, const double* y, int64_t n, std::vector<int64_t>& leaf,
                  std::string& err) {
    leaf.assign(n, 0);
    const Box root{t.box[0], t.box[1], t.box[2], t.box[3]};
    for (int64_t i = 0; i < n; ++i) {
        if (!(x[i] >= root.xlo && x[i] < root.xhi && y[i] >= root.ylo && y[i] < root.yhi)) {
            err = "prediction location " + std::to_string(i) + " lies outside the root region";
            return MRA_EDOMAIN;
        }
        int64_t k = 0;
        for (int m = 0; m + 1 < t.M; ++m) {
            const int64_t g = t.lvl_start[m] + k;
            const Box b{t.box[4 * g], t.box[4 * g + 1], t.box[4 * g + 2], t.box[4 * g + 3]};
            k = t.J * k + which_child(b, t.J, x[i], y[i]);
        }
        leaf[i] = t.lvl_start[t.M - 1] + k;
    }
    return MRA_OK;
}

}  // namespace mra
