// lbm_post.cpp -- liquid components of a density field (aerosol detection).
//
// Sec. 3.2-3.3 of arXiv 2103.08301 track the droplets that break away from the
// plug and the wall films when the plug ruptures and report their mass.  A
// component is a 4- or 8-connected region of cells with rho > threshold; an
// aerosol is a component with no cell on a wall row.
//
// Labelling is union-find in one raster pass: each liquid cell is joined to
// its already-visited neighbours (left, below, and the two lower corners for
// 8-connectivity), then the periodic seams are joined.  Every union keeps the
// smaller index as the root, so a component's root is its first cell in raster
// order and a second raster pass meets the roots in increasing order.  That
// pass also accumulates the per-component sums (in raster order).
#include <cmath>
#include <cstdint>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

struct Dsu {
    std::vector<int64_t> parent;
    explicit Dsu(int64_t n) : parent((size_t)n, -1) {}
    int64_t find(int64_t a) {
        int64_t r = a;
        while (parent[(size_t)r] != r) r = parent[(size_t)r];
        while (parent[(size_t)a] != r) {  // path compression
            const int64_t next = parent[(size_t)a];
            parent[(size_t)a] = r;
            a = next;
        }
        return r;
    }
    void join(int64_t a, int64_t b) {
        a = find(a);
        b = find(b);
        if (a == b) return;
        if (a < b)
            parent[(size_t)b] = a;
        else
            parent[(size_t)a] = b;
    }
};

// Offset d, moved to the nearest periodic image (-n/2 <= d < n/2).
int64_t nearest(int64_t d, int64_t n, bool periodic) {
    if (!periodic) return d;
    d %= n;
    if (d < -(n / 2)) d += n;
    if (d >= n - n / 2) d -= n;
    return d;
}

double wrap_into(double v, int n) {
    double r = std::fmod(v, (double)n);
    return r < 0 ? r + n : r;
}

}  // namespace

lbm_status label_components(const double* rho, int nx, int ny, bool xper, bool yper, double threshold, double rho_g,
                            int connectivity, lbm_component* out, int64_t cap, int64_t* n_out,
                            lbm_aerosol_summary* summary) {
    if (!rho || nx < 1 || ny < 1 || (connectivity != 4 && connectivity != 8) || cap < 0 || (cap > 0 && !out) ||
        std::isnan(threshold))
        return LBM_EINVAL;
    const int64_t n = (int64_t)nx * ny;
    Dsu d(n);
    auto liquid = [&](int64_t i) { return rho[i] > threshold; };
    for (int64_t i = 0; i < n; ++i)
        if (liquid(i)) d.parent[(size_t)i] = i;
    auto link = [&](int64_t a, int x, int y) {  // join a with (x, y) if that is a liquid cell
        if (x < 0 || x >= nx) {
            if (!xper) return;
            x = (x + nx) % nx;
        }
        if (y < 0 || y >= ny) {
            if (!yper) return;
            y = (y + ny) % ny;
        }
        const int64_t b = (int64_t)y * nx + x;
        if (liquid(b)) d.join(a, b);
    };
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t a = (int64_t)y * nx + x;
            if (!liquid(a)) continue;
            if (x > 0) link(a, x - 1, y);
            if (y > 0) {
                link(a, x, y - 1);
                if (connectivity == 8) {
                    if (x > 0) link(a, x - 1, y - 1);
                    if (x + 1 < nx) link(a, x + 1, y - 1);
                }
            }
        }
    // periodic seams: the raster pass only looked at lower-index neighbours inside the grid
    if (xper)
        for (int y = 0; y < ny; ++y) {
            const int64_t a = (int64_t)y * nx + (nx - 1);
            if (!liquid(a)) continue;
            link(a, 0, y);
            if (connectivity == 8) {
                if (y > 0 || yper) link(a, 0, y - 1);
                if (y + 1 < ny || yper) link(a, 0, y + 1);
            }
        }
    if (yper)
        for (int x = 0; x < nx; ++x) {
            const int64_t a = (int64_t)(ny - 1) * nx + x;
            if (!liquid(a)) continue;
            link(a, x, 0);
            if (connectivity == 8) {
                if (x > 0 || xper) link(a, x - 1, 0);
                if (x + 1 < nx || xper) link(a, x + 1, 0);
            }
        }
    // second pass: roots appear in increasing order; sums in raster order
    std::vector<int64_t> slot((size_t)n, -1);
    struct Acc {
        int64_t first, cells = 0;
        bool wall = false;
        double mass = 0, excess = 0, sx = 0, sy = 0;
    };
    std::vector<Acc> comps;
    double liquid_mass = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!liquid(i)) continue;
        const int64_t r = d.find(i);
        if (slot[(size_t)r] < 0) {
            slot[(size_t)r] = (int64_t)comps.size();
            comps.push_back(Acc{});
            comps.back().first = r;
        }
        Acc& c = comps[(size_t)slot[(size_t)r]];
        const int x = (int)(i % nx), y = (int)(i / nx);
        const int x0 = (int)(r % nx), y0 = (int)(r / nx);
        c.cells += 1;
        c.mass += rho[i];
        c.excess += rho[i] - rho_g;
        c.sx += (double)nearest(x - x0, nx, xper);
        c.sy += (double)nearest(y - y0, ny, yper);
        if (!yper && (y == 0 || y == ny - 1)) c.wall = true;
        liquid_mass += rho[i];
    }
    lbm_aerosol_summary sum{};
    sum.threshold = threshold;
    sum.liquid_mass = liquid_mass;
    sum.components = (int64_t)comps.size();
    for (size_t k = 0; k < comps.size(); ++k) {
        const Acc& c = comps[k];
        lbm_component o{};
        o.first_cell = c.first;
        o.cells = (int32_t)c.cells;
        o.wall = c.wall ? 1 : 0;
        o.mass = c.mass;
        o.excess_mass = c.excess;
        const double x0 = (double)(c.first % nx), y0 = (double)(c.first / nx);
        o.cx = xper ? wrap_into(x0 + c.sx / (double)c.cells, nx) : x0 + c.sx / (double)c.cells;
        o.cy = yper ? wrap_into(y0 + c.sy / (double)c.cells, ny) : y0 + c.sy / (double)c.cells;
        if ((int64_t)k < cap) out[k] = o;
        if (!c.wall) {
            sum.aerosols += 1;
            sum.aerosol_cells += c.cells;
            sum.aerosol_mass += c.mass;
            sum.aerosol_excess_mass += c.excess;
        }
    }
    if (n_out) *n_out = sum.components;
    if (summary) *summary = sum;
    return LBM_OK;
}

}  // namespace lbm

extern "C" lbm_status lbm_components_field(const double* rho, int nx, int ny, int x_periodic, int y_periodic,
                                           double threshold, double rho_g, int connectivity, lbm_component* out,
                                           int64_t cap, int64_t* n_out, lbm_aerosol_summary* summary) {
    if ((x_periodic != 0 && x_periodic != 1) || (y_periodic != 0 && y_periodic != 1)) return LBM_EINVAL;
    return lbm::label_components(rho, nx, ny, x_periodic == 1, y_periodic == 1, threshold, rho_g, connectivity, out,
                                 cap, n_out, summary);
}
