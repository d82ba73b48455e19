// Lattice tables of the pyhea library (host side).
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace pyhea {

namespace {

// Squared shell radii in half-lattice units (a = 2): FCC a^2/2, a^2, 3a^2/2,
// 2a^2; BCC 3a^2/4, a^2, 2a^2, 11a^2/4.
const int kFccR2[kMaxShells] = {2, 4, 6, 8};
const int kBccR2[kMaxShells] = {3, 4, 8, 11};

bool on_lattice(int lattice, int x, int y, int z) {
    const int px = x & 1, py = y & 1, pz = z & 1;
    if (lattice == PYHEA_FCC) return ((px ^ py ^ pz) == 0);
    return px == py && py == pz;
}

int floor_div2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

}  // namespace

void basis_vector(int lattice, int b, int out[3]) {
    static const int fcc[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    static const int bcc[2][3] = {{0, 0, 0}, {1, 1, 1}};
    const int *v = lattice == PYHEA_FCC ? fcc[b] : bcc[b];
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
}

static int basis_of_parity(int lattice, int px, int py, int pz) {
    const int A = lattice == PYHEA_FCC ? 4 : 2;
    for (int b = 0; b < A; ++b) {
        int v[3];
        basis_vector(lattice, b, v);
        if (v[0] == px && v[1] == py && v[2] == pz) return b;
    }
    return -1;
}

void offset_target(const Geometry &g, int b, int t, int dc[3], int *b_to) {
    int v[3];
    basis_vector(g.lattice, b, v);
    int pos[3];
    for (int a = 0; a < 3; ++a) {
        pos[a] = v[a] + g.off[t][a];
        dc[a] = floor_div2(pos[a]);
    }
    *b_to = basis_of_parity(g.lattice, pos[0] & 1, pos[1] & 1, pos[2] & 1);
}

int32_t padded_delta(const Geometry &g, int b, int t) {
    int dc[3], bt;
    offset_target(g, b, t, dc, &bt);
    const int64_t d = ((int64_t)dc[2] * g.P[1] + dc[1]) * g.P[0] + dc[0];
    return (int32_t)(d * g.A + (bt - b));
}

namespace {
pyhea_status build_geometry_uncached(const pyhea_lattice *lat, Geometry *g, std::string *err);
}

// Geometries are a pure function of the descriptor: built ones are kept (up to
// 4096 distinct descriptors) so that calls with many chains of few shapes, and
// repeated calls, skip the shell and offset enumeration.
pyhea_status build_geometry(const pyhea_lattice *lat, Geometry *g, std::string *err) {
    using Key = std::tuple<int, int, int, int, int, int>;
    static std::mutex mu;
    static std::map<Key, Geometry> cache;
    if (lat) {
        const Key key{lat->lattice, lat->L[0], lat->L[1], lat->L[2], lat->n_species, lat->n_shells};
        {
            std::lock_guard<std::mutex> lock(mu);
            auto it = cache.find(key);
            if (it != cache.end()) {
                *g = it->second;
                return PYHEA_OK;
            }
        }
        const pyhea_status s = build_geometry_uncached(lat, g, err);
        if (s == PYHEA_OK) {
            std::lock_guard<std::mutex> lock(mu);
            if (cache.size() >= 4096) cache.clear();
            cache.emplace(key, *g);
        }
        return s;
    }
    return build_geometry_uncached(lat, g, err);
}

namespace {

pyhea_status build_geometry_uncached(const pyhea_lattice *lat, Geometry *g, std::string *err) {
    *g = Geometry();
    if (!lat) {
        *err = "lattice descriptor is NULL";
        return PYHEA_EINVAL;
    }
    if (lat->lattice != PYHEA_FCC && lat->lattice != PYHEA_BCC) {
        *err = "lattice must be PYHEA_FCC (0) or PYHEA_BCC (1)";
        return PYHEA_EINVAL;
    }
    if (lat->n_species < 2 || lat->n_species > kMaxSpecies) {
        *err = "n_species must be in [2, 8]";
        return PYHEA_EINVAL;
    }
    if (lat->n_shells < 1 || lat->n_shells > kMaxShells) {
        *err = "n_shells must be in [1, 4]";
        return PYHEA_EINVAL;
    }
    for (int a = 0; a < 3; ++a) {
        if (lat->L[a] < 1 || lat->L[a] > 511) {
            *err = "each L must be in [1, 511]";
            return PYHEA_EINVAL;
        }
    }
    g->lattice = lat->lattice;
    g->A = lat->lattice == PYHEA_FCC ? 4 : 2;
    g->lgA = lat->lattice == PYHEA_FCC ? 2 : 1;
    for (int a = 0; a < 3; ++a) g->L[a] = lat->L[a];
    g->M = lat->n_species;
    g->S = lat->n_shells;
    g->N = (int64_t)g->A * g->L[0] * g->L[1] * g->L[2];

    const int *r2 = lat->lattice == PYHEA_FCC ? kFccR2 : kBccR2;
    int n = 0, maxc = 0;
    for (int k = 0; k < g->S; ++k) {
        g->r2[k] = r2[k];
        g->zstart[k] = n;
        for (int x = -3; x <= 3; ++x)
            for (int y = -3; y <= 3; ++y)
                for (int z = -3; z <= 3; ++z) {
                    if (x * x + y * y + z * z != r2[k] || !on_lattice(g->lattice, x, y, z)) continue;
                    g->off[n][0] = (int8_t)x;
                    g->off[n][1] = (int8_t)y;
                    g->off[n][2] = (int8_t)z;
                    maxc = std::max(maxc, std::max(std::abs(x), std::max(std::abs(y), std::abs(z))));
                    ++n;
                }
        g->z[k] = n - g->zstart[k];
    }
    g->Z = n;
    g->zstart[g->S] = n;

    // an offset congruent to 0 modulo the box maps every site onto itself
    for (int t = 0; t < n; ++t) {
        bool self = true;
        for (int a = 0; a < 3; ++a) {
            const int m = 2 * g->L[a];
            if (((g->off[t][a] % m) + m) % m != 0) self = false;
        }
        if (self) {
            *err = "a shell offset maps a site onto itself: the cell is too small for n_shells";
            return PYHEA_EINVAL;
        }
    }
    const int64_t zmax = *std::max_element(g->z, g->z + g->S);
    if (g->N * zmax >= (int64_t(1) << 31)) {
        *err = "N_sites * z_max must be below 2^31";
        return PYHEA_EINVAL;
    }
    // the shortcut "partner multiplicity = [|min-image d|^2 == r2_k]" needs every
    // offset component to be shorter than half the box along its axis
    g->small_cell = 0;
    for (int a = 0; a < 3; ++a)
        if (g->L[a] <= maxc) g->small_cell = 1;

    int halo = 0;
    for (int b = 0; b < g->A; ++b)
        for (int t = 0; t < n; ++t) {
            int dc[3], bt;
            offset_target(*g, b, t, dc, &bt);
            for (int a = 0; a < 3; ++a) halo = std::max(halo, std::abs(dc[a]));
        }
    g->halo = std::max(halo, 1);
    for (int a = 0; a < 3; ++a) g->P[a] = g->L[a] + 2 * g->halo;
    g->Npad = (int64_t)g->A * g->P[0] * g->P[1] * g->P[2];
    return PYHEA_OK;
}

}  // namespace

void fill_chain_geometry(const Geometry &g, ChainDesc *d) {
    d->A = g.A;
    d->lgA = g.lgA;
    d->Lx = g.L[0];
    d->Ly = g.L[1];
    d->Lz = g.L[2];
    d->M = g.M;
    d->S = g.S;
    d->Z = g.Z;
    d->halo = g.halo;
    d->PX = g.P[0];
    d->PY = g.P[1];
    d->PZ = g.P[2];
    d->small_cell = g.small_cell;
    for (int k = 0; k < kMaxShells; ++k) {
        d->zk[k] = k < g.S ? g.z[k] : 0;
        d->r2[k] = k < g.S ? g.r2[k] : -1;
    }
    for (int k = 0; k <= kMaxShells; ++k) d->zstart[k] = k <= g.S ? g.zstart[k] : g.Z;
    d->N = (uint32_t)g.N;
    d->Npad = (uint32_t)g.Npad;
    d->inv_Lx = 1.0 / (double)g.L[0];
    d->inv_Ly = 1.0 / (double)g.L[1];
    std::memset(d->off, 0, sizeof(d->off));
    std::memset(d->dlin, 0, sizeof(d->dlin));
    std::memset(d->off_mod, 0, sizeof(d->off_mod));
    for (int t = 0; t < g.Z; ++t) {
        int shell = 0;
        while (t >= g.zstart[shell + 1]) ++shell;
        d->off[t][0] = g.off[t][0];
        d->off[t][1] = g.off[t][1];
        d->off[t][2] = g.off[t][2];
        d->off[t][3] = (int8_t)shell;
        int packed = 0;
        for (int a = 0; a < 3; ++a) {
            const int m = 2 * g.L[a];
            packed |= (((g.off[t][a] % m) + m) % m) << (10 * a);
        }
        d->off_mod[t] = packed;
        for (int b = 0; b < g.A; ++b) d->dlin[b][t] = padded_delta(g, b, t);
    }
}

int symmetric_target(const double *t, int S, int M) {
    for (int k = 0; k < S; ++k)
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < i; ++j) {
                const double a = t[(k * M + i) * M + j], b = t[(k * M + j) * M + i];
                if (std::memcmp(&a, &b, sizeof(double)) != 0) return 0;
            }
    return 1;
}

}  // namespace pyhea
