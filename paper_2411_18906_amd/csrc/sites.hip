// Nearest-site assignment of structures from other codes (the analysis step of
// the application workflow, Sec. 2.3): a configuration relaxed or simulated
// elsewhere (LAMMPS, DFT) comes back as Cartesian positions and is read onto
// the FCC/BCC supercell so that its SRO can be evaluated (Sec. 4.3, Eq. 2) and
// used as a target.
//
// Positions are scaled per axis to half lattice units (u = x * 2 L / box),
// wrapped into the periodic box, and decoded to the nearest lattice point in
// the Cartesian metric: FCC points are the integer points with an even
// coordinate sum, so per-axis rounding is followed, when the sum is odd, by
// moving the one coordinate whose move to its second-nearest integer costs the
// least Cartesian distance; BCC points are the even points and the all-odd
// points, each rounded per axis, and the nearer of the two is taken.  One
// thread per atom claims its site with a compare-and-swap, so double
// occupancy is detected exactly; a second pass writes species and finds
// vacancies.
#include <hip/hip_runtime.h>

#include <cmath>

#include "geometry.h"
#include "sites.h"

namespace pyhea {

namespace {

__global__ void fill_i32_kernel(int32_t *__restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// wrap an integer coordinate into [0, m)
__device__ __forceinline__ int wrap_i(int v, int m) {
    v %= m;
    return v < 0 ? v + m : v;
}

__global__ void map_atoms_kernel(SiteMapDesc md, int64_t n, const double *__restrict__ xyz,
                                 const int8_t *__restrict__ types, int32_t *__restrict__ owner,
                                 int32_t *__restrict__ flags) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    double u[3], w[3];
    int r[3];
    for (int ax = 0; ax < 3; ++ax) {
        const double period = 2.0 * md.L[ax];
        double v = xyz[3 * a + ax] * md.scale[ax];   // half lattice units
        v -= period * floor(v / period);              // into [0, 2L)
        u[ax] = v;
        w[ax] = 1.0 / (md.scale[ax] * md.scale[ax]);   // squared Cartesian length of one half unit
    }
    double d2;
    if (md.lattice == PYHEA_FCC) {
        int sum = 0;
        for (int ax = 0; ax < 3; ++ax) {
            r[ax] = (int)rint(u[ax]);
            sum += r[ax];
        }
        if (sum & 1) {
            // move the coordinate whose second-nearest integer costs least: w (1 - 2e)
            int best = 0;
            double cost = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                const double e = fabs(u[ax] - r[ax]);
                const double c = w[ax] * (1.0 - 2.0 * e);
                if (ax == 0 || c < cost) {
                    cost = c;
                    best = ax;
                }
            }
            r[best] += u[best] >= r[best] ? 1 : -1;
        }
        d2 = 0.0;
        for (int ax = 0; ax < 3; ++ax) d2 += w[ax] * (u[ax] - r[ax]) * (u[ax] - r[ax]);
    } else {
        int re[3], ro[3];
        double de = 0.0, dodd = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            re[ax] = 2 * (int)rint(u[ax] * 0.5);
            ro[ax] = 2 * (int)rint((u[ax] - 1.0) * 0.5) + 1;
            de += w[ax] * (u[ax] - re[ax]) * (u[ax] - re[ax]);
            dodd += w[ax] * (u[ax] - ro[ax]) * (u[ax] - ro[ax]);
        }
        const bool even = de <= dodd;
        for (int ax = 0; ax < 3; ++ax) r[ax] = even ? re[ax] : ro[ax];
        d2 = even ? de : dodd;
    }
    if (!(d2 <= md.max_disp2)) {
        atomicOr(&flags[0], 1);
        return;
    }
    const int t = types[a];
    if (t < 0 || t >= md.M) {
        atomicOr(&flags[2], 1);
        return;
    }
    int c[3], par[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int v = wrap_i(r[ax], 2 * md.L[ax]);
        c[ax] = v >> 1;
        par[ax] = v & 1;
    }
    int b;
    if (md.lattice == PYHEA_FCC)   // basis (0,0,0), (1,1,0), (1,0,1), (0,1,1)
        b = par[2] == 0 ? (par[0] ? 1 : 0) : (par[0] ? 2 : 3);
    else
        b = par[0];
    const int64_t p = (((int64_t)c[2] * md.L[1] + c[1]) * md.L[0] + c[0]) * md.A + b;
    if (atomicCAS(&owner[p], -1, (int32_t)a) != -1) atomicOr(&flags[1], 1);
}

__global__ void scatter_species_kernel(int64_t N, const int32_t *__restrict__ owner, const int8_t *__restrict__ types,
                                       int8_t *__restrict__ species, int32_t *__restrict__ flags) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int32_t a = owner[p];
    if (a < 0) {
        atomicOr(&flags[3], 1);
        species[p] = 0;
        return;
    }
    species[p] = types[a];
}

}  // namespace

hipError_t launch_map_sites(const SiteMapDesc &md, int64_t n, const double *xyz, const int8_t *types,
                            int32_t *owner, int32_t *flags, int8_t *species, hipStream_t stream) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, stream, flags, (int64_t)4, 0);
    const int64_t N = md.N;
    const unsigned gfill = (unsigned)std::min<int64_t>((N + 255) / 256, 65535);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(gfill), dim3(256), 0, stream, owner, N, -1);
    if (n > 0)
        hipLaunchKernelGGL(map_atoms_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, md, n, xyz,
                           types, owner, flags);
    hipLaunchKernelGGL(scatter_species_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, N, owner,
                       types, species, flags);
    return hipGetLastError();
}

}  // namespace pyhea
