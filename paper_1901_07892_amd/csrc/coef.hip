// Coefficient step: face densities and cell viscosities from level sets.
//
// The material fields the Stokes solve takes are set from two signed-distance
// level sets (Sec. 4.1): phi for the liquid/gas interface (liquid where
// phi < 0) and, for each immersed solid, psi (solid where psi < 0).  A smoothed
// Heaviside of half-width eps = n_cells * hx (eq_heaviside) turns each into a
// volume fraction; the property of the flowing phase follows from phi
// (eq_ls_flow) and each solid then overrides it where its psi is negative
// (eq_ls_solid), several solids being applied in turn.  Viscosity is set at
// cell centres from the cell level sets; density on each face from the level
// sets averaged onto that face (Sec. 4.2.2), an interior face taking the mean
// of its two cells and a boundary face the one cell it touches.  The flow-only
// face density (no solid) that the well-balanced gravity force uses (Sec. 5)
// comes out of the same pass.
//
// One HBM-bound pass: each thread owns one (i, j) point of the
// (Nx+1) x (Ny+1) index plane and marches over a chunk of z planes, keeping
// the level sets of the plane below in registers and loading the next plane
// one step ahead; the x- and y-neighbours are the neighbouring threads' loads
// and come from cache.  Per point it writes
// the viscosity of cell (i, j, k), the x-face i, the y-face j and the z-face k
// that exist there, directly in the caller's C-order layouts.
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace {

constexpr int kCoefBlock = 256;
constexpr int kCoefPlanes = 8;    // z planes per block

struct CoefArgs {
    int nx, ny, nz, dim;
    double eps;
    double rho_l, rho_g, mu_l, mu_g;
    const double *psi[STOKES_MAX_SOLIDS];
    double rho_s[STOKES_MAX_SOLIDS], mu_s[STOKES_MAX_SOLIDS];
};

__device__ inline double smoothed_heaviside(double x, double eps) {
    if (x < -eps) return 0.0;
    if (x > eps) return 1.0;
    const double t = x / eps;
    return 0.5 * (1.0 + t + sinpi(t) * (1.0 / M_PI));   // sinpi(t) = sin(pi t), |t| <= 1
}

// Property at a point from the averaged liquid/gas level set f and the solids'
// averaged level sets s[0..NS).
template <int NS>
__device__ inline double material(double zl, double zg, const double *zs, double f, const double *s, double eps,
                                  double &flow) {
    double z = zl + (zg - zl) * smoothed_heaviside(f, eps);
    flow = z;
#pragma unroll
    for (int q = 0; q < NS; ++q) z = zs[q] + (z - zs[q]) * smoothed_heaviside(s[q], eps);
    return z;
}

// Outputs are written once and consumed by a later call (the solver's setup),
// so they are stored with the non-temporal hint.
__device__ inline void put(double *p, double v) { __builtin_nontemporal_store(v, p); }

template <int NS>
__global__ void __launch_bounds__(kCoefBlock) k_coefficients(CoefArgs a, const double *__restrict__ phi,
        double *__restrict__ rx, double *__restrict__ ry, double *__restrict__ rz, double *__restrict__ mu,
        double *__restrict__ fx, double *__restrict__ fy, double *__restrict__ fz) {
    const int px = a.nx + 1, py = a.ny + 1;
    const int p = blockIdx.x * kCoefBlock + threadIdx.x;
    if (p >= px * py) return;
    const int i = p % px, j = p / px;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ci = min(i, nx - 1), cj = min(j, ny - 1), iw = max(i - 1, 0), js = max(j - 1, 0);
    const int kend = a.dim == 3 ? nz + 1 : 1;      // z-face index runs to nz; 2D: one plane
    const int k0 = blockIdx.y * kCoefPlanes, k1 = min(k0 + kCoefPlanes, kend);
    const long long plane = (long long)nx * ny;
    // level sets of the cell below (k - 1, clamped) for the z-face average
    const long long rowc = ci + (long long)nx * cj;
    double fb, sb[NS > 0 ? NS : 1];
    {
        const long long o = rowc + plane * max(min(k0 - 1, nz - 1), 0);
        fb = phi[o];
#pragma unroll
        for (int q = 0; q < NS; ++q) sb[q] = a.psi[q][o];
    }
    // own, west and south level sets of the next plane, loaded one plane ahead so
    // that their latency overlaps the current plane's arithmetic and stores
    const long long roww = iw + (long long)nx * cj, rows = ci + (long long)nx * js;
    double nfc, nfw, nfs, nsc[NS > 0 ? NS : 1], nsw[NS > 0 ? NS : 1], nss[NS > 0 ? NS : 1];
    {
        const long long pk = plane * min(k0, nz - 1);
        nfc = phi[rowc + pk]; nfw = phi[roww + pk]; nfs = phi[rows + pk];
#pragma unroll
        for (int q = 0; q < NS; ++q) { nsc[q] = a.psi[q][rowc + pk]; nsw[q] = a.psi[q][roww + pk]; nss[q] = a.psi[q][rows + pk]; }
    }
    for (int k = k0; k < k1; ++k) {
        const double fc = nfc, fw = nfw, fs = nfs;
        double sc[NS > 0 ? NS : 1], sw[NS > 0 ? NS : 1], ss[NS > 0 ? NS : 1];
#pragma unroll
        for (int q = 0; q < NS; ++q) { sc[q] = nsc[q]; sw[q] = nsw[q]; ss[q] = nss[q]; }
        if (k + 1 < k1) {
            const long long pk = plane * min(k + 1, nz - 1);
            nfc = phi[rowc + pk]; nfw = phi[roww + pk]; nfs = phi[rows + pk];
#pragma unroll
            for (int q = 0; q < NS; ++q) { nsc[q] = a.psi[q][rowc + pk]; nsw[q] = a.psi[q][roww + pk]; nss[q] = a.psi[q][rows + pk]; }
        }
        if (k == 0) {                         // the plane below the first is the first (mirror)
            fb = fc;
#pragma unroll
            for (int q = 0; q < NS; ++q) sb[q] = sc[q];
        }
        const bool in_z = k < nz;
        double t[NS > 0 ? NS : 1], fl;
        if (in_z && i < nx && j < ny)
            put(mu + i + (long long)nx * j + plane * k, material<NS>(a.mu_l, a.mu_g, a.mu_s, fc, sc, a.eps, fl));
        if (in_z && j < ny) {                 // x-face i (i = 0 and nx take their one cell)
#pragma unroll
            for (int q = 0; q < NS; ++q) t[q] = 0.5 * (sw[q] + sc[q]);
            const long long o = i + (long long)px * (j + (long long)ny * k);
            put(rx + o, material<NS>(a.rho_l, a.rho_g, a.rho_s, 0.5 * (fw + fc), t, a.eps, fl));
            if (fx) put(fx + o, fl);
        }
        if (in_z && i < nx) {                 // y-face j
#pragma unroll
            for (int q = 0; q < NS; ++q) t[q] = 0.5 * (ss[q] + sc[q]);
            const long long o = i + (long long)nx * (j + (long long)py * k);
            put(ry + o, material<NS>(a.rho_l, a.rho_g, a.rho_s, 0.5 * (fs + fc), t, a.eps, fl));
            if (fy) put(fy + o, fl);
        }
        if (a.dim == 3 && i < nx && j < ny) { // z-face k (k = 0 and nz take their one cell)
#pragma unroll
            for (int q = 0; q < NS; ++q) t[q] = 0.5 * (sb[q] + sc[q]);
            const long long o = i + (long long)nx * j + plane * k;
            put(rz + o, material<NS>(a.rho_l, a.rho_g, a.rho_s, 0.5 * (fb + fc), t, a.eps, fl));
            if (fz) put(fz + o, fl);
        }
        fb = fc;
#pragma unroll
        for (int q = 0; q < NS; ++q) sb[q] = sc[q];
    }
}

template <int NS>
void launch(dim3 g, hipStream_t s, const CoefArgs &a, const double *phi, double *const r[3], double *mu,
            double *const f[3]) {
    k_coefficients<NS><<<g, kCoefBlock, 0, s>>>(a, phi, r[0], r[1], r[2], mu, f[0], f[1], f[2]);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

}  // namespace

extern "C" stokes_status stokes_coefficients(const stokes_grid *grid, const stokes_fluids *fluids,
        const double *phi, int n_solids, const double *const *psi, const double *rho_solid,
        const double *mu_solid, double *const rho_face[3], double *mu_cell, double *const rho_flow_face[3],
        void *stream) {
    if (!grid || !fluids || !phi || !rho_face || !mu_cell) return STOKES_EINVAL;
    const int dim = grid->dim;
    if (dim != 2 && dim != 3) return STOKES_EINVAL;
    for (int a = 0; a < dim; ++a) {
        if (grid->periodic[a]) return STOKES_EINVAL;     // walls only (mirrored out-of-domain cells)
        if (grid->n[a] < 1) return STOKES_ESHAPE;
        if (!finite_pos(grid->h[a])) return STOKES_EINVAL;
    }
    const long long nz = dim == 3 ? grid->n[2] : 1;
    // point count in double: a product of three 32-bit extents can exceed 64 bits
    if (((double)grid->n[0] + 1) * ((double)grid->n[1] + 1) * ((double)nz + 1) >= 2147483648.0) return STOKES_ESHAPE;
    if (!finite_pos(fluids->rho_liquid) || !finite_pos(fluids->rho_gas) || !finite_nonneg(fluids->mu_liquid) ||
        !finite_nonneg(fluids->mu_gas) || !finite_pos(fluids->n_cells))
        return STOKES_EINVAL;
    if (n_solids < 0 || n_solids > STOKES_MAX_SOLIDS) return STOKES_EINVAL;
    if (n_solids > 0 && (!psi || !rho_solid || !mu_solid)) return STOKES_EINVAL;
    CoefArgs a{};
    for (int q = 0; q < n_solids; ++q) {
        if (!psi[q] || !finite_pos(rho_solid[q]) || !finite_nonneg(mu_solid[q])) return STOKES_EINVAL;
        a.psi[q] = psi[q];
        a.rho_s[q] = rho_solid[q];
        a.mu_s[q] = mu_solid[q];
    }
    double *r[3] = {rho_face[0], rho_face[1], dim == 3 ? rho_face[2] : nullptr};
    double *f[3] = {nullptr, nullptr, nullptr};
    for (int d = 0; d < dim; ++d)
        if (!r[d]) return STOKES_EINVAL;
    if (rho_flow_face) {
        for (int d = 0; d < dim; ++d) {
            f[d] = rho_flow_face[d];
            if (!f[d]) return STOKES_EINVAL;
        }
    }
    a.nx = grid->n[0];
    a.ny = grid->n[1];
    a.nz = (int)nz;
    a.dim = dim;
    a.eps = fluids->n_cells * grid->h[0];
    a.rho_l = fluids->rho_liquid;
    a.rho_g = fluids->rho_gas;
    a.mu_l = fluids->mu_liquid;
    a.mu_g = fluids->mu_gas;
    const long long pts = (long long)(a.nx + 1) * (a.ny + 1);
    const int kend = dim == 3 ? a.nz + 1 : 1;
    dim3 g((unsigned)((pts + kCoefBlock - 1) / kCoefBlock), (unsigned)((kend + kCoefPlanes - 1) / kCoefPlanes));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (n_solids) {
        case 0: launch<0>(g, s, a, phi, r, mu_cell, f); break;
        case 1: launch<1>(g, s, a, phi, r, mu_cell, f); break;
        case 2: launch<2>(g, s, a, phi, r, mu_cell, f); break;
        case 3: launch<3>(g, s, a, phi, r, mu_cell, f); break;
        case 4: launch<4>(g, s, a, phi, r, mu_cell, f); break;
        case 5: launch<5>(g, s, a, phi, r, mu_cell, f); break;
        case 6: launch<6>(g, s, a, phi, r, mu_cell, f); break;
        case 7: launch<7>(g, s, a, phi, r, mu_cell, f); break;
        default: launch<8>(g, s, a, phi, r, mu_cell, f); break;
    }
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}
