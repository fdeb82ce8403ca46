// Explicit momentum right-hand side of one time step.
//
// Moving the explicit terms of the discrete momentum equations to the right
// (Sec. 4.2.2, eq_nc_discrete_momentum, and eq_c_discrete_momentum with the old
// density), with the viscous term split as theta (new) + (1 - theta) (old),
// gives on every interior face
//     f = (rho/dt) u^n + (1 - theta) L_mu u^n + rho_force g,
// L_mu u = div[mu (grad u + grad u^T)] the strain-rate operator of the solve
// (shear viscosity on cell edges = harmonic mean of the four cells around the
// edge, out-of-domain cells mirrored; no-slip walls: wall-normal velocity zero,
// tangential ghost = minus the interior value).  theta = 1/2 is the paper's
// Crank-Nicolson split; rho_force is the flow-only density for the
// well-balanced gravity force (Sec. 5).  The convective term is the caller's.
//
// Two kernels: in 3D, a z-marching one with the old velocity and viscosity in a
// three-plane LDS ring (k_explicit_rhs3_z, below); in 2D, one thread per point
// (i, j) of the (Nx+1)(Ny+1) index space, which holds the x-face i and the
// y-face j of cell (i, j), neighbours from cache (k_explicit_rhs2).  All arrays
// are the caller's C-order layouts.
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace {

constexpr int kRhsBlock = 256;

struct RhsArgs {
    int dim, nx, ny, nz;
    double ihx, ihy, ihz;
    double idt, expl;        // 1/dt, 1 - theta
    double g[3];
    const double *u, *v, *w, *mu;
    const double *rx, *ry, *rz;      // density of the mass term
    const double *fx, *fy, *fz;      // density of the gravity force (may be null)
};

struct Fields {
    const RhsArgs &a;
    __device__ int cx(int i) const { return min(max(i, 0), a.nx - 1); }
    __device__ int cy(int j) const { return min(max(j, 0), a.ny - 1); }
    __device__ int cz(int k) const { return min(max(k, 0), a.nz - 1); }
    __device__ double M(int i, int j, int k) const {        // cell viscosity, mirrored outside
        return a.mu[cx(i) + a.nx * (cy(j) + a.ny * cz(k))];
    }
    // harmonic mean of four viscosities, 4 / (1/p + 1/q + 1/r + 1/s), with one
    // division: 4 pq rs / ((p + q) rs + (r + s) pq); 0 if any of them is 0
    __device__ static double hm4(double p, double q, double r, double s) {
        const double pq = p * q, rs = r * s;
        const double num = pq * rs;
        return num == 0.0 ? 0.0 : 4.0 * num / ((p + q) * rs + (r + s) * pq);
    }
    __device__ double Mxy(int i, int j, int k) const {
        return hm4(M(i - 1, j - 1, k), M(i, j - 1, k), M(i - 1, j, k), M(i, j, k));
    }
    // velocity components with the wall rules: wall-normal entries read as 0,
    // tangential ghosts beyond a wall are minus the mirrored interior value
    __device__ double U(int i, int j, int k) const {
        if (i <= 0 || i >= a.nx) return 0.0;
        double s = 1.0;
        if (j < 0) { j = -1 - j; s = -s; } else if (j >= a.ny) { j = 2 * a.ny - 1 - j; s = -s; }
        if (a.dim == 3) { if (k < 0) { k = -1 - k; s = -s; } else if (k >= a.nz) { k = 2 * a.nz - 1 - k; s = -s; } }
        return s * a.u[i + (a.nx + 1) * (j + a.ny * k)];
    }
    __device__ double V(int i, int j, int k) const {
        if (j <= 0 || j >= a.ny) return 0.0;
        double s = 1.0;
        if (i < 0) { i = -1 - i; s = -s; } else if (i >= a.nx) { i = 2 * a.nx - 1 - i; s = -s; }
        if (a.dim == 3) { if (k < 0) { k = -1 - k; s = -s; } else if (k >= a.nz) { k = 2 * a.nz - 1 - k; s = -s; } }
        return s * a.v[i + a.nx * (j + (a.ny + 1) * k)];
    }
    __device__ double W(int i, int j, int k) const {
        if (a.dim != 3 || k <= 0 || k >= a.nz) return 0.0;
        double s = 1.0;
        if (i < 0) { i = -1 - i; s = -s; } else if (i >= a.nx) { i = 2 * a.nx - 1 - i; s = -s; }
        if (j < 0) { j = -1 - j; s = -s; } else if (j >= a.ny) { j = 2 * a.ny - 1 - j; s = -s; }
        return s * a.w[i + a.nx * (j + a.ny * k)];
    }
};

__global__ void __launch_bounds__(kRhsBlock) k_explicit_rhs2(RhsArgs a, double *__restrict__ ox,
                                                             double *__restrict__ oy) {
    const int px = a.nx + 1, py = a.ny + 1;
    const int p = blockIdx.x * kRhsBlock + threadIdx.x;
    if (p >= px * py) return;
    const int i = p % px, j = p / px;
    const Fields F{a};
    const double hx = a.ihx, hy = a.ihy;
    // x-face i of row j
    if (j < a.ny) {
        double r = 0.0;
        if (i > 0 && i < a.nx) {
            const double u0 = F.U(i, j, 0);
            double L = 2.0 * hx * hx * (F.M(i, j, 0) * (F.U(i + 1, j, 0) - u0) - F.M(i - 1, j, 0) * (u0 - F.U(i - 1, j, 0)));
            L += hy * (F.Mxy(i, j + 1, 0) * ((F.U(i, j + 1, 0) - u0) * hy + (F.V(i, j + 1, 0) - F.V(i - 1, j + 1, 0)) * hx) -
                       F.Mxy(i, j, 0) * ((u0 - F.U(i, j - 1, 0)) * hy + (F.V(i, j, 0) - F.V(i - 1, j, 0)) * hx));
            const int o = i + px * j;
            r = a.rx[o] * a.idt * u0 + a.expl * L;
            if (a.fx) r += a.fx[o] * a.g[0];
        }
        ox[i + px * j] = r;
    }
    // y-face j of column i
    if (i < a.nx) {
        double r = 0.0;
        if (j > 0 && j < a.ny) {
            const double v0 = F.V(i, j, 0);
            double L = 2.0 * hy * hy * (F.M(i, j, 0) * (F.V(i, j + 1, 0) - v0) - F.M(i, j - 1, 0) * (v0 - F.V(i, j - 1, 0)));
            L += hx * (F.Mxy(i + 1, j, 0) * ((F.V(i + 1, j, 0) - v0) * hx + (F.U(i + 1, j, 0) - F.U(i + 1, j - 1, 0)) * hy) -
                       F.Mxy(i, j, 0) * ((v0 - F.V(i - 1, j, 0)) * hx + (F.U(i, j, 0) - F.U(i, j - 1, 0)) * hy));
            const int o = i + a.nx * j;
            r = a.ry[o] * a.idt * v0 + a.expl * L;
            if (a.fy) r += a.fy[o] * a.g[1];
        }
        oy[i + a.nx * j] = r;
    }
}

// 3D form: a block owns a TX x TY tile of cells and a chunk of z planes and
// marches in z with a three-plane LDS ring of u, v, w and mu on the tile plus a
// one-cell halo, filled with the wall rules already applied (wall-normal
// entries 0, tangential ghosts odd, viscosity mirrored), so that every plane is
// read from memory once per block and the stencil reads LDS without branches.
// Each thread writes the x-, y- and z-face rows of its cell (i, j, k); the
// wall-normal faces beyond the last cell of a row, column or stack (i = Nx,
// j = Ny, k = Nz) hold zero and are written by that last cell's thread.
constexpr int kZX = 64, kZY = 8, kZC = 16;
constexpr int kHX = kZX + 2, kHY = kZY + 2, kHP = kHX * kHY;

__global__ void __launch_bounds__(kZX *kZY) k_explicit_rhs3_z(RhsArgs a, double *__restrict__ ox,
                                                              double *__restrict__ oy, double *__restrict__ oz) {
    __shared__ double sU[3][kHP], sV[3][kHP], sW[3][kHP], sM[3][kHP];
    const Fields F{a};
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * kZX, j0 = blockIdx.y * kZY;
    const int k0 = blockIdx.z * kZC, k1 = min(k0 + kZC, a.nz);
    auto slot = [](int k) { return (k + 3) % 3; };                     // k >= -1
    auto load = [&](int k) {                                           // plane k, -1 <= k <= nz
        const int sl = slot(k);
        for (int t = tid; t < kHP; t += kZX * kZY) {
            const int gi = i0 - 1 + t % kHX, gj = j0 - 1 + t / kHX;
            double u = 0.0, v = 0.0, w = 0.0, m = 0.0;
            if (gi >= -1 && gi <= a.nx && gj >= -1 && gj <= a.ny) {
                u = F.U(gi, gj, k);
                v = F.V(gi, gj, k);
                w = F.W(gi, gj, k);
                m = F.M(gi, gj, k);
            }
            sU[sl][t] = u;
            sV[sl][t] = v;
            sW[sl][t] = w;
            sM[sl][t] = m;
        }
    };
    const int tx = tid % kZX, ty = tid / kZX;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < a.nx && j < a.ny;
    const int c = (ty + 1) * kHX + (tx + 1);
    const double hx = a.ihx, hy = a.ihy, hz = a.ihz;
    load(k0 - 1);
    load(k0);
    for (int k = k0; k < k1; ++k) {
        load(k + 1);
        __syncthreads();
        if (own) {
            const int sm = slot(k - 1), s0 = slot(k), sp = slot(k + 1);
            const int ss[3] = {sm, s0, sp};
            auto Us = [&](int di, int dj, int dk) { return sU[ss[dk + 1]][c + di + dj * kHX]; };
            auto Vs = [&](int di, int dj, int dk) { return sV[ss[dk + 1]][c + di + dj * kHX]; };
            auto Ws = [&](int di, int dj, int dk) { return sW[ss[dk + 1]][c + di + dj * kHX]; };
            auto Ms = [&](int di, int dj, int dk) { return sM[ss[dk + 1]][c + di + dj * kHX]; };
            auto Mxy = [&](int di, int dj) {
                return Fields::hm4(Ms(di - 1, dj - 1, 0), Ms(di, dj - 1, 0), Ms(di - 1, dj, 0), Ms(di, dj, 0));
            };
            auto Mxz = [&](int di, int dk) {
                return Fields::hm4(Ms(di - 1, 0, dk - 1), Ms(di, 0, dk - 1), Ms(di - 1, 0, dk), Ms(di, 0, dk));
            };
            auto Myz = [&](int dj, int dk) {
                return Fields::hm4(Ms(0, dj - 1, dk - 1), Ms(0, dj, dk - 1), Ms(0, dj - 1, dk), Ms(0, dj, dk));
            };
            // x-face i
            {
                double r = 0.0;
                if (i > 0) {
                    const double u0 = Us(0, 0, 0);
                    double L = 2.0 * hx * hx * (Ms(0, 0, 0) * (Us(1, 0, 0) - u0) - Ms(-1, 0, 0) * (u0 - Us(-1, 0, 0)));
                    L += hy * (Mxy(0, 1) * ((Us(0, 1, 0) - u0) * hy + (Vs(0, 1, 0) - Vs(-1, 1, 0)) * hx) -
                               Mxy(0, 0) * ((u0 - Us(0, -1, 0)) * hy + (Vs(0, 0, 0) - Vs(-1, 0, 0)) * hx));
                    L += hz * (Mxz(0, 1) * ((Us(0, 0, 1) - u0) * hz + (Ws(0, 0, 1) - Ws(-1, 0, 1)) * hx) -
                               Mxz(0, 0) * ((u0 - Us(0, 0, -1)) * hz + (Ws(0, 0, 0) - Ws(-1, 0, 0)) * hx));
                    const int o = i + (a.nx + 1) * (j + a.ny * k);
                    r = a.rx[o] * a.idt * u0 + a.expl * L;
                    if (a.fx) r += a.fx[o] * a.g[0];
                }
                const int o = i + (a.nx + 1) * (j + a.ny * k);
                ox[o] = r;
                if (i == a.nx - 1) ox[o + 1] = 0.0;            // wall face i = nx
            }
            // y-face j
            {
                double r = 0.0;
                if (j > 0) {
                    const double v0 = Vs(0, 0, 0);
                    double L = 2.0 * hy * hy * (Ms(0, 0, 0) * (Vs(0, 1, 0) - v0) - Ms(0, -1, 0) * (v0 - Vs(0, -1, 0)));
                    L += hx * (Mxy(1, 0) * ((Vs(1, 0, 0) - v0) * hx + (Us(1, 0, 0) - Us(1, -1, 0)) * hy) -
                               Mxy(0, 0) * ((v0 - Vs(-1, 0, 0)) * hx + (Us(0, 0, 0) - Us(0, -1, 0)) * hy));
                    L += hz * (Myz(0, 1) * ((Vs(0, 0, 1) - v0) * hz + (Ws(0, 0, 1) - Ws(0, -1, 1)) * hy) -
                               Myz(0, 0) * ((v0 - Vs(0, 0, -1)) * hz + (Ws(0, 0, 0) - Ws(0, -1, 0)) * hy));
                    const int o = i + a.nx * (j + (a.ny + 1) * k);
                    r = a.ry[o] * a.idt * v0 + a.expl * L;
                    if (a.fy) r += a.fy[o] * a.g[1];
                }
                const int o = i + a.nx * (j + (a.ny + 1) * k);
                oy[o] = r;
                if (j == a.ny - 1) oy[o + a.nx] = 0.0;         // wall face j = ny
            }
            // z-face k
            {
                double r = 0.0;
                if (k > 0) {
                    const double w0 = Ws(0, 0, 0);
                    double L = 2.0 * hz * hz * (Ms(0, 0, 0) * (Ws(0, 0, 1) - w0) - Ms(0, 0, -1) * (w0 - Ws(0, 0, -1)));
                    L += hx * (Mxz(1, 0) * ((Ws(1, 0, 0) - w0) * hx + (Us(1, 0, 0) - Us(1, 0, -1)) * hz) -
                               Mxz(0, 0) * ((w0 - Ws(-1, 0, 0)) * hx + (Us(0, 0, 0) - Us(0, 0, -1)) * hz));
                    L += hy * (Myz(1, 0) * ((Ws(0, 1, 0) - w0) * hy + (Vs(0, 1, 0) - Vs(0, 1, -1)) * hz) -
                               Myz(0, 0) * ((w0 - Ws(0, -1, 0)) * hy + (Vs(0, 0, 0) - Vs(0, 0, -1)) * hz));
                    const int o = i + a.nx * (j + a.ny * k);
                    r = a.rz[o] * a.idt * w0 + a.expl * L;
                    if (a.fz) r += a.fz[o] * a.g[2];
                }
                const int o = i + a.nx * (j + a.ny * k);
                oz[o] = r;
                if (k == a.nz - 1) oz[o + a.nx * a.ny] = 0.0;  // wall face k = nz
            }
        }
        __syncthreads();
    }
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

extern "C" stokes_status stokes_explicit_rhs(const stokes_grid *grid, const double *const rho_face[3],
        const double *mu_cell, double dt, double theta, const double *const u_n[3],
        const double *const rho_force[3], const double gravity[3], double *const f[3], void *stream) {
    if (!grid || !rho_face || !mu_cell || !u_n || !f) return STOKES_EINVAL;
    const int dim = grid->dim;
    if (dim != 2 && dim != 3) return STOKES_EINVAL;
    for (int d = 0; d < dim; ++d) {
        if (grid->periodic[d]) return STOKES_EINVAL;     // walls only
        if (grid->n[d] < 2) return STOKES_ESHAPE;
        if (!finite_pos(grid->h[d])) return STOKES_EINVAL;
        if (!rho_face[d] || !u_n[d] || !f[d] || (rho_force && !rho_force[d])) return STOKES_EINVAL;
    }
    if (!finite_pos(dt) || !std::isfinite(theta) || theta < 0.0 || theta > 1.0) return STOKES_EINVAL;
    if (rho_force && (!gravity || !std::isfinite(gravity[0]) || !std::isfinite(gravity[1]) ||
                      (dim == 3 && !std::isfinite(gravity[2]))))
        return STOKES_EINVAL;
    const long long nz = dim == 3 ? grid->n[2] : 1;
    // point count in double: a product of three 32-bit extents can exceed 64 bits
    const double pts = ((double)grid->n[0] + 1) * ((double)grid->n[1] + 1) * (dim == 3 ? (double)nz + 1 : 1.0);
    if (pts >= (double)((1LL << 31) - kRhsBlock)) return STOKES_ESHAPE;   // 32-bit point and array indices
    RhsArgs a{};
    a.dim = dim;
    a.nx = grid->n[0];
    a.ny = grid->n[1];
    a.nz = (int)nz;
    a.ihx = 1.0 / grid->h[0];
    a.ihy = 1.0 / grid->h[1];
    a.ihz = dim == 3 ? 1.0 / grid->h[2] : 0.0;
    a.idt = 1.0 / dt;
    a.expl = 1.0 - theta;
    a.u = u_n[0];
    a.v = u_n[1];
    a.w = dim == 3 ? u_n[2] : nullptr;
    a.mu = mu_cell;
    a.rx = rho_face[0];
    a.ry = rho_face[1];
    a.rz = dim == 3 ? rho_face[2] : nullptr;
    if (rho_force) {
        a.fx = rho_force[0];
        a.fy = rho_force[1];
        a.fz = dim == 3 ? rho_force[2] : nullptr;
        for (int d = 0; d < 3; ++d) a.g[d] = d < dim ? gravity[d] : 0.0;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dim == 3) {
        const dim3 g((a.nx + kZX - 1) / kZX, (a.ny + kZY - 1) / kZY, (a.nz + kZC - 1) / kZC);
        k_explicit_rhs3_z<<<g, kZX * kZY, 0, s>>>(a, f[0], f[1], f[2]);
    } else {
        const unsigned blocks = (unsigned)((pts + kRhsBlock - 1) / kRhsBlock);
        k_explicit_rhs2<<<blocks, kRhsBlock, 0, s>>>(a, f[0], f[1]);
    }
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}
