// Rigid-body constraint projection after the Stokes solve.
//
// The solve leaves a velocity u~ that ignores the rigidity of an immersed body.
// The correction (Sec. 4.2.5, eq_velocity_correction) is
//     u = u~ + S (U_b - J u~),
// with J the interpolation of face velocities onto the body's Lagrangian
// markers and S the spreading of marker values back onto the faces (Sec. 3.3),
// both through the four-point regularised delta function of Peskin (2002),
// delta_h(x) = prod_d phi(x_d/h_d)/h_d.  U_b = U_r + W_r x (X - X_com) is the
// rigid motion: given (prescribed motion, eq_prescribed_velocity) or obtained
// by redistributing the linear and angular momentum of J u~ over the markers
// (free body, eqs. eq_linear_conservation and eq_angular_conservation).  Near a
// no-slip wall the stencil points beyond it take the odd mirror image of the
// interior (the wall holds zero velocity) and wall-normal points on the wall
// hold zero; the spreading is the exact transpose of that interpolation, so
// S = J^* also near walls.
//
// GPU mapping: one thread per marker.  Kernel 1 gathers the 4^d stencil of
// each velocity component (cache-resident neighbourhoods) and reduces the
// momentum sums of the block deterministically (fixed tree, no atomics).  The
// host sums the block partials in block order and solves the 3x3 inertia
// system.  Kernel 2 scatters the correction with vector atomic adds (markers'
// stencils overlap).
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

// Sets the message stokes_last_error(NULL) returns in this thread (stokes.hip).
void stk_set_thread_error(const char *msg);

namespace {

constexpr int kRigidBlock = 256;
constexpr int kRigidMaxBlocks = 1024;
constexpr int kSums = 13;   // P (3), L (3), I (xx xy xz yy yz zz), markers outside the domain

struct RigidGrid {
    int dim;
    int n[3];
    double h[3];
    double L[3];            // domain lengths n * h
};

__device__ inline double peskin4(double r) {
    const double a = fabs(r);
    if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(fmax(1.0 + 4.0 * a - 4.0 * a * a, 0.0)));
    if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(fmax(-7.0 + 12.0 * a - 4.0 * a * a, 0.0)));
    return 0.0;
}

// The four stencil points of one axis for component c: mirrored array index,
// weight times the mirror sign (0 for a wall-normal point on the wall).
__device__ inline void axis_stencil(int c, int d, double x, double h, int n, int idx[4], double w[4]) {
    if (d == c) {                                // faces at i*h, i = 0..n (walls 0 and n)
        const double t = x / h;
        const int base = (int)floor(t) - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = base + q;
            double s = 1.0;
            int m = i;
            if (i < 0) { m = -i; s = -1.0; }
            else if (i > n) { m = 2 * n - i; s = -1.0; }
            else if (i == 0 || i == n) s = 0.0;
            if (m < 0 || m > n) { m = 0; s = 0.0; }      // unreachable for n >= 2 and 0 <= x <= n h
            idx[q] = m;
            w[q] = s * peskin4((double)i - t);
        }
    } else {                                     // cell centres at (j + 1/2) h, j = 0..n-1
        const double t = x / h - 0.5;
        const int base = (int)floor(t) - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = base + q;
            double s = 1.0;
            int m = j;
            if (j < 0) { m = -1 - j; s = -1.0; }
            else if (j >= n) { m = 2 * n - 1 - j; s = -1.0; }
            if (m < 0 || m > n - 1) { m = 0; s = 0.0; }  // unreachable for n >= 2 and 0 <= x <= n h
            idx[q] = m;
            w[q] = s * peskin4((double)j - t);
        }
    }
}

__device__ inline bool inside(const RigidGrid &g, const double *x) {
    bool ok = true;
    for (int d = 0; d < g.dim; ++d) ok = ok && (x[d] >= 0.0) && (x[d] <= g.L[d]);   // NaN fails
    return ok;
}

// Visit the 4^DIM stencil points of component c at marker position x:
// fn(array offset, weight) for every point whose weight is not zero.
template <int DIM, class Fn>
__device__ inline void for_stencil(const RigidGrid &g, int c, const double *x, Fn fn) {
    int ix[4], iy[4], iz[4] = {0, 0, 0, 0};
    double wx[4], wy[4], wz[4] = {1.0, 0.0, 0.0, 0.0};
    axis_stencil(c, 0, x[0], g.h[0], g.n[0], ix, wx);
    axis_stencil(c, 1, x[1], g.h[1], g.n[1], iy, wy);
    if (DIM == 3) axis_stencil(c, 2, x[2], g.h[2], g.n[2], iz, wz);
    const long long sx = g.n[0] + (c == 0), sy = g.n[1] + (c == 1);
    for (int a = 0; a < (DIM == 3 ? 4 : 1); ++a)
        for (int b = 0; b < 4; ++b) {
            const double wab = wz[a] * wy[b];
            const long long row = sx * (iy[b] + sy * (long long)iz[a]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double w = wx[e] * wab;
                if (w != 0.0) fn(ix[e] + row, w);
            }
        }
}

template <int DIM>
__global__ void __launch_bounds__(kRigidBlock) k_rigid_interp(RigidGrid g, long long nm,
        const double *__restrict__ X, double xc0, double xc1, double xc2, double dV,
        const double *__restrict__ u0, const double *__restrict__ u1, const double *__restrict__ u2,
        double *__restrict__ JU, double *__restrict__ partial) {
    __shared__ double red[kSums][kRigidBlock];
    double acc[kSums];
#pragma unroll
    for (int s = 0; s < kSums; ++s) acc[s] = 0.0;
    const double *uc[3] = {u0, u1, u2};
    const double xc[3] = {xc0, xc1, xc2};
    for (long long m = (long long)blockIdx.x * kRigidBlock + threadIdx.x; m < nm;
         m += (long long)gridDim.x * kRigidBlock) {
        double x[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < DIM; ++d) x[d] = X[m * DIM + d];
        double U[3] = {0.0, 0.0, 0.0};
        if (!inside(g, x)) {
            acc[12] += 1.0;
        } else {
            for (int c = 0; c < DIM; ++c) {
                const double *uu = uc[c];
                double s = 0.0;
                for_stencil<DIM>(g, c, x, [&](long long o, double w) { s += w * uu[o]; });
                U[c] = s;
            }
            double R[3] = {x[0] - xc[0], x[1] - xc[1], DIM == 3 ? x[2] - xc[2] : 0.0};
            acc[0] += U[0] * dV;
            acc[1] += U[1] * dV;
            acc[2] += U[2] * dV;
            acc[3] += (R[1] * U[2] - R[2] * U[1]) * dV;
            acc[4] += (R[2] * U[0] - R[0] * U[2]) * dV;
            acc[5] += (R[0] * U[1] - R[1] * U[0]) * dV;
            const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
            acc[6] += (rr - R[0] * R[0]) * dV;
            acc[7] += -R[0] * R[1] * dV;
            acc[8] += -R[0] * R[2] * dV;
            acc[9] += (rr - R[1] * R[1]) * dV;
            acc[10] += -R[1] * R[2] * dV;
            acc[11] += (rr - R[2] * R[2]) * dV;
        }
        for (int d = 0; d < DIM; ++d) JU[m * DIM + d] = U[d];
    }
#pragma unroll
    for (int s = 0; s < kSums; ++s) red[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int w = kRigidBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int s = 0; s < kSums; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kSums) partial[(long long)blockIdx.x * kSums + threadIdx.x] = red[threadIdx.x][0];
}

template <int DIM>
__global__ void __launch_bounds__(kRigidBlock) k_rigid_spread(RigidGrid g, long long nm,
        const double *__restrict__ X, const double *__restrict__ JU, double xc0, double xc1, double xc2,
        double ur0, double ur1, double ur2, double wr0, double wr1, double wr2, double scale,
        double *u0, double *u1, double *u2) {
    double *uc[3] = {u0, u1, u2};
    for (long long m = (long long)blockIdx.x * kRigidBlock + threadIdx.x; m < nm;
         m += (long long)gridDim.x * kRigidBlock) {
        double x[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < DIM; ++d) x[d] = X[m * DIM + d];
        const double R0 = x[0] - xc0, R1 = x[1] - xc1, R2 = DIM == 3 ? x[2] - xc2 : 0.0;
        double dU[3];
        if (DIM == 3) {
            dU[0] = ur0 + (wr1 * R2 - wr2 * R1) - JU[m * 3 + 0];
            dU[1] = ur1 + (wr2 * R0 - wr0 * R2) - JU[m * 3 + 1];
            dU[2] = ur2 + (wr0 * R1 - wr1 * R0) - JU[m * 3 + 2];
        } else {                                 // wr0: rotation rate about z
            dU[0] = ur0 - wr0 * R1 - JU[m * 2 + 0];
            dU[1] = ur1 + wr0 * R0 - JU[m * 2 + 1];
            dU[2] = 0.0;
        }
        for (int c = 0; c < DIM; ++c) {
            double *uu = uc[c];
            const double f = dU[c] * scale;
            for_stencil<DIM>(g, c, x, [&](long long o, double w) { atomicAdd(uu + o, w * f); });
        }
    }
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Host copy of the block partials (per thread, so that no call allocates).
thread_local double t_partials[kRigidMaxBlocks * kSums];

// Scratch of the allocation-free entry point: the interpolated marker
// velocities (n_markers x dim) and the block partials, in a file-scope device
// array that every GPU the library runs on holds until the process ends.  Host
// code never uses the array's name as an address: each device's address comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr long long kScratchMarkers = STOKES_RIGID_NOALLOC_MAX_MARKERS;
constexpr size_t kScratchDoubles = (size_t)kScratchMarkers * 3 + (size_t)kRigidMaxBlocks * kSums;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_of_current_device(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Argument checks shared by both entry points; fills g.  STOKES_OK means "go on".
stokes_status rigid_check(const stokes_grid *grid, double *const u[3], long long n_markers, double dV,
                          int free_body, const stokes_body *body, RigidGrid &g) {
    if (!grid || !u || !body || n_markers < 0) return STOKES_EINVAL;
    const int dim = grid->dim;
    if (dim != 2 && dim != 3) return STOKES_EINVAL;
    for (int d = 0; d < dim; ++d)
        if (grid->periodic[d]) return STOKES_EINVAL;     // walls only (mirrored stencils)
    g = RigidGrid{};
    g.dim = dim;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = d < dim ? grid->n[d] : 1;
        g.h[d] = d < dim ? grid->h[d] : 1.0;
    }
    for (int d = 0; d < dim; ++d) {
        if (g.n[d] < 2) return STOKES_ESHAPE;
        if (!finite_pos(g.h[d])) return STOKES_EINVAL;
        g.L[d] = g.n[d] * g.h[d];
        if (!u[d]) return STOKES_EINVAL;
    }
    // point count in double: a product of three 32-bit extents can exceed 64 bits
    if (((double)g.n[0] + 1) * ((double)g.n[1] + 1) * (dim == 3 ? (double)g.n[2] + 1 : 1.0) >= 1099511627776.0)
        return STOKES_ESHAPE;
    if (!finite_pos(dV) || (free_body != 0 && free_body != 1)) return STOKES_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(body->x_com[d]) || !std::isfinite(body->u_r[d]) || !std::isfinite(body->w_r[d]))
            return STOKES_EINVAL;
    if (n_markers == 0 && free_body) return STOKES_EINVAL;   // a free body needs markers
    return STOKES_OK;
}

// The projection itself, with its scratch given: JU (n_markers x dim) and the
// block partials (at most kRigidMaxBlocks x kSums) after it.  Neither needs
// clearing: every entry is written before it is read.
stokes_status rigid_impl(const RigidGrid &g, double *const u[3], long long n_markers, const double *X, double dV,
                         int free_body, stokes_body *body, double *JU, hipStream_t s) {
    const int dim = g.dim;
    const int blocks = (int)std::min<long long>((n_markers + kRigidBlock - 1) / kRigidBlock, kRigidMaxBlocks);
    double *partial = JU + n_markers * dim;
    const double *x = body->x_com;
    if (dim == 3)
        k_rigid_interp<3><<<blocks, kRigidBlock, 0, s>>>(g, n_markers, X, x[0], x[1], x[2], dV, u[0], u[1], u[2],
                                                         JU, partial);
    else
        k_rigid_interp<2><<<blocks, kRigidBlock, 0, s>>>(g, n_markers, X, x[0], x[1], 0.0, dV, u[0], u[1], nullptr,
                                                         JU, partial);
    if (hipGetLastError() != hipSuccess) return STOKES_EHIP;
    double *hp = t_partials;
    if (hipMemcpyAsync(hp, partial, (size_t)blocks * kSums * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return STOKES_EHIP;
    double S[kSums] = {0.0};
    for (int b = 0; b < blocks; ++b)
        for (int k = 0; k < kSums; ++k) S[k] += hp[(size_t)b * kSums + k];
    if (S[12] > 0.0) return STOKES_EINVAL;             // a marker outside the domain: nothing written
    double ur[3] = {body->u_r[0], body->u_r[1], body->u_r[2]};
    double wr[3] = {body->w_r[0], body->w_r[1], body->w_r[2]};
    if (free_body) {
        const double M = dV * (double)n_markers;
        for (int d = 0; d < 3; ++d) ur[d] = d < dim ? S[d] / M : 0.0;
        if (dim == 2) {
            const double I = S[11];                    // sum (Rx^2 + Ry^2) dV
            if (!(I > 0.0)) return STOKES_EINVAL;      // fewer than two distinct markers
            wr[0] = S[5] / I;
            wr[1] = wr[2] = 0.0;
        } else {
            const double a = S[6], b = S[7], c = S[8], d = S[9], e = S[10], f = S[11];
            // symmetric [[a b c] [b d e] [c e f]]: cofactors and determinant
            const double A = d * f - e * e, B = c * e - b * f, C = b * e - c * d;
            const double D = a * f - c * c, E = b * c - a * e, F = a * d - b * b;
            const double det = a * A + b * B + c * C;
            const double tr = a + d + f;
            if (!(det > 1e-12 * tr * tr * tr)) return STOKES_EINVAL;   // collinear markers
            const double l0 = S[3], l1 = S[4], l2 = S[5];
            wr[0] = (A * l0 + B * l1 + C * l2) / det;
            wr[1] = (B * l0 + D * l1 + E * l2) / det;
            wr[2] = (C * l0 + E * l1 + F * l2) / det;
        }
    }
    const double scale = dV / (g.h[0] * g.h[1] * (dim == 3 ? g.h[2] : 1.0));
    if (dim == 3)
        k_rigid_spread<3><<<blocks, kRigidBlock, 0, s>>>(g, n_markers, X, JU, x[0], x[1], x[2], ur[0], ur[1], ur[2],
                                                         wr[0], wr[1], wr[2], scale, u[0], u[1], u[2]);
    else
        k_rigid_spread<2><<<blocks, kRigidBlock, 0, s>>>(g, n_markers, X, JU, x[0], x[1], 0.0, ur[0], ur[1], 0.0,
                                                         wr[0], 0.0, 0.0, scale, u[0], u[1], nullptr);
    if (hipGetLastError() != hipSuccess) return STOKES_EHIP;
    for (int d = 0; d < 3; ++d) {
        body->u_r[d] = ur[d];
        body->w_r[d] = wr[d];
    }
    return STOKES_OK;
}

}  // namespace

extern "C" size_t stokes_rigid_workspace_size(int dim, long long n_markers) {
    if ((dim != 2 && dim != 3) || n_markers < 0) return 0;
    const long long blocks = std::min<long long>(std::max<long long>((n_markers + kRigidBlock - 1) / kRigidBlock, 1),
                                                 kRigidMaxBlocks);
    return (size_t)(n_markers * dim + blocks * kSums) * sizeof(double);
}

extern "C" stokes_status stokes_rigid_projection(const stokes_grid *grid, double *const u[3], long long n_markers,
        const double *X, double dV, int free_body, stokes_body *body, void *workspace, size_t ws_bytes,
        void *stream) {
    RigidGrid g;
    stokes_status st = rigid_check(grid, u, n_markers, dV, free_body, body, g);
    if (st != STOKES_OK || n_markers == 0) return st;
    if (!X || !workspace || ws_bytes < stokes_rigid_workspace_size(g.dim, n_markers)) {
        return !X || !workspace ? STOKES_EINVAL : STOKES_ENOMEM;
    }
    return rigid_impl(g, u, n_markers, X, dV, free_body, body, static_cast<double *>(workspace),
                      reinterpret_cast<hipStream_t>(stream));
}

extern "C" stokes_status stokes_rigid_projection_noalloc(const stokes_grid *grid, double *const u[3],
        long long n_markers, const double *X, double dV, int free_body, stokes_body *body, void *stream) {
    RigidGrid g;
    stokes_status st = rigid_check(grid, u, n_markers, dV, free_body, body, g);
    if (st != STOKES_OK || n_markers == 0) return st;
    if (!X) return STOKES_EINVAL;
    if (n_markers > kScratchMarkers) {
        stk_set_thread_error("stokes_rigid_projection_noalloc: more markers than its fixed scratch holds "
                             "(STOKES_RIGID_NOALLOC_MAX_MARKERS = 524288)");
        return STOKES_ENOMEM;
    }
    double *ws = nullptr;
    if (scratch_of_current_device(&ws) != hipSuccess) {
        stk_set_thread_error("stokes_rigid_projection_noalloc: hipGetSymbolAddress of the scratch array failed");
        return STOKES_EHIP;
    }
    return rigid_impl(g, u, n_markers, X, dV, free_body, body, ws, reinterpret_cast<hipStream_t>(stream));
}
