// Face-density transport of the conservative scheme: the three-stage SSP-RK3
// update of the face densities (Sec. 4.2.2, eqs. eq_rk1, eq_rk2, eq_rk3),
//     rho1 = rho_n - dt R(u1, rho_n)
//     rho2 = 3/4 rho_n + 1/4 rho1 - 1/4 dt R(u2, rho1)
//     rho  = 1/3 rho_n + 2/3 rho2 - 2/3 dt R(u3, rho2),
// whose result is the face density that stokes_setup takes.  R(u, rho) is the
// divergence of u_adv rho_lim over the control volume of each face (one cell
// long in every direction, centred on the face):
//   - u_adv on a control-volume face normal to d is the mean of the two nearest
//     d-velocities (along the face's own axis the two faces around the cell
//     centre; across it the d-faces of the cells on either side of the edge);
//     wall-normal velocities are zero, so nothing crosses a wall;
//   - rho_lim is the CUI-limited cubic upwind value (Waterson and Deconinck
//     2007) from the far-upwind, upwind and downwind densities U, C, D along d:
//     r = (C - U)/(D - U), f = 3r on (0, 2/13], 5r/6 + 1/3 on (2/13, 4/5],
//     1 on (4/5, 1), r otherwise; rho_lim = U + f (D - U), or C when D = U;
//   - densities beyond a wall mirror the interior (homogeneous Neumann);
//   - wall-normal faces are not transported and hold rho_n in every stage.
//
// GPU mapping: one launch per stage, one thread per point (i, j, k) of the
// (Nx+1)(Ny+1)(Nz+1) index space, which owns the x-face i, the y-face j and the
// z-face k of cell (i, j, k) -- all in the caller's C-order layouts; stencil
// neighbours come from cache.  Every control-volume face flux is evaluated by
// both faces that share it, in the same arithmetic, so the update is exactly
// conservative in the same sense as its definition.
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace {

constexpr int kTrBlock = 256;

struct TrGrid {
    int dim;
    int n[3];
    double ih[3];
};

struct StageArgs {
    double a_n, a_s, c_dt;                   // out = a_n rho_n + a_s rho_s - c_dt R(u, rho_s)
    const double *rn[3], *rs[3], *u[3];
    double *out[3];
};

// extent of component c's array along axis d
__device__ __host__ inline int ext(const TrGrid &g, int c, int d) { return g.n[d] + (c == d ? 1 : 0); }

__device__ inline long long lin(const TrGrid &g, int c, int i, int j, int k) {
    return (long long)i + (long long)ext(g, c, 0) * ((long long)j + (long long)ext(g, c, 1) * k);
}

__device__ inline double cui(double U, double C, double D) {
    const double den = D - U;
    if (den == 0.0) return C;
    const double r = (C - U) / den;
    double f = r;
    if (r > 0.0 && r <= 2.0 / 13.0) f = 3.0 * r;
    else if (r > 2.0 / 13.0 && r <= 0.8) f = (5.0 / 6.0) * r + 1.0 / 3.0;
    else if (r > 0.8 && r < 1.0) f = 1.0;
    return U + f * den;
}

// density of component c at index m along d from the face (i, j, k), mirrored
// beyond a wall (about the wall face along c itself, about the wall across it)
__device__ inline double rho_at(const TrGrid &g, const double *rc, int c, int d, const int p[3], int m) {
    const int E = ext(g, c, d);
    int mm = m;
    if (c == d) mm = m < 0 ? -m : (m > E - 1 ? 2 * (E - 1) - m : m);
    else mm = m < 0 ? -m - 1 : (m > E - 1 ? 2 * E - 1 - m : m);
    int q[3] = {p[0], p[1], p[2]};
    q[d] = mm;
    return rc[lin(g, c, q[0], q[1], q[2])];
}

// advective velocity on the control-volume face between entries m-1 and m
// along d of the interior c-face p
__device__ inline double adv(const TrGrid &g, const double *const u[3], int c, int d, const int p[3], int m) {
    if (d == c) {
        if (m == 0 || m == ext(g, c, d)) return 0.0;
        int q0[3] = {p[0], p[1], p[2]}, q1[3] = {p[0], p[1], p[2]};
        q0[d] = m - 1;
        q1[d] = m;
        return 0.5 * (u[d][lin(g, d, q0[0], q0[1], q0[2])] + u[d][lin(g, d, q1[0], q1[1], q1[2])]);
    }
    int q0[3] = {p[0], p[1], p[2]}, q1[3] = {p[0], p[1], p[2]};
    q0[c] -= 1;
    q0[d] = m;
    q1[d] = m;
    return 0.5 * (u[d][lin(g, d, q0[0], q0[1], q0[2])] + u[d][lin(g, d, q1[0], q1[1], q1[2])]);
}

__device__ inline double flux(const TrGrid &g, const double *const u[3], const double *rc, int c, int d,
                              const int p[3], int m) {
    const double a = adv(g, u, c, d, p, m);
    double lim;
    if (a > 0.0) lim = cui(rho_at(g, rc, c, d, p, m - 2), rho_at(g, rc, c, d, p, m - 1), rho_at(g, rc, c, d, p, m));
    else lim = cui(rho_at(g, rc, c, d, p, m + 1), rho_at(g, rc, c, d, p, m), rho_at(g, rc, c, d, p, m - 1));
    return a * lim;
}

__global__ void __launch_bounds__(kTrBlock) k_rk3_stage(TrGrid g, StageArgs s) {
    const long long px = g.n[0] + 1, py = g.n[1] + 1, pz = g.dim == 3 ? g.n[2] + 1 : 1;
    const long long t = (long long)blockIdx.x * kTrBlock + threadIdx.x;
    if (t >= px * py * pz) return;
    const int i = (int)(t % px), j = (int)((t / px) % py), k = (int)(t / (px * py));
    const int p[3] = {i, j, k};
    for (int c = 0; c < g.dim; ++c) {
        // does point (i, j, k) hold a c-face?
        bool has = true;
        for (int d = 0; d < g.dim; ++d)
            if (p[d] >= ext(g, c, d)) has = false;
        if (!has) continue;
        const long long q = lin(g, c, i, j, k);
        const double rn = s.rn[c][q];
        if (p[c] == 0 || p[c] == g.n[c]) {          // wall-normal face: not transported
            s.out[c][q] = rn;
            continue;
        }
        double R = 0.0;
        for (int d = 0; d < g.dim; ++d) {
            const int m = p[d];
            R += (flux(g, s.u, s.rs[c], c, d, p, m + 1) - flux(g, s.u, s.rs[c], c, d, p, m)) * g.ih[d];
        }
        s.out[c][q] = s.a_n * rn + s.a_s * s.rs[c][q] - s.c_dt * R;
    }
}

size_t face_count(const stokes_grid *g, int c) {
    const int d = g->dim;
    size_t n = 1;
    for (int a = 0; a < d; ++a) n *= (size_t)g->n[a] + (a == c ? 1 : 0);
    return n;
}

}  // namespace

extern "C" size_t stokes_density_workspace_size(const stokes_grid *grid) {
    if (!grid || (grid->dim != 2 && grid->dim != 3)) return 0;
    for (int a = 0; a < grid->dim; ++a)
        if (grid->n[a] < 2) return 0;
    size_t tot = 0;
    for (int c = 0; c < grid->dim; ++c) tot += face_count(grid, c);
    return tot * sizeof(double);
}

extern "C" stokes_status stokes_density_rk3(const stokes_grid *grid, double dt, const double *const rho_n[3],
                                            const double *const u_stage[9], double *const rho_out[3],
                                            void *workspace, size_t ws_bytes, void *stream) {
    if (!grid || !rho_n || !u_stage || !rho_out) return STOKES_EINVAL;
    const int dim = grid->dim;
    if (dim != 2 && dim != 3) return STOKES_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return STOKES_EINVAL;
    TrGrid g{};
    g.dim = dim;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = a < dim ? grid->n[a] : 1;
        g.ih[a] = 0.0;
    }
    long long pts = 1;
    for (int a = 0; a < dim; ++a) {
        if (grid->n[a] < 2) return STOKES_ESHAPE;
        if (!(grid->h[a] > 0.0) || !std::isfinite(grid->h[a])) return STOKES_EINVAL;
        g.ih[a] = 1.0 / grid->h[a];
        pts *= (long long)grid->n[a] + 1;
    }
    if (pts >= (1LL << 40)) return STOKES_ESHAPE;
    for (int c = 0; c < dim; ++c) {
        if (!rho_n[c] || !rho_out[c]) return STOKES_EINVAL;
        for (int st = 0; st < 3; ++st)
            if (!u_stage[3 * st + c]) return STOKES_EINVAL;
    }
    const size_t need = stokes_density_workspace_size(grid);
    if (!workspace) return STOKES_EINVAL;
    if (ws_bytes < need) return STOKES_ENOMEM;
    // rho1 lives in rho_out, rho2 in the workspace
    double *r2[3] = {nullptr, nullptr, nullptr};
    {
        double *w = static_cast<double *>(workspace);
        for (int c = 0; c < dim; ++c) {
            r2[c] = w;
            w += face_count(grid, c);
        }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const unsigned blocks = (unsigned)((pts + kTrBlock - 1) / kTrBlock);
    auto stage = [&](double a_n, double a_s, double c_dt, const double *const rs[3], int st, double *const out[3]) {
        StageArgs a{};
        a.a_n = a_n;
        a.a_s = a_s;
        a.c_dt = c_dt;
        for (int c = 0; c < 3; ++c) {
            a.rn[c] = c < dim ? rho_n[c] : nullptr;
            a.rs[c] = c < dim ? rs[c] : nullptr;
            a.u[c] = c < dim ? u_stage[3 * st + c] : nullptr;
            a.out[c] = c < dim ? out[c] : nullptr;
        }
        k_rk3_stage<<<blocks, kTrBlock, 0, s>>>(g, a);
    };
    stage(0.0, 1.0, dt, rho_n, 0, rho_out);
    stage(0.75, 0.25, 0.25 * dt, rho_out, 1, r2);
    stage(1.0 / 3.0, 2.0 / 3.0, (2.0 / 3.0) * dt, r2, 2, rho_out);
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}
