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
// GPU mapping: one launch per stage, one thread per face (blockIdx.y is the
// component), in the caller's C-order layouts; stencil neighbours come from
// cache.  Every control-volume face flux is evaluated by both faces that share
// it, in the same arithmetic, so the update is exactly conservative in the same
// sense as its definition.
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <algorithm>
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

// CUI-limited face value from far-upwind U, upwind C and downwind D.  The
// normalised upwind value r = (C - U) / (D - U) only selects the branch, so the
// comparisons are made on N = C - U and A = D - U with A's sign folded in
// (no division); each branch's value U + f(r) A is written without r:
// 3 r A = 3 N, (5/6 r + 1/3) A = 5/6 N + A/3, A, and N.
__device__ inline double cui(double U, double C, double D) {
    const double A = D - U, N = C - U;
    if (A == 0.0) return C;
    const double An = fabs(A), Nn = A > 0.0 ? N : -N;
    if (Nn <= 0.0 || Nn >= An) return C;                   // r <= 0 or r >= 1: upwind
    if (13.0 * Nn <= 2.0 * An) return U + 3.0 * N;         // 0 < r <= 2/13
    if (5.0 * Nn <= 4.0 * An) return U + (5.0 / 6.0) * N + A / 3.0;   // 2/13 < r <= 4/5
    return D;                                              // 4/5 < r < 1
}

// Index of entry m along d (mirrored beyond a wall: about the wall face along the
// component's own axis, about the wall across it) for an array of extent E.
__device__ inline int mirror(int m, int E, bool face_axis) {
    if (face_axis) return m < 0 ? -m : (m > E - 1 ? 2 * (E - 1) - m : m);
    return m < 0 ? -m - 1 : (m > E - 1 ? 2 * E - 1 - m : m);
}

// One thread per c-face (blockIdx.y = c): out = a_n rho_n + a_s rho_s - c_dt R on
// interior faces, rho_n on wall-normal ones.  32-bit indices (the host checks
// that every array has fewer than 2^31 entries).
__global__ void __launch_bounds__(kTrBlock) k_rk3_stage(TrGrid g, StageArgs s) {
    const int c = blockIdx.y;
    const int E0 = ext(g, c, 0), E1 = ext(g, c, 1), E2 = g.dim == 3 ? ext(g, c, 2) : 1;
    const int t = blockIdx.x * kTrBlock + threadIdx.x;
    if (t >= E0 * E1 * E2) return;
    const int p[3] = {t % E0, (t / E0) % E1, t / (E0 * E1)};
    const double *rc = s.rs[c];
    const double rn = s.rn[c][t];
    if (p[c] == 0 || p[c] == g.n[c]) {                  // wall-normal face: not transported
        s.out[c][t] = rn;
        return;
    }
    const int Ec[3] = {E0, E1, E2};
    const int st[3] = {1, E0, E0 * E1};
    double R = 0.0;
    for (int d = 0; d < g.dim; ++d) {
        const int m = p[d], E = Ec[d];
        const bool fa = d == c;
        const int base = t - m * st[d];
        // densities at m-2 .. m+2 along d
        double r5[5];
#pragma unroll
        for (int o = 0; o < 5; ++o) r5[o] = rc[base + mirror(m - 2 + o, E, fa) * st[d]];
        // advective velocities on the control-volume faces m (lower) and m+1 (upper)
        double alo, ahi;
        const double *ud = s.u[d];
        if (fa) {
            // c-faces around the cell centres m-1 | m and m | m+1; zero beyond the walls
            const int sd = st[d];
            const double uc = ud[t];
            alo = m == 0 ? 0.0 : 0.5 * (ud[t - sd] + uc);
            ahi = m == E - 1 ? 0.0 : 0.5 * (uc + ud[t + sd]);
        } else {
            // d-faces of the cells p[c]-1 and p[c] at edge index m and m+1 along d
            const int Ed[3] = {g.n[0] + (d == 0), g.n[1] + (d == 1), g.dim == 3 ? g.n[2] + (d == 2) : 1};
            const int sd1 = 1, sd2 = Ed[0], sd3 = Ed[0] * Ed[1];
            const int sdd[3] = {sd1, sd2, sd3};
            const int q = p[0] * sdd[0] + p[1] * sdd[1] + p[2] * sdd[2];   // the d-face at cell p[c], index m
            const int qm = q - sdd[c];                                     // cell p[c] - 1
            alo = 0.5 * (ud[qm] + ud[q]);
            ahi = 0.5 * (ud[qm + sdd[d]] + ud[q + sdd[d]]);
        }
        const double flo = alo * (alo > 0.0 ? cui(r5[0], r5[1], r5[2]) : cui(r5[3], r5[2], r5[1]));
        const double fhi = ahi * (ahi > 0.0 ? cui(r5[1], r5[2], r5[3]) : cui(r5[4], r5[3], r5[2]));
        R += (fhi - flo) * g.ih[d];
    }
    s.out[c][t] = s.a_n * rn + s.a_s * rc[t] - s.c_dt * R;
}

size_t face_count(const stokes_grid *g, int c) {
    const int d = g->dim;
    size_t n = 1;
    for (int a = 0; a < d; ++a) n *= (size_t)g->n[a] + (a == c ? 1 : 0);
    return n;
}

// True when a face array would hold 2^31 faces or more (32-bit thread and face
// indices); counted in double, since a product of 32-bit extents can exceed 64 bits.
bool too_many_faces(const stokes_grid *g) {
    for (int c = 0; c < g->dim; ++c) {
        double n = 1.0;
        for (int a = 0; a < g->dim; ++a) n *= (double)g->n[a] + (a == c ? 1.0 : 0.0);
        if (n >= 2147483648.0) return true;
    }
    return false;
}

}  // namespace

extern "C" size_t stokes_density_workspace_size(const stokes_grid *grid) {
    if (!grid || (grid->dim != 2 && grid->dim != 3)) return 0;
    for (int a = 0; a < grid->dim; ++a)
        if (grid->n[a] < 2) return 0;
    if (too_many_faces(grid)) return 0;
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
    for (int d = 0; d < dim; ++d)
        if (grid->periodic[d]) return STOKES_EINVAL;     // walls only
    if (!(dt > 0.0) || !std::isfinite(dt)) return STOKES_EINVAL;
    TrGrid g{};
    g.dim = dim;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = a < dim ? grid->n[a] : 1;
        g.ih[a] = 0.0;
    }
    for (int a = 0; a < dim; ++a) {
        if (grid->n[a] < 2) return STOKES_ESHAPE;
        if (!(grid->h[a] > 0.0) || !std::isfinite(grid->h[a])) return STOKES_EINVAL;
        g.ih[a] = 1.0 / grid->h[a];
    }
    if (too_many_faces(grid)) return STOKES_ESHAPE;
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
    // one thread per face of the largest component array
    long long most = 0;
    for (int c = 0; c < dim; ++c) most = std::max<long long>(most, (long long)face_count(grid, c));
    const unsigned blocks = (unsigned)((most + kTrBlock - 1) / kTrBlock);
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
        k_rk3_stage<<<dim3(blocks, dim), kTrBlock, 0, s>>>(g, a);
    };
    stage(0.0, 1.0, dt, rho_n, 0, rho_out);
    stage(0.75, 0.25, 0.25 * dt, rho_out, 1, r2);
    stage(1.0 / 3.0, 2.0 / 3.0, (2.0 / 3.0) * dt, r2, 2, rho_out);
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}
