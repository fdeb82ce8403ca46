// Device kernels of the MAC-grid Stokes solver (gfx950).
//
// All kernels are memory-bound stencils or streaming BLAS-1 operations.  One
// thread handles one point of the padded box (see box.hpp); launches use
// 256-thread blocks (four wave64 wavefronts).  Templates: DIM (2 or 3) and R,
// the number type of the multigrid data (double, or float for the FP32
// multigrid form).  The fine-level Stokes operator, FGMRES vectors and inner
// products are always double.
#pragma once
#include <hip/hip_runtime.h>
#include "box.hpp"

namespace stk {

constexpr int kBlock = 256;

// Workgroups are dealt to the 8 XCDs round-robin by workgroup id, and each XCD
// has its own L2.  This bijection of [0, G) gives XCD x a contiguous range of
// about G/8 logical blocks, so that neighbouring tiles (and their stencil
// halos) share one L2.
__device__ inline int xcd_swizzle(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, local = b >> 3;
    return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Box point handled by this thread of a flat launch of nblocks_box() blocks.
__device__ inline int box_thread_index() {
    return xcd_swizzle(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
}

__device__ inline void decompose(const Box &b, int idx, int &i, int &j, int &k) {
    i = idx % b.px;
    int t = idx / b.px;
    j = t % b.py;
    k = t / b.py;
}

// Coefficients of one level's velocity operator A = mass - theta * L_mu.
template <class R>
struct VelCoef {
    const R *mass[3];   // rho_face / dt
    const R *mu;        // cell viscosity
    const R *mxy, *mxz, *myz;  // edge viscosity (harmonic)
    R theta;
};

// Which velocity arrays hold valid values during a smoothing pass.  Invalid
// arrays read as zero: the first sweep after a zero initial guess skips the
// zero fill of the correction.
enum { VALID_U = 1, VALID_V = 2, VALID_W = 4 };

// Neighbour offsets of box point (i, j, k) along each axis.  A wall axis steps
// to the next slot (the padding or guard holds zero beyond the last cell); a
// periodic axis wraps index 0 to n-1 and n-1 to 0, for cells, faces and edges
// alike (all indexed 0 .. n-1 along that axis).
struct Nbr {
    int xm, xp, ym, yp, zm, zp;
};
// PER = false: the caller knows that the level has walls on every side (the
// offsets are then the plain +-1, +-px, +-plane).
template <bool PER = true>
__device__ inline Nbr nbr(const Box &b, int i, int j, int k) {
    Nbr o;
    if (!PER) {
        o.xm = -1; o.xp = 1; o.ym = -b.px; o.yp = b.px; o.zm = -b.plane; o.zp = b.plane;
        return o;
    }
    o.xm = (b.per[0] && i == 0) ? b.nx - 1 : -1;
    o.xp = (b.per[0] && i == b.nx - 1) ? 1 - b.nx : 1;
    o.ym = ((b.per[1] && j == 0) ? b.ny - 1 : -1) * b.px;
    o.yp = ((b.per[1] && j == b.ny - 1) ? 1 - b.ny : 1) * b.px;
    o.zm = ((b.per[2] && k == 0) ? b.nz - 1 : -1) * b.plane;
    o.zp = ((b.per[2] && k == b.nz - 1) ? 1 - b.nz : 1) * b.plane;
    return o;
}

// ---------------------------------------------------------------- momentum rows
// Each returns the off-diagonal part of one momentum row (the row evaluated with
// the centre value set to zero, wall ghosts included) and its diagonal, so that
// (A u)_row = diag * u_c + off.  Formulas: strain-rate divergence on the MAC
// grid; normal stresses 2 mu du/dx at cells, shear stresses mu_e (du/dy + dv/dx)
// at edges; tangential ghosts beyond a wall are minus the interior value; a
// periodic axis has no wall (its neighbours wrap, see Nbr).

template <int DIM, class R>
__device__ inline void row_u(const Box &b, int idx, int i, int j, int k, const R *u, const R *v,
                             const R *w, int valid, const VelCoef<R> &c, R &off, R &diag) {
    const Nbr o = nbr(b, i, j, k);
    const R ihx = (R)b.ihx, ihy = (R)b.ihy, ihz = (R)b.ihz;
    const bool vu = valid & VALID_U, vv = valid & VALID_V, vw = valid & VALID_W;
    const bool hN = b.per[1] || j + 1 < b.ny, hS = b.per[1] || j > 0;
    R uE = vu ? u[idx + o.xp] : R(0), uW = vu ? u[idx + o.xm] : R(0);
    R uN = (hN && vu) ? u[idx + o.yp] : R(0);
    R uS = (hS && vu) ? u[idx + o.ym] : R(0);
    R gN = hN ? R(1) : R(2), gS = hS ? R(1) : R(2);
    R m1 = c.mu[idx], m0 = c.mu[idx + o.xm];
    R mN = c.mxy[idx + o.yp], mS = c.mxy[idx];
    R dvN = vv ? (v[idx + o.yp] - v[idx + o.yp + o.xm]) : R(0);
    R dvS = vv ? (v[idx] - v[idx + o.xm]) : R(0);
    // lap with u_c = 0
    R lap = R(2) * (m1 * uE + m0 * uW) * ihx * ihx
          + (mN * (uN * ihy + dvN * ihx) - mS * (-uS * ihy + dvS * ihx)) * ihy;
    R dg = R(2) * (m0 + m1) * ihx * ihx + (mN * gN + mS * gS) * ihy * ihy;
    if (DIM == 3) {
        const bool hT = b.per[2] || k + 1 < b.nz, hB = b.per[2] || k > 0;
        R uT = (hT && vu) ? u[idx + o.zp] : R(0);
        R uB = (hB && vu) ? u[idx + o.zm] : R(0);
        R gT = hT ? R(1) : R(2), gB = hB ? R(1) : R(2);
        R mT = c.mxz[idx + o.zp], mB = c.mxz[idx];
        R dwT = vw ? (w[idx + o.zp] - w[idx + o.zp + o.xm]) : R(0);
        R dwB = vw ? (w[idx] - w[idx + o.xm]) : R(0);
        lap += (mT * (uT * ihz + dwT * ihx) - mB * (-uB * ihz + dwB * ihx)) * ihz;
        dg += (mT * gT + mB * gB) * ihz * ihz;
    }
    off = -c.theta * lap;
    diag = c.mass[0][idx] + c.theta * dg;
}

template <int DIM, class R>
__device__ inline void row_v(const Box &b, int idx, int i, int j, int k, const R *u, const R *v,
                             const R *w, int valid, const VelCoef<R> &c, R &off, R &diag) {
    const Nbr o = nbr(b, i, j, k);
    const R ihx = (R)b.ihx, ihy = (R)b.ihy, ihz = (R)b.ihz;
    const bool vu = valid & VALID_U, vv = valid & VALID_V, vw = valid & VALID_W;
    // on an open top (2D, j = ny) the cell above is a ghost: its normal stress is
    // minus the one below (v and mu mirrored) and the tangential u above is minus
    // the one below
    const bool tp = b.dim == 2 && b.open_top && j == b.ny;
    const bool hE = b.per[0] || i + 1 < b.nx, hW = b.per[0] || i > 0;
    R vN = vv ? v[tp ? idx + o.ym : idx + o.yp] : R(0), vS = vv ? v[idx + o.ym] : R(0);
    R vE = (hE && vv) ? v[idx + o.xp] : R(0);
    R vW = (hW && vv) ? v[idx + o.xm] : R(0);
    R gE = hE ? R(1) : R(2), gW = hW ? R(1) : R(2);
    R m1 = c.mu[tp ? idx + o.ym : idx], m0 = c.mu[idx + o.ym];
    R mE = c.mxy[idx + o.xp], mW = c.mxy[idx];
    R duE = vu ? (tp ? R(-2) * u[idx + o.xp + o.ym] : u[idx + o.xp] - u[idx + o.xp + o.ym]) : R(0);
    R duW = vu ? (tp ? R(-2) * u[idx + o.ym] : u[idx] - u[idx + o.ym]) : R(0);
    R lap = R(2) * (m1 * vN + m0 * vS) * ihy * ihy
          + (mE * (vE * ihx + duE * ihy) - mW * (-vW * ihx + duW * ihy)) * ihx;
    R dg = R(2) * (m0 + m1) * ihy * ihy + (mE * gE + mW * gW) * ihx * ihx;
    if (DIM == 3) {
        const bool hT = b.per[2] || k + 1 < b.nz, hB = b.per[2] || k > 0;
        R vT = (hT && vv) ? v[idx + o.zp] : R(0);
        R vB = (hB && vv) ? v[idx + o.zm] : R(0);
        R gT = hT ? R(1) : R(2), gB = hB ? R(1) : R(2);
        R mT = c.myz[idx + o.zp], mB = c.myz[idx];
        R dwT = vw ? (w[idx + o.zp] - w[idx + o.zp + o.ym]) : R(0);
        R dwB = vw ? (w[idx] - w[idx + o.ym]) : R(0);
        lap += (mT * (vT * ihz + dwT * ihy) - mB * (-vB * ihz + dwB * ihy)) * ihz;
        dg += (mT * gT + mB * gB) * ihz * ihz;
    }
    off = -c.theta * lap;
    diag = c.mass[1][idx] + c.theta * dg;
}

template <class R>
__device__ inline void row_w(const Box &b, int idx, int i, int j, int k, const R *u, const R *v,
                             const R *w, int valid, const VelCoef<R> &c, R &off, R &diag) {
    const Nbr o = nbr(b, i, j, k);
    const R ihx = (R)b.ihx, ihy = (R)b.ihy, ihz = (R)b.ihz;
    const bool vu = valid & VALID_U, vv = valid & VALID_V, vw = valid & VALID_W;
    // on an open top (k = nz) the cell above is a ghost: its normal stress is minus
    // the one below (w and mu mirrored) and the tangential u, v above are minus the
    // ones below
    const bool tp = b.open_top && k == b.nz;
    const bool hE = b.per[0] || i + 1 < b.nx, hW = b.per[0] || i > 0;
    const bool hN = b.per[1] || j + 1 < b.ny, hS = b.per[1] || j > 0;
    R wT = vw ? w[tp ? idx + o.zm : idx + o.zp] : R(0), wB = vw ? w[idx + o.zm] : R(0);
    R wE = (hE && vw) ? w[idx + o.xp] : R(0);
    R wW = (hW && vw) ? w[idx + o.xm] : R(0);
    R wN = (hN && vw) ? w[idx + o.yp] : R(0);
    R wS = (hS && vw) ? w[idx + o.ym] : R(0);
    R gE = hE ? R(1) : R(2), gW = hW ? R(1) : R(2);
    R gN = hN ? R(1) : R(2), gS = hS ? R(1) : R(2);
    R m1 = c.mu[tp ? idx + o.zm : idx], m0 = c.mu[idx + o.zm];
    R mE = c.mxz[idx + o.xp], mW = c.mxz[idx];
    R mN = c.myz[idx + o.yp], mS = c.myz[idx];
    R duE = vu ? (tp ? R(-2) * u[idx + o.xp + o.zm] : u[idx + o.xp] - u[idx + o.xp + o.zm]) : R(0);
    R duW = vu ? (tp ? R(-2) * u[idx + o.zm] : u[idx] - u[idx + o.zm]) : R(0);
    R dvN = vv ? (tp ? R(-2) * v[idx + o.yp + o.zm] : v[idx + o.yp] - v[idx + o.yp + o.zm]) : R(0);
    R dvS = vv ? (tp ? R(-2) * v[idx + o.zm] : v[idx] - v[idx + o.zm]) : R(0);
    R lap = R(2) * (m1 * wT + m0 * wB) * ihz * ihz
          + (mE * (wE * ihx + duE * ihz) - mW * (-wW * ihx + duW * ihz)) * ihx
          + (mN * (wN * ihy + dvN * ihz) - mS * (-wS * ihy + dvS * ihz)) * ihy;
    R dg = R(2) * (m0 + m1) * ihz * ihz + (mE * gE + mW * gW) * ihx * ihx + (mN * gN + mS * gS) * ihy * ihy;
    off = -c.theta * lap;
    diag = c.mass[2][idx] + c.theta * dg;
}

// Unknown faces of each component: interior faces, plus the faces of the open top
// (y = Ly in 2D, z = Lz in 3D) when the box has one.
__device__ inline bool top_v(const Box &b, int j) { return b.open_top && b.dim == 2 && j == b.ny; }
__device__ inline bool top_w(const Box &b, int k) { return b.open_top && b.dim == 3 && k == b.nz; }
__device__ inline bool is_ux(const Box &b, int i, int j, int k) {
    return (i >= 1 || b.per[0]) && i < b.nx && j < b.ny && k < b.nz;
}
__device__ inline bool is_vy(const Box &b, int i, int j, int k) {
    return (j >= 1 || b.per[1]) && (j < b.ny || top_v(b, j)) && i < b.nx && k < b.nz;
}
__device__ inline bool is_wz(const Box &b, int i, int j, int k) {
    return (k >= 1 || b.per[2]) && (k < b.nz || top_w(b, k)) && i < b.nx && j < b.ny;
}
__device__ inline bool is_cell(const Box &b, int i, int j, int k) { return i < b.nx && j < b.ny && k < b.nz; }

// ---------------------------------------------------------------- fine operator (FP64)
// y = K x  (or y = f - K x when f != nullptr) for the coupled system
// K = [A G; -D 0]; all four outputs of a box point are written by one thread.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_apply(Box b, VelCoef<double> c,
        const double *__restrict__ xu, const double *__restrict__ xv,
        const double *__restrict__ xw, const double *__restrict__ xp,
        const double *__restrict__ fu, const double *__restrict__ fv,
        const double *__restrict__ fw, const double *__restrict__ fp,
        double *__restrict__ yu, double *__restrict__ yv,
        double *__restrict__ yw, double *__restrict__ yp) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    const int sy = b.px, sz = b.plane;
    const int all = VALID_U | VALID_V | VALID_W;
    double off, dg, r;
    r = 0.0;
    const Nbr o = nbr(b, i, j, k);
    if (is_ux(b, i, j, k)) {
        row_u<DIM, double>(b, idx, i, j, k, xu, xv, xw, all, c, off, dg);
        r = dg * xu[idx] + off + (xp[idx] - xp[idx + o.xm]) * b.ihx;
        if (fu) r = fu[idx] - r;
    }
    yu[idx] = r;
    r = 0.0;
    if (is_vy(b, i, j, k)) {
        row_v<DIM, double>(b, idx, i, j, k, xu, xv, xw, all, c, off, dg);
        // open top: zero pressure on the face, the ghost above is minus the cell below
        const double pN = top_v(b, j) ? -xp[idx + o.ym] : xp[idx];
        r = dg * xv[idx] + off + (pN - xp[idx + o.ym]) * b.ihy;
        if (fv) r = fv[idx] - r;
    }
    yv[idx] = r;
    if (DIM == 3) {
        r = 0.0;
        if (is_wz(b, i, j, k)) {
            row_w<double>(b, idx, i, j, k, xu, xv, xw, all, c, off, dg);
            const double pT = top_w(b, k) ? -xp[idx + o.zm] : xp[idx];
            r = dg * xw[idx] + off + (pT - xp[idx + o.zm]) * b.ihz;
            if (fw) r = fw[idx] - r;
        }
        yw[idx] = r;
    }
    r = 0.0;
    if (is_cell(b, i, j, k)) {
        double dv = (xu[idx + o.xp] - xu[idx]) * b.ihx + (xv[idx + o.yp] - xv[idx]) * b.ihy;
        if (DIM == 3) dv += (xw[idx + o.zp] - xw[idx]) * b.ihz;
        r = -dv;
        if (fp) r = fp[idx] - r;
    }
    yp[idx] = r;
}

// 3D y = K x (or f - K x) marching in z: a block owns a TX x TY tile of cells
// and a chunk of kc planes.  u, v and w sit in three-plane LDS rings (planes
// k-1, k, k+1) and the cell and xy-edge viscosity of plane k in LDS, each on the
// tile plus a one-point halo, so every plane of those five fields is read from
// memory once per block (the stencil's in-plane neighbours come from LDS, not
// from caches that the other blocks' streams evict); the centre-only fields
// (mass, f), the pressure and the xz / yz edge viscosity (one-sided
// neighbours) are read from memory directly, with their values at k-1 / k+1
// carried in registers.  Only unknown positions (i < nx, j < ny, k < nz) are
// visited: the padding and wall-normal slots of y hold zero already and are not
// written.  Halo points outside the box (index -1) are never used by a row and
// are not loaded.  Same row formulas as k_apply.
template <int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_apply3_z(Box b, int kc, VelCoef<double> c,
        const double *__restrict__ xu, const double *__restrict__ xv,
        const double *__restrict__ xw, const double *__restrict__ xp,
        const double *__restrict__ fu, const double *__restrict__ fv,
        const double *__restrict__ fw, const double *__restrict__ fp,
        double *__restrict__ yu, double *__restrict__ yv,
        double *__restrict__ yw, double *__restrict__ yp) {
    constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY, NT = TX * TY;
    __shared__ double sU[3][HP], sV[3][HP], sW[3][HP], sM[HP], sXY[HP];
    const int G = gridDim.x * gridDim.y * gridDim.z;
    int t = xcd_swizzle(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), G);
    const int bx_ = t % gridDim.x;
    t /= gridDim.x;
    const int by_ = t % gridDim.y, bz_ = t / gridDim.y;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int i0 = bx_ * TX, j0 = by_ * TY;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < b.nx && j < b.ny;
    const int k0 = bz_ * kc, k1 = min(k0 + kc, b.nz);
    const int sy = b.px, sz = b.plane;
    const double ihx = b.ihx, ihy = b.ihy, ihz = b.ihz, th = c.theta;
    auto slot = [](int k) { return (k + 3) % 3; };          // k >= -1
    // halo point t of plane k: box point (i0 - 1 + t % HX, j0 - 1 + t / HX, k) if it
    // lies in the box (0 <= i <= nx, 0 <= j <= ny, 0 <= k <= nz), else none
    auto hq = [&](int tt, int k) {
        const int gi = i0 - 1 + tt % HX, gj = j0 - 1 + tt / HX;
        return (gi >= 0 && gi <= b.nx && gj >= 0 && gj <= b.ny && k >= 0 && k <= b.nz) ? gi + sy * (gj + b.py * k) : -1;
    };
    auto load_vel = [&](int k) {
        const int sl = slot(k);
        for (int tt = tid; tt < HP; tt += NT) {
            const int q = hq(tt, k);
            sU[sl][tt] = q >= 0 ? xu[q] : 0.0;
            sV[sl][tt] = q >= 0 ? xv[q] : 0.0;
            sW[sl][tt] = q >= 0 ? xw[q] : 0.0;
        }
    };
    auto load_mu = [&](int k) {
        for (int tt = tid; tt < HP; tt += NT) {
            const int q = hq(tt, k);
            sM[tt] = q >= 0 ? c.mu[q] : 0.0;
            sXY[tt] = q >= 0 ? c.mxy[q] : 0.0;
        }
    };
    const double gE = i + 1 < b.nx ? 1.0 : 2.0, gW = i > 0 ? 1.0 : 2.0;
    const double gN = j + 1 < b.ny ? 1.0 : 2.0, gS = j > 0 ? 1.0 : 2.0;
    const bool ux = i >= 1, vy = j >= 1;
    const int c0 = (ty + 1) * HX + (tx + 1);
    int idx = own ? box_index(b, i, j, k0) : 0;
    // values at k-1 carried in registers (the guard plane below k = 0 holds zeros)
    double P0 = own ? xp[idx - sz] : 0.0, M0 = own ? c.mu[idx - sz] : 0.0;
    double XZ1 = own ? c.mxz[idx] : 0.0, YZ1 = own ? c.myz[idx] : 0.0;
    load_vel(k0 - 1);
    load_vel(k0);
    for (int k = k0; k < k1; ++k, idx += sz) {
        load_vel(k + 1);
        load_mu(k);
        __syncthreads();
        if (own) {
            const double *Um = sU[slot(k - 1)], *U0 = sU[slot(k)], *Up = sU[slot(k + 1)];
            const double *Vm = sV[slot(k - 1)], *V0 = sV[slot(k)], *Vp = sV[slot(k + 1)];
            const double *Wm = sW[slot(k - 1)], *W0 = sW[slot(k)], *Wp = sW[slot(k + 1)];
            const double U1 = U0[c0], V1 = V0[c0], W1 = W0[c0];
            const double W2 = Wp[c0];
            const double XZ2 = c.mxz[idx + sz], YZ2 = c.myz[idx + sz];
            const double P1 = xp[idx], M1 = sM[c0];
            const bool top = k + 1 < b.nz, bot = k > 0;
            const double gT = top ? 1.0 : 2.0, gB = bot ? 1.0 : 2.0;
            // x-momentum
            if (ux) {
                const double uE = U0[c0 + 1], uW = U0[c0 - 1];
                const double uN = j + 1 < b.ny ? U0[c0 + HX] : 0.0, uS = j > 0 ? U0[c0 - HX] : 0.0;
                const double uT = top ? Up[c0] : 0.0, uB = bot ? Um[c0] : 0.0;
                const double m0 = sM[c0 - 1], mN = sXY[c0 + HX], mS = sXY[c0];
                const double dvN = V0[c0 + HX] - V0[c0 + HX - 1], dvS = V1 - V0[c0 - 1];
                const double dwT = W2 - Wp[c0 - 1], dwB = W1 - W0[c0 - 1];
                double lap = 2.0 * (M1 * uE + m0 * uW) * ihx * ihx
                           + (mN * (uN * ihy + dvN * ihx) - mS * (-uS * ihy + dvS * ihx)) * ihy
                           + (XZ2 * (uT * ihz + dwT * ihx) - XZ1 * (-uB * ihz + dwB * ihx)) * ihz;
                double dg = 2.0 * (m0 + M1) * ihx * ihx + (mN * gN + mS * gS) * ihy * ihy + (XZ2 * gT + XZ1 * gB) * ihz * ihz;
                double r = (c.mass[0][idx] + th * dg) * U1 - th * lap + (P1 - xp[idx - 1]) * ihx;
                yu[idx] = fu ? fu[idx] - r : r;
            }
            // y-momentum
            if (vy) {
                const double vN = V0[c0 + HX], vS = V0[c0 - HX];
                const double vE = i + 1 < b.nx ? V0[c0 + 1] : 0.0, vW = i > 0 ? V0[c0 - 1] : 0.0;
                const double vT = top ? Vp[c0] : 0.0, vB = bot ? Vm[c0] : 0.0;
                const double m0 = sM[c0 - HX], mE = sXY[c0 + 1], mW = sXY[c0];
                const double duE = U0[c0 + 1] - U0[c0 + 1 - HX], duW = U1 - U0[c0 - HX];
                const double dwT = W2 - Wp[c0 - HX], dwB = W1 - W0[c0 - HX];
                double lap = 2.0 * (M1 * vN + m0 * vS) * ihy * ihy
                           + (mE * (vE * ihx + duE * ihy) - mW * (-vW * ihx + duW * ihy)) * ihx
                           + (YZ2 * (vT * ihz + dwT * ihy) - YZ1 * (-vB * ihz + dwB * ihy)) * ihz;
                double dg = 2.0 * (m0 + M1) * ihy * ihy + (mE * gE + mW * gW) * ihx * ihx + (YZ2 * gT + YZ1 * gB) * ihz * ihz;
                double r = (c.mass[1][idx] + th * dg) * V1 - th * lap + (P1 - xp[idx - sy]) * ihy;
                yv[idx] = fv ? fv[idx] - r : r;
            }
            // z-momentum
            if (bot) {
                const double W0c = Wm[c0];
                const double wE = i + 1 < b.nx ? W0[c0 + 1] : 0.0, wW = i > 0 ? W0[c0 - 1] : 0.0;
                const double wN = j + 1 < b.ny ? W0[c0 + HX] : 0.0, wS = j > 0 ? W0[c0 - HX] : 0.0;
                const double mE = c.mxz[idx + 1], mN = c.myz[idx + sy];
                const double duE = U0[c0 + 1] - Um[c0 + 1], duW = U1 - Um[c0];
                const double dvN = V0[c0 + HX] - Vm[c0 + HX], dvS = V1 - Vm[c0];
                double lap = 2.0 * (M1 * W2 + M0 * W0c) * ihz * ihz
                           + (mE * (wE * ihx + duE * ihz) - XZ1 * (-wW * ihx + duW * ihz)) * ihx
                           + (mN * (wN * ihy + dvN * ihz) - YZ1 * (-wS * ihy + dvS * ihz)) * ihy;
                double dg = 2.0 * (M0 + M1) * ihz * ihz + (mE * gE + XZ1 * gW) * ihx * ihx + (mN * gN + YZ1 * gS) * ihy * ihy;
                double r = (c.mass[2][idx] + th * dg) * W1 - th * lap + (P1 - P0) * ihz;
                yw[idx] = fw ? fw[idx] - r : r;
            }
            // continuity
            {
                double d = (U0[c0 + 1] - U1) * ihx + (V0[c0 + HX] - V1) * ihy + (W2 - W1) * ihz;
                yp[idx] = fp ? fp[idx] + d : -d;
            }
            P0 = P1;
            M0 = M1;
            XZ1 = XZ2;
            YZ1 = YZ2;
        }
        __syncthreads();                        // the next step overwrites plane k-1's slot and sM, sXY
    }
}

// z-momentum rows of the open top's faces (k = nz), which the z-marching matvec
// does not visit: one thread per (i, j), same row formulas as k_apply.
__global__ void __launch_bounds__(kBlock) k_apply_top3(Box b, VelCoef<double> c,
        const double *__restrict__ xu, const double *__restrict__ xv, const double *__restrict__ xw,
        const double *__restrict__ xp, const double *__restrict__ fw, double *__restrict__ yw) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= b.nx * b.ny) return;
    const int i = t % b.nx, j = t / b.nx;
    const int idx = box_index(b, i, j, b.nz);
    double off, dg;
    row_w<double>(b, idx, i, j, b.nz, xu, xv, xw, VALID_U | VALID_V | VALID_W, c, off, dg);
    const double r = dg * xw[idx] + off + (-xp[idx - b.plane] - xp[idx - b.plane]) * b.ihz;
    yw[idx] = fw ? fw[idx] - r : r;
}

// ---------------------------------------------------------------- velocity multigrid
// t = r - A e on interior faces (0 elsewhere), all components.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_vel_residual(Box b, VelCoef<R> c,
        const R *__restrict__ eu, const R *__restrict__ ev, const R *__restrict__ ew,
        const R *__restrict__ ru, const R *__restrict__ rv, const R *__restrict__ rw,
        R *__restrict__ tu, R *__restrict__ tv, R *__restrict__ tw) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    const int all = VALID_U | VALID_V | VALID_W;
    R off, dg;
    R t = 0;
    if (is_ux(b, i, j, k)) { row_u<DIM, R>(b, idx, i, j, k, eu, ev, ew, all, c, off, dg); t = ru[idx] - (dg * eu[idx] + off); }
    tu[idx] = t;
    t = 0;
    if (is_vy(b, i, j, k)) { row_v<DIM, R>(b, idx, i, j, k, eu, ev, ew, all, c, off, dg); t = rv[idx] - (dg * ev[idx] + off); }
    tv[idx] = t;
    if (DIM == 3) {
        t = 0;
        if (is_wz(b, i, j, k)) { row_w<R>(b, idx, i, j, k, eu, ev, ew, all, c, off, dg); t = rw[idx] - (dg * ew[idx] + off); }
        tw[idx] = t;
    }
}

// One colour of a red-black Gauss-Seidel pass on one velocity component:
// e_c = (r - off) / diag on faces with (i+j+k) % 2 == colour.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_vel_gs(Box b, VelCoef<R> c, int comp, int colour, int valid,
        R *eu, R *ev, R *ew, const R *__restrict__ ru, const R *__restrict__ rv, const R *__restrict__ rw) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    if (((i + j + k) & 1) != colour) return;
    R off, dg;
    if (comp == 0) {
        if (!is_ux(b, i, j, k)) return;
        row_u<DIM, R>(b, idx, i, j, k, eu, ev, ew, valid, c, off, dg);
        eu[idx] = (ru[idx] - off) / dg;
    } else if (comp == 1) {
        if (!is_vy(b, i, j, k)) return;
        row_v<DIM, R>(b, idx, i, j, k, eu, ev, ew, valid, c, off, dg);
        ev[idx] = (rv[idx] - off) / dg;
    } else {
        if (!is_wz(b, i, j, k)) return;
        row_w<R>(b, idx, i, j, k, eu, ev, ew, valid, c, off, dg);
        ew[idx] = (rw[idx] - off) / dg;
    }
}

// Face restriction for component comp: the coarse face averages the fine faces
// it covers with weight 2 for the coincident ones and 1 for those half a coarse
// cell to either side (2D: (1/8)[2 2 1 1 1 1]); coarse wall faces get 0.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_face_restrict(Box fb, Box cb, int comp,
        const R *__restrict__ f, R *__restrict__ c) {
    int idx = box_thread_index();
    if (idx >= cb.nb) return;
    int I, J, K;
    decompose(cb, idx, I, J, K);
    bool inner = comp == 0 ? is_ux(cb, I, J, K) : comp == 1 ? is_vy(cb, I, J, K) : is_wz(cb, I, J, K);
    if (!inner) { c[idx] = R(0); return; }
    const int s[3] = {1, fb.px, fb.plane};
    int base = box_index(fb, 2 * I, 2 * J, DIM == 3 ? 2 * K : 0);
    const int sn = s[comp];
    const int CI[3] = {I, J, K}, nfine[3] = {fb.nx, fb.ny, fb.nz};
    // the fine face half a coarse cell below coarse face 0 wraps on a periodic axis
    const int snm = (fb.per[comp] && CI[comp] == 0) ? (nfine[comp] - 1) * sn : -sn;
    const int t1 = comp == 0 ? s[1] : s[0];
    const int t2 = comp == 2 ? s[1] : s[2];
    R acc = 0;
    const int n2 = DIM == 3 ? 2 : 1;
    for (int a2 = 0; a2 < n2; ++a2)
        for (int a1 = 0; a1 < 2; ++a1) {
            int q = base + a1 * t1 + a2 * t2;
            acc += R(2) * f[q] + f[q + snm] + f[q + sn];
        }
    c[idx] = acc * (DIM == 3 ? R(1.0 / 16.0) : R(1.0 / 8.0));
}

// Face prolongation for component comp, added to the fine correction: linear
// along the face normal, constant across; fine wall faces untouched.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_face_prolong_add(Box fb, Box cb, int comp,
        const R *__restrict__ c, R *__restrict__ f) {
    int idx = box_thread_index();
    if (idx >= fb.nb) return;
    int i, j, k;
    decompose(fb, idx, i, j, k);
    bool inner = comp == 0 ? is_ux(fb, i, j, k) : comp == 1 ? is_vy(fb, i, j, k) : is_wz(fb, i, j, k);
    if (!inner) return;
    int ci[3] = {i >> 1, j >> 1, DIM == 3 ? (k >> 1) : 0};
    int fi[3] = {i, j, k};
    const int cs[3] = {1, cb.px, cb.plane};
    int q = box_index(cb, ci[0], ci[1], ci[2]);
    const int ncs[3] = {cb.nx, cb.ny, cb.nz};
    // the coarse face above the last one is coarse face 0 on a periodic axis
    const int up = (cb.per[comp] && ci[comp] == ncs[comp] - 1) ? (1 - ncs[comp]) * cs[comp] : cs[comp];
    R val;
    if ((fi[comp] & 1) == 0) {
        val = c[q];
    } else {
        val = R(0.5) * (c[q] + c[q + up]);
    }
    f[idx] += val;
}

// ---------------------------------------------------------------- pressure multigrid
// -L_rho phi = -D beta G phi at cell (i, j, k) (box point idx); beta is zero on
// wall faces, so the Neumann walls need no branch; periodic axes wrap (Nbr).
template <int DIM, class R, bool PER = true>
__device__ inline void prow(const Box &b, int idx, int i, int j, int k, const R *e, const R *bx, const R *by,
                            const R *bz, R &off, R &diag) {
    const Nbr o = nbr<PER>(b, i, j, k);
    const R ix2 = R(b.ihx * b.ihx), iy2 = R(b.ihy * b.ihy), iz2 = R(b.ihz * b.ihz);
    R wW = bx[idx] * ix2, wE = bx[idx + o.xp] * ix2;
    R wS = by[idx] * iy2, wN = by[idx + o.yp] * iy2;
    off = wW * e[idx + o.xm] + wE * e[idx + o.xp] + wS * e[idx + o.ym] + wN * e[idx + o.yp];
    diag = wW + wE + wS + wN;
    if (DIM == 3) {
        R wB = bz[idx] * iz2, wT = bz[idx + o.zp] * iz2;
        off += wB * e[idx + o.zm] + wT * e[idx + o.zp];
        diag += wB + wT;
    }
}

// Red-black SOR update of one point: the Gauss-Seidel value gs (its equation
// solved with the neighbours held) relaxed by omega from the old value.
// omega = 1 is plain Gauss-Seidel and returns gs itself (no blend), so that its
// results stay those of the unrelaxed sweep.
template <class R>
__device__ inline R sor(R old, R gs, R omega) {
    return omega == R(1) ? gs : old + omega * (gs - old);
}

template <int DIM, class R, bool PER>
__global__ void __launch_bounds__(kBlock) k_p_gs(Box b, int colour, int zero_guess, R omega, R *e,
        const R *__restrict__ r, const R *__restrict__ bx, const R *__restrict__ by,
        const R *__restrict__ bz) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    if (!is_cell(b, i, j, k)) return;
    if (((i + j + k) & 1) != colour) {
        // a relaxed update reads the point's own old value: after a zero guess
        // the points of the other colour must read as zero too
        if (zero_guess && omega != R(1)) e[idx] = R(0);
        return;
    }
    R off, dg;
    prow<DIM, R, PER>(b, idx, i, j, k, e, bx, by, bz, off, dg);
    if (zero_guess) off = R(0);
    e[idx] = dg > R(0) ? sor(zero_guess ? R(0) : e[idx], (r[idx] + off) / dg, omega) : R(0);
}

// Coarse right-hand side: average over the 2^d children of the fine residual
// r - (-L_rho) e.
template <int DIM, class R, bool PER>
__global__ void __launch_bounds__(kBlock) k_p_residual_restrict(Box fb, Box cb, const R *__restrict__ e,
        const R *__restrict__ r, const R *__restrict__ bx, const R *__restrict__ by,
        const R *__restrict__ bz, R *__restrict__ rc) {
    int idx = box_thread_index();
    if (idx >= cb.nb) return;
    int I, J, K;
    decompose(cb, idx, I, J, K);
    if (!is_cell(cb, I, J, K)) { rc[idx] = R(0); return; }
    R acc = 0;
    const int n2 = DIM == 3 ? 2 : 1;
    for (int dk = 0; dk < n2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const int fi = 2 * I + di, fj = 2 * J + dj, fk = DIM == 3 ? 2 * K + dk : 0;
                int q = box_index(fb, fi, fj, fk);
                R off, dg;
                prow<DIM, R, PER>(fb, q, fi, fj, fk, e, bx, by, bz, off, dg);
                acc += r[q] - (dg * e[q] - off);
            }
    rc[idx] = acc * (DIM == 3 ? R(0.125) : R(0.25));
}

// 3D residual + restriction marching in z: a thread owns one coarse column
// (I, J) and a chunk of kc coarse planes; the fine values of its 2x2 fine
// columns at the four planes a coarse plane needs (2K-1 .. 2K+2) stay in
// registers, so each fine plane is read once instead of twice (the per-cell
// kernel above re-reads the planes shared with the coarse cells below and
// above) and the upper z coefficient of plane 2K+1 is reused; the fine columns
// just west and east of a thread's pair come from the neighbouring lanes
// (shuffles), not from memory.  Same formulas and summation order as
// k_p_residual_restrict.
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_p_residual_restrict3_z(Box fb, Box cb, int kc,
        const R *__restrict__ e, const R *__restrict__ r, const R *__restrict__ bx,
        const R *__restrict__ by, const R *__restrict__ bz, R *__restrict__ rc) {
    const int G = gridDim.x * gridDim.y * gridDim.z;
    int t = xcd_swizzle(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), G);
    const int bx_ = t % gridDim.x;
    t /= gridDim.x;
    const int by_ = t % gridDim.y, bz_ = t / gridDim.y;
    static_assert(TX == 64, "one wavefront per row of the tile: x-neighbours by lane shuffles");
    const int lane = (int)(threadIdx.x % TX);
    const int I0 = bx_ * TX + lane, J0 = by_ * TY + (int)(threadIdx.x / TX);
    // lanes past the last coarse column or row take part in the shuffles with the
    // values of a valid column and store nothing
    const bool active = I0 < cb.nx && J0 < cb.ny;
    const int I = min(I0, cb.nx - 1), J = min(J0, cb.ny - 1);
    const bool east_in = I0 + 1 < cb.nx;                 // lane + 1 holds the column to the east
    const int K0 = bz_ * kc, K1 = min(K0 + kc, cb.nz);
    if (K0 >= K1) return;                                // uniform over the block
    const int sy = fb.px, sz = fb.plane;
    const R ix2 = R(fb.ihx * fb.ihx), iy2 = R(fb.ihy * fb.ihy), iz2 = R(fb.ihz * fb.ihz);
    // fine columns c = di + 2 dj at offsets co[c] from the (2I, 2J) column
    const int co[4] = {0, 1, sy, sy + 1};
    int q = box_index(fb, 2 * I, 2 * J, 2 * K0);     // fine point (2I, 2J, 2K)
    // e of the four columns at planes 2K-1 (em), 2K (ea), 2K+1 (eb), 2K+2 (ep); the
    // guard plane below plane 0 and the padding plane nz hold zeros
    R em[4], ea[4], eb[4], ep[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        em[c] = e[q + co[c] - sz];
        ea[c] = e[q + co[c]];
        eb[c] = e[q + co[c] + sz];
        ep[c] = e[q + co[c] + 2 * sz];
    }
    for (int K = K0; K < K1; ++K, q += 2 * sz) {
        R acc = 0;
#pragma unroll
        for (int dk = 0; dk < 2; ++dk) {
            const R *lo = dk == 0 ? em : ea;
            const R *ce = dk == 0 ? ea : eb;
            const R *hi = dk == 0 ? eb : ep;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                // the fine columns west and east of this thread's pair are the
                // neighbouring lanes' east and west columns
                const R from_w = __shfl_up(ce[1 + 2 * dj], 1, 64);
                const R from_e = __shfl_down(ce[2 * dj], 1, 64);
#pragma unroll
                for (int di = 0; di < 2; ++di) {
                    const int c = di + 2 * dj;
                    const int p = q + co[c] + dk * sz;
                    R eW, eE;
                    if (di == 1) {
                        eW = ce[c - 1];
                        eE = east_in && lane < 63 ? from_e : e[p + 1];
                    } else {
                        eW = lane > 0 ? from_w : e[p - 1];
                        eE = ce[c + 1];
                    }
                    const R eS = dj == 1 ? ce[c - 2] : e[p - sy];
                    const R eN = dj == 0 ? ce[c + 2] : e[p + sy];
                    const R wW = bx[p] * ix2, wE = bx[p + 1] * ix2;
                    const R wS = by[p] * iy2, wN = by[p + sy] * iy2;
                    R off = wW * eW + wE * eE + wS * eS + wN * eN;
                    R dg = wW + wE + wS + wN;
                    const R wB = bz[p] * iz2, wT = bz[p + sz] * iz2;
                    off += wB * lo[c] + wT * hi[c];
                    dg += wB + wT;
                    acc += r[p] - (dg * ce[c] - off);
                }
            }
        }
        if (active) rc[box_index(cb, I, J, K)] = acc * R(0.125);
        if (K + 1 < K1) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                em[c] = eb[c];
                ea[c] = ep[c];
                eb[c] = e[q + co[c] + 3 * sz];
                ep[c] = e[q + co[c] + 4 * sz];
            }
        }
    }
}

// Prolonged coarse correction at fine cell (i,j,k).  lin == 0: the parent's
// value (piecewise constant).  lin == 1: bi/trilinear interpolation between the
// cell centres, weights 3/4 (parent) and 1/4 (the coarse neighbour on the
// child's side) per axis; beyond a wall the parent is mirrored, along a
// periodic axis the neighbour wraps (PER = false: walls only, for the
// z-marching kernels, which periodic levels never reach).
template <int DIM, class R, bool PER = true>
__device__ inline R prolong_value(const Box &cb, const R *ec, int i, int j, int k, int lin) {
    const int I = i >> 1, J = j >> 1, K = DIM == 3 ? (k >> 1) : 0;
    if (!lin) return ec[box_index(cb, I, J, K)];
    int I2 = (i & 1) ? I + 1 : I - 1;
    int J2 = (j & 1) ? J + 1 : J - 1;
    I2 = (PER && cb.per[0]) ? (I2 + cb.nx) % cb.nx : (I2 < 0 ? 0 : (I2 >= cb.nx ? cb.nx - 1 : I2));
    J2 = (PER && cb.per[1]) ? (J2 + cb.ny) % cb.ny : (J2 < 0 ? 0 : (J2 >= cb.ny ? cb.ny - 1 : J2));
    const R a = R(0.75), b = R(0.25);
    if (DIM == 2) {
        return a * (a * ec[box_index(cb, I, J, 0)] + b * ec[box_index(cb, I2, J, 0)])
             + b * (a * ec[box_index(cb, I, J2, 0)] + b * ec[box_index(cb, I2, J2, 0)]);
    }
    int K2 = (k & 1) ? K + 1 : K - 1;
    K2 = (PER && cb.per[2]) ? (K2 + cb.nz) % cb.nz : (K2 < 0 ? 0 : (K2 >= cb.nz ? cb.nz - 1 : K2));
    R p0 = a * (a * ec[box_index(cb, I, J, K)] + b * ec[box_index(cb, I2, J, K)])
         + b * (a * ec[box_index(cb, I, J2, K)] + b * ec[box_index(cb, I2, J2, K)]);
    R p1 = a * (a * ec[box_index(cb, I, J, K2)] + b * ec[box_index(cb, I2, J, K2)])
         + b * (a * ec[box_index(cb, I, J2, K2)] + b * ec[box_index(cb, I2, J2, K2)]);
    return a * p0 + b * p1;
}

// Fine correction += prolonged coarse correction (see prolong_value).
template <int DIM, class R, bool PER>
__global__ void __launch_bounds__(kBlock) k_p_prolong_add(Box fb, Box cb, int lin, const R *__restrict__ c,
        R *__restrict__ f) {
    int idx = box_thread_index();
    if (idx >= fb.nb) return;
    int i, j, k;
    decompose(fb, idx, i, j, k);
    if (!is_cell(fb, i, j, k)) return;
    f[idx] += prolong_value<DIM, R, PER>(cb, c, i, j, k, lin);
}

// One colour pass of the first red-black sweep after a coarse correction on a
// flat level (walls only), with the prolongation folded in: every cell reads as
// e + P(ec) (prolong_value) until its colour is updated, points outside the
// domain as the zero they hold.  Colour 0 reads its neighbours and, relaxed, its
// own old value that way; colour 1 only its own old value (its neighbours are
// colour 0 and already updated).  Same values, summed in the same order, as
// k_p_prolong_add followed by the two k_p_gs passes, with one launch less.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_p_gs_ec(Box b, int colour, R omega, R *e,
        const R *__restrict__ r, const R *__restrict__ bx, const R *__restrict__ by,
        const R *__restrict__ bz, Box cb, int lin, const R *__restrict__ ec) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    if (!is_cell(b, i, j, k) || ((i + j + k) & 1) != colour) return;
    auto val = [&](int q, int ii, int jj, int kk) -> R {
        if (ii < 0 || ii >= b.nx || jj < 0 || jj >= b.ny || kk < 0 || kk >= b.nz) return e[q];
        return e[q] + prolong_value<DIM, R, false>(cb, ec, ii, jj, kk, lin);
    };
    R off, dg;
    if (colour == 0) {
        const int sy = b.px, sz = b.plane;
        const R ix2 = R(b.ihx * b.ihx), iy2 = R(b.ihy * b.ihy), iz2 = R(b.ihz * b.ihz);
        R wW = bx[idx] * ix2, wE = bx[idx + 1] * ix2;
        R wS = by[idx] * iy2, wN = by[idx + sy] * iy2;
        off = wW * val(idx - 1, i - 1, j, k) + wE * val(idx + 1, i + 1, j, k) + wS * val(idx - sy, i, j - 1, k)
            + wN * val(idx + sy, i, j + 1, k);
        dg = wW + wE + wS + wN;
        if (DIM == 3) {
            R wB = bz[idx] * iz2, wT = bz[idx + sz] * iz2;
            off += wB * val(idx - sz, i, j, k - 1) + wT * val(idx + sz, i, j, k + 1);
            dg += wB + wT;
        }
    } else {
        prow<DIM, R, false>(b, idx, i, j, k, e, bx, by, bz, off, dg);
    }
    e[idx] = dg > R(0) ? sor(omega == R(1) ? R(0) : val(idx, i, j, k), (r[idx] + off) / dg, omega) : R(0);
}

// Coarsest pressure level: e = M r with M the dense pseudo-inverse of the
// level's Neumann operator (it also projects out the constant).  One block of
// 1024 threads, 16 per row (dense_row).
// Row t of M rs, computed by 16 lanes: lane g of the group sums the contiguous
// segment q = g*L .. g*L + L - 1 (L = ceil(n/16)) in order, then the 16 partial
// sums are added pairwise (lanes g and g^8, then ^4, ^2, ^1).  Every lane of the
// group returns the row's value.  blockDim.x is a multiple of 64, so a group
// never straddles wavefronts and all of its lanes take part.
template <class R, class MP>
__device__ inline R dense_row(MP M, const R *rs, int n, int t, int g) {
    const int L = (n + 15) >> 4;
    R acc = 0;
    if (t < n) {
        const int q0 = g * L, q1 = min(q0 + L, n);
        for (int q = q0; q < q1; ++q) acc += M[(size_t)t * n + q] * rs[q];
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    return acc;
}

template <class R>
__global__ void __launch_bounds__(1024) k_dense_solve(int n, const R *__restrict__ M, const int *__restrict__ map,
        const R *__restrict__ r, R *__restrict__ e) {
    extern __shared__ unsigned char smem_raw[];
    R *rs = reinterpret_cast<R *>(smem_raw);
    for (int t = threadIdx.x; t < n; t += blockDim.x) rs[t] = r[map[t]];
    __syncthreads();
    const int g = threadIdx.x & 15, rows = blockDim.x >> 4;
    for (int t0 = 0; t0 < n; t0 += rows) {
        const int t = t0 + (threadIdx.x >> 4);
        const R v = dense_row<R, const R *__restrict__>(M, rs, n, t, g);
        if (t < n && g == 0) e[map[t]] = v;
    }
}

// ---------------------------------------------------------------- small levels in one workgroup
// Below a few thousand cells a pressure level costs one launch per colour pass
// when it is cycled pass by pass, and under W-cycles the small levels are
// visited 2^l times per cycle, so their launches dominate.  One workgroup runs
// the whole cycle from such a level down instead: the iterate and right-hand
// side of every level, and the face coefficients of every level but the first
// (read from global memory, where they stay in L2), live in LDS, and every
// pass ends at a workgroup barrier.  The host lists the passes in the order the
// pass-by-pass cycle launches them; their arithmetic is that of k_p_gs,
// k_p_residual_restrict, k_p_prolong_add and k_dense_solve.
enum { SOP_GS = 0, SOP_RESTRICT = 1, SOP_PROLONG = 2, SOP_DENSE = 3, SOP_ZERO = 4 };
constexpr int kSmallMaxLev = 8;
constexpr int kSmallThreads = 1024;
constexpr int kSmallCached = 2;     // first-level cells per thread and colour set up once per launch

// One pass: x = kind, y = level (0 = the first small level), z = colour of a
// smoothing pass, w = its zero-guess flag (0 no, 1 yes, 2 the launch's).
struct SmallOp {
    int kind, level, colour, zero_guess;
};

template <class R>
struct SmallMG {
    int nl;                          // levels in LDS: the first small level and all coarser
    Box b[kSmallMaxLev];
    int off_e[kSmallMaxLev];         // LDS element offset of box point 0 of each level's iterate
    int off_r[kSmallMaxLev];         // ... of its right-hand side
    int off_b[kSmallMaxLev];         // ... of its three face coefficients (level >= 1), nb + plane apart
    int stride_b[kSmallMaxLev];
    const R *gbeta[kSmallMaxLev][3]; // global face coefficients of each level
    const R *dense;                  // coarsest level: dense pseudo-inverse (global), n x n
    int ndense;
    int off_dense;                   // LDS copy of the dense matrix (-1: read from global)
    int off_rs;                      // LDS staging of the coarsest right-hand side (ndense)
    int lin;                         // prolongation (see prolong_value)
    int lds_elems;                   // LDS size in elements of R
    R omega;                         // smoother over-relaxation (1: Gauss-Seidel)
};

template <class R, class BP, bool PER>
__device__ inline void small_gs(const Box &b, R *e, const R *r, BP bx, BP by, BP bz, int colour, bool zg,
                                R omega) {
    const int hx = (b.nx + 1) >> 1;
    const int total = hx * b.ny * b.nz;
    for (int t = threadIdx.x; t < total; t += kSmallThreads) {
        const int ii = t % hx, jk = t / hx;
        const int j = jk % b.ny, k = jk / b.ny;
        const int i = 2 * ii + ((j + k + colour) & 1);
        if (zg && omega != R(1)) {
            const int i2 = 2 * ii + ((j + k + colour + 1) & 1);     // the other colour (see k_p_gs)
            if (i2 < b.nx) e[box_index(b, i2, j, k)] = R(0);
        }
        if (i >= b.nx) continue;
        const int idx = box_index(b, i, j, k);
        R off, dg;
        prow<3, R, PER>(b, idx, i, j, k, e, bx, by, bz, off, dg);
        if (zg) off = R(0);
        e[idx] = dg > R(0) ? sor(zg ? R(0) : e[idx], (r[idx] + off) / dg, omega) : R(0);
    }
}

template <class R, class BP, bool PER>
__device__ inline void small_restrict(const Box &fb, const Box &cb, const R *e, const R *r, BP bx, BP by, BP bz,
                                      R *rc) {
    const int total = cb.nx * cb.ny * cb.nz;
    for (int t = threadIdx.x; t < total; t += kSmallThreads) {
        const int I = t % cb.nx, JK = t / cb.nx;
        const int J = JK % cb.ny, K = JK / cb.ny;
        R acc = 0;
#pragma unroll 1
        for (int dk = 0; dk < 2; ++dk)
#pragma unroll 1
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll 1
                for (int di = 0; di < 2; ++di) {
                    const int q = box_index(fb, 2 * I + di, 2 * J + dj, 2 * K + dk);
                    R off, dg;
                    prow<3, R, PER>(fb, q, 2 * I + di, 2 * J + dj, 2 * K + dk, e, bx, by, bz, off, dg);
                    acc += r[q] - (dg * e[q] - off);
                }
        rc[box_index(cb, I, J, K)] = acc * R(0.125);
    }
}

template <class R, class MP>
__device__ inline void small_dense(const Box &b, int n, MP M, R *rs, const R *r, R *e) {
    for (int t = threadIdx.x; t < n; t += kSmallThreads) {
        const int i = t % b.nx, jk = t / b.nx;
        rs[t] = r[box_index(b, i, jk % b.ny, jk / b.ny)];
    }
    __syncthreads();
    const int g = threadIdx.x & 15;
    for (int t0 = 0; t0 < n; t0 += kSmallThreads / 16) {
        const int t = t0 + (threadIdx.x >> 4);
        const R v = dense_row<R, MP>(M, rs, n, t, g);
        if (t < n && g == 0) {
            const int i = t % b.nx, jk = t / b.nx;
            e[box_index(b, i, jk % b.ny, jk / b.ny)] = v;
        }
    }
}

template <class R, bool PER>
__global__ void __launch_bounds__(kSmallThreads) k_p_small_cycle(SmallMG<R> m, const SmallOp *__restrict__ ops,
        int nops, int zero_guess, R *__restrict__ e, const R *__restrict__ r) {
    extern __shared__ unsigned char smem_raw[];
    R *S = reinterpret_cast<R *>(smem_raw);
    // The first level's smoothing passes dominate the cycle and are bound by the
    // instructions of one CU.  When that level has walls on every side and each
    // thread has at most kSmallCached of its cells per colour, the thread's cells
    // (box index, or -1) and their weights beta/h^2 are set up once, before the
    // LDS fills so that their loads overlap them; the passes then only load the
    // iterate from LDS (the same products and sums as prow, so the results do
    // not change).
    const Box &b0 = m.b[0];
    const int hx0 = (b0.nx + 1) >> 1, half0 = hx0 * b0.ny * b0.nz;
    const bool fast0 = !PER && b0.dim == 3 && half0 <= kSmallThreads * kSmallCached;
    int q0[2][kSmallCached];
    R w0[2][kSmallCached][6];
    if (fast0) {
        const R ix2 = R(b0.ihx * b0.ihx), iy2 = R(b0.ihy * b0.ihy), iz2 = R(b0.ihz * b0.ihz);
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
            for (int q = 0; q < kSmallCached; ++q) {
                const int t = threadIdx.x + q * kSmallThreads;
                q0[col][q] = -1;
#pragma unroll
                for (int a = 0; a < 6; ++a) w0[col][q][a] = R(0);
                if (t >= half0) continue;
                const int ii = t % hx0, jk = t / hx0;
                const int j = jk % b0.ny, k = jk / b0.ny;
                const int i = 2 * ii + ((j + k + col) & 1);
                if (i >= b0.nx) continue;
                const int idx = box_index(b0, i, j, k);
                q0[col][q] = idx;
                w0[col][q][0] = m.gbeta[0][0][idx] * ix2;
                w0[col][q][1] = m.gbeta[0][0][idx + 1] * ix2;
                w0[col][q][2] = m.gbeta[0][1][idx] * iy2;
                w0[col][q][3] = m.gbeta[0][1][idx + b0.px] * iy2;
                w0[col][q][4] = m.gbeta[0][2][idx] * iz2;
                w0[col][q][5] = m.gbeta[0][2][idx + b0.plane] * iz2;
            }
    }
    for (int t = threadIdx.x; t < m.lds_elems; t += kSmallThreads) S[t] = R(0);
    __syncthreads();
    for (int t = threadIdx.x; t < b0.nb; t += kSmallThreads) {
        S[m.off_r[0] + t] = r[t];
        if (!zero_guess) S[m.off_e[0] + t] = e[t];
    }
    for (int l = 1; l < m.nl; ++l)
        for (int a = 0; a < 3; ++a) {
            R *dst = S + m.off_b[l] + a * m.stride_b[l];
            const R *src = m.gbeta[l][a];
            for (int t = threadIdx.x; t < m.b[l].nb; t += kSmallThreads) dst[t] = src[t];
        }
    if (m.off_dense >= 0)
        for (int t = threadIdx.x; t < m.ndense * m.ndense; t += kSmallThreads) S[m.off_dense + t] = m.dense[t];
    __syncthreads();
    for (int o = 0; o < nops; ++o) {
        const SmallOp op = ops[o];
        const int l = op.level;
        const Box &b = m.b[l];
        R *E = S + m.off_e[l];
        R *Rr = S + m.off_r[l];
        if (op.kind == SOP_GS) {
            const bool zg = op.zero_guess == 2 ? zero_guess != 0 : op.zero_guess != 0;
            if (l == 0 && fast0) {
                const int col = op.colour, sy = b.px, sz = b.plane;
#pragma unroll
                for (int q = 0; q < kSmallCached; ++q) {
                    const int idx = col ? q0[1][q] : q0[0][q];
                    if (zg && m.omega != R(1)) {                  // the other colour reads as zero (see k_p_gs)
                        const int i2 = col ? q0[0][q] : q0[1][q];
                        if (i2 >= 0) E[i2] = R(0);
                    }
                    if (idx < 0) continue;
                    const R wW = col ? w0[1][q][0] : w0[0][q][0], wE = col ? w0[1][q][1] : w0[0][q][1];
                    const R wS = col ? w0[1][q][2] : w0[0][q][2], wN = col ? w0[1][q][3] : w0[0][q][3];
                    const R wB = col ? w0[1][q][4] : w0[0][q][4], wT = col ? w0[1][q][5] : w0[0][q][5];
                    R off = wW * E[idx - 1] + wE * E[idx + 1] + wS * E[idx - sy] + wN * E[idx + sy];
                    R dg = wW + wE + wS + wN;
                    off += wB * E[idx - sz] + wT * E[idx + sz];
                    dg += wB + wT;
                    if (zg) off = R(0);
                    E[idx] = dg > R(0) ? sor(zg ? R(0) : E[idx], (Rr[idx] + off) / dg, m.omega) : R(0);
                }
            } else if (l == 0) {
                small_gs<R, const R *__restrict__, PER>(b, E, Rr, m.gbeta[0][0], m.gbeta[0][1], m.gbeta[0][2], op.colour, zg, m.omega);
            } else {
                const R *B = S + m.off_b[l];
                small_gs<R, const R *, PER>(b, E, Rr, B, B + m.stride_b[l], B + 2 * m.stride_b[l], op.colour, zg, m.omega);
            }
        } else if (op.kind == SOP_RESTRICT) {
            R *rc = S + m.off_r[l + 1];
            if (l == 0) {
                small_restrict<R, const R *__restrict__, PER>(b, m.b[1], E, Rr, m.gbeta[0][0], m.gbeta[0][1], m.gbeta[0][2], rc);
            } else {
                const R *B = S + m.off_b[l];
                small_restrict<R, const R *, PER>(b, m.b[l + 1], E, Rr, B, B + m.stride_b[l], B + 2 * m.stride_b[l], rc);
            }
        } else if (op.kind == SOP_PROLONG) {
            const Box &cb = m.b[l + 1];
            const R *ec = S + m.off_e[l + 1];
            const int total = b.nx * b.ny * b.nz;
            for (int t = threadIdx.x; t < total; t += kSmallThreads) {
                const int i = t % b.nx, jk = t / b.nx;
                const int j = jk % b.ny, k = jk / b.ny;
                E[box_index(b, i, j, k)] += prolong_value<3, R, PER>(cb, ec, i, j, k, m.lin);
            }
        } else if (op.kind == SOP_DENSE) {
            if (m.off_dense >= 0) small_dense<R, const R *>(b, m.ndense, S + m.off_dense, S + m.off_rs, Rr, E);
            else small_dense<R, const R *__restrict__>(b, m.ndense, m.dense, S + m.off_rs, Rr, E);
        } else {   // SOP_ZERO
            for (int t = threadIdx.x; t < b.nb; t += kSmallThreads) E[t] = R(0);
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < b0.nb; t += kSmallThreads) e[t] = S[m.off_e[0] + t];
}

// One full red-black Gauss-Seidel sweep of -L_rho e = r in 3D, both colours in
// one launch.  A block owns a TX x TY column of cells and a chunk of kc planes
// and marches in z.  LDS holds rings of four planes: the old values (tile plus
// a 2-cell x-y halo) and the values after the red half-sweep (tile plus 1).
// Step k loads old plane k+3, does the red half-sweep of plane k+1 and the
// black half-sweep of plane k-1; the three touch disjoint ring slots, so one
// barrier per step suffices and all of a step's global loads are issued
// together.  Red points of the 1-cell halo ring and of the planes next to the
// chunk are recomputed by every block that needs them, so blocks are
// independent and the result equals the global two-pass sweep (colour 0 =
// (i+j+k) even first).  Input and output are separate arrays (ein is never
// written), so blocks never race.  With zero_guess the old values are taken as
// zero (ein is not read).  With ec != nullptr the old value is ein + the
// prolonged coarse correction (see prolong_value): the prolongation is folded
// into the sweep that follows it.
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_p_sweep3(Box b, int kc, int zero_guess, R omega, const R *__restrict__ ein,
        const R *__restrict__ ec, Box cb, int lin, R *__restrict__ eout, const R *__restrict__ r,
        const R *__restrict__ bx, const R *__restrict__ by, const R *__restrict__ bz) {
    constexpr int NT = TX * TY;
    constexpr int EX1 = TX + 2, EY1 = TY + 2, N1 = EX1 * EY1;
    constexpr int EX2 = TX + 4, EY2 = TY + 4, N2 = EX2 * EY2;
    constexpr int P2 = (N2 + NT - 1) / NT, P1 = (N1 + NT - 1) / NT;
    __shared__ R oldp[4][N2];
    __shared__ R newp[4][N1];
    const int tid = threadIdx.x;
    // logical tile from the XCD-swizzled linear block id, z slowest
    const int G = gridDim.x * gridDim.y * gridDim.z;
    int t = xcd_swizzle(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), G);
    const int bx_ = t % gridDim.x;
    t /= gridDim.x;
    const int by_ = t % gridDim.y, bz_ = t / gridDim.y;
    const int i0 = bx_ * TX, j0 = by_ * TY;
    const int k0 = bz_ * kc, k1 = min(k0 + kc, b.nz);
    const int sy = b.px, sz = b.plane;
    const R ix2 = R(b.ihx * b.ihx), iy2 = R(b.ihy * b.ihy), iz2 = R(b.ihz * b.ihz);
    auto slot = [](int k) { return (k + 8) & 3; };
    auto load_old = [&](int k) {
        R v[P2];
#pragma unroll
        for (int p = 0; p < P2; ++p) {
            const int e = tid + p * NT;
            const int i = i0 + (e % EX2) - 2, j = j0 + (e / EX2) - 2;
            v[p] = R(0);
            if (e < N2 && !zero_guess && k >= 0 && k < b.nz && i >= 0 && i < b.nx && j >= 0 && j < b.ny) {
                const int q = box_index(b, i, j, k);
                v[p] = ein[q];
                if (ec) v[p] += prolong_value<3, R, false>(cb, ec, i, j, k, lin);
            }
        }
        R *dst = oldp[slot(k)];
#pragma unroll
        for (int p = 0; p < P2; ++p)
            if (tid + p * NT < N2) dst[tid + p * NT] = v[p];
    };
    // red half-sweep of plane k over the tile plus a 1-cell ring
    auto red = [&](int k) {
        R wv[P1][6], rv[P1];
        bool act[P1];
#pragma unroll
        for (int p = 0; p < P1; ++p) {
            const int e = tid + p * NT;
            const int i = i0 + (e % EX1) - 1, j = j0 + (e / EX1) - 1;
            act[p] = e < N1 && k >= 0 && k < b.nz && i >= 0 && i < b.nx && j >= 0 && j < b.ny &&
                     ((i + j + k) & 1) == 0;
            if (act[p]) {
                const int q = box_index(b, i, j, k);
                wv[p][0] = bx[q] * ix2; wv[p][1] = bx[q + 1] * ix2;
                wv[p][2] = by[q] * iy2; wv[p][3] = by[q + sy] * iy2;
                wv[p][4] = bz[q] * iz2; wv[p][5] = bz[q + sz] * iz2;
                rv[p] = r[q];
            }
        }
        const R *om = oldp[slot(k - 1)], *oc = oldp[slot(k)], *op = oldp[slot(k + 1)];
        R *dst = newp[slot(k)];
#pragma unroll
        for (int p = 0; p < P1; ++p) {
            const int e = tid + p * NT;
            if (e >= N1) continue;
            const int ex = e % EX1, ey = e / EX1;
            const int i = i0 + ex - 1, j = j0 + ey - 1;
            const int o2 = (ey + 1) * EX2 + (ex + 1);
            R v = R(0);
            if (act[p]) {
                R dg = wv[p][0] + wv[p][1] + wv[p][2] + wv[p][3] + wv[p][4] + wv[p][5];
                R off = wv[p][0] * oc[o2 - 1] + wv[p][1] * oc[o2 + 1] + wv[p][2] * oc[o2 - EX2] +
                        wv[p][3] * oc[o2 + EX2] + wv[p][4] * om[o2] + wv[p][5] * op[o2];
                v = dg > R(0) ? sor(oc[o2], (rv[p] + off) / dg, omega) : R(0);
            } else if (k >= 0 && k < b.nz && i >= 0 && i < b.nx && j >= 0 && j < b.ny) {
                v = oc[o2];
            }
            dst[e] = v;
        }
    };
    // black half-sweep of plane k over the tile, written out with the red values
    const int tx = tid % TX, ty = tid / TX;
    const int ib = i0 + tx, jb = j0 + ty;
    auto black = [&](int k) {
        if (ib >= b.nx || jb >= b.ny) return;
        const int q = box_index(b, ib, jb, k);
        const bool blk = ((ib + jb + k) & 1) == 1;
        R w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0, rr = 0;
        if (blk) {
            w0 = bx[q] * ix2; w1 = bx[q + 1] * ix2; w2 = by[q] * iy2; w3 = by[q + sy] * iy2;
            w4 = bz[q] * iz2; w5 = bz[q + sz] * iz2; rr = r[q];
        }
        const R *nm = newp[slot(k - 1)], *nc = newp[slot(k)], *np = newp[slot(k + 1)];
        const int o1 = (ty + 1) * EX1 + (tx + 1);
        R v = nc[o1];
        if (blk) {
            R dg = w0 + w1 + w2 + w3 + w4 + w5;
            R off = w0 * nc[o1 - 1] + w1 * nc[o1 + 1] + w2 * nc[o1 - EX1] + w3 * nc[o1 + EX1] + w4 * nm[o1] + w5 * np[o1];
            v = dg > R(0) ? sor(nc[o1], (rr + off) / dg, omega) : R(0);
        }
        eout[q] = v;
    };
    // prologue: old planes k0-2 .. k0+2 and red planes k0-1, k0
    load_old(k0 - 2);
    load_old(k0 - 1);
    load_old(k0);
    load_old(k0 + 1);
    __syncthreads();
    red(k0 - 1);
    red(k0);
    __syncthreads();
    load_old(k0 + 2);
    __syncthreads();
    for (int k = k0; k <= k1; ++k) {
        if (k + 3 <= k1 + 1) load_old(k + 3);
        if (k + 1 <= k1) red(k + 1);
        if (k - 1 >= k0) black(k - 1);
        __syncthreads();
    }
}


// Two-barrier form of the fused 3D sweep, used on the largest levels (1024-thread
// tiles keep the halo fraction low): one full red-black Gauss-Seidel sweep of
// -L_rho e = r, both colours in one launch.  A block owns a TX x TY column of
// cells and a chunk of kc planes and marches in z with rings of three planes in
// LDS: the old values (tile plus a 2-cell x-y halo) and the values after the red
// half-sweep (tile plus 1).  Step k loads old plane k+1, does the red half-sweep
// of plane k and the black half-sweep of plane k-1.  Red points of the 1-cell
// halo ring and of the planes next to the chunk are recomputed by every block
// that needs them, so blocks are independent and the result equals the global
// two-pass sweep; input and output are separate arrays, so blocks never race.
// With zero_guess the old values are taken as zero (ein is not read); with
// ec != nullptr the old value is ein + the prolonged coarse correction (see
// prolong_value), so the prolongation is folded into the sweep that follows it.
// Every thread owns one point of the tile through both half-sweeps: in the red
// step of plane k it reads its point's six face coefficients and right-hand side
// once, updates the point if it is red, and otherwise keeps the seven values in
// registers for the black step of plane k one step later (a plane later they
// would no longer be in L2).  The upper z-face coefficient of plane k is the
// lower one of plane k+1 and is carried over as well.  Threads below the ring
// size also take one point of the 1-cell halo ring, read directly.  At most 64
// VGPRs, so that two 1024-thread blocks share a CU.  With EARLY all global loads
// of a step are issued before its first barrier so that their latencies overlap
// (one HBM round trip per plane instead of two); that keeps the coefficients
// live across the barrier and fits the 64 registers only in float.
template <class R, int TX, int TY, bool EARLY>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(8))) k_p_sweep3c(Box b, int kc, int zero_guess, R omega, const R *__restrict__ ein,
        const R *__restrict__ ec, Box cb, int lin, R *__restrict__ eout, const R *__restrict__ r,
        const R *__restrict__ bx, const R *__restrict__ by, const R *__restrict__ bz) {
    constexpr int NT = TX * TY;
    constexpr int EX1 = TX + 2, EY1 = TY + 2, N1 = EX1 * EY1;
    constexpr int EX2 = TX + 4, EY2 = TY + 4, N2 = EX2 * EY2;
    constexpr int NRING = N1 - NT;
    static_assert(NRING <= NT, "ring larger than the tile");
    __shared__ R oldp[3][N2];
    __shared__ R newp[3][N1];
    const int tid = threadIdx.x;
    const int G = gridDim.x * gridDim.y * gridDim.z;
    int t = xcd_swizzle(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), G);
    const int bx_ = t % gridDim.x;
    t /= gridDim.x;
    const int by_ = t % gridDim.y, bz_ = t / gridDim.y;
    const int i0 = bx_ * TX, j0 = by_ * TY;
    const int k0 = bz_ * kc, k1 = min(k0 + kc, b.nz);
    const int sy = b.px, sz = b.plane;
    const R ix2 = R(b.ihx * b.ihx), iy2 = R(b.ihy * b.ihy), iz2 = R(b.ihz * b.ihz);
    auto slot = [](int k) { return ((k % 3) + 3) % 3; };
    auto load_old = [&](int k) {
        R *dst = oldp[slot(k)];
        for (int t = tid; t < N2; t += NT) {
            int i = i0 + (t % EX2) - 2, j = j0 + (t / EX2) - 2;
            R v = R(0);
            if (!zero_guess && k >= 0 && k < b.nz && i >= 0 && i < b.nx && j >= 0 && j < b.ny) {
                int q = box_index(b, i, j, k);
                v = ein[q];
                if (ec) v += prolong_value<3, R, false>(cb, ec, i, j, k, lin);
            }
            dst[t] = v;
        }
    };
    // own tile point
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < b.nx && j < b.ny;
    const int o1 = (ty + 1) * EX1 + (tx + 1), o2 = (ty + 2) * EX2 + (tx + 2);
    // own ring point (tid < NRING): top row, bottom row, left column, right column
    int rex = 0, rey = 0;
    if (tid < EX1) { rex = tid; rey = 0; }
    else if (tid < 2 * EX1) { rex = tid - EX1; rey = EY1 - 1; }
    else if (tid < 2 * EX1 + TY) { rex = 0; rey = 1 + tid - 2 * EX1; }
    else { rex = EX1 - 1; rey = 1 + tid - 2 * EX1 - TY; }
    const int ri = i0 + rex - 1, rj = j0 + rey - 1;
    const bool ring = tid < NRING && ri >= 0 && ri < b.nx && rj >= 0 && rj < b.ny;
    const int ro1 = rey * EX1 + rex, ro2 = (rey + 1) * EX2 + (rex + 1);
    // kept for the black step: weights and right-hand side of the own point
    R kW = 0, kE = 0, kS = 0, kN = 0, kB = 0, kT = 0, kr = 0;
    R carryB = 0;          // own point's lower z weight of the next plane
    bool have_carry = false;
    load_old(k0 - 2);
    load_old(k0 - 1);
    const bool two = tid + NT < N2;
    for (int k = k0 - 1; k <= k1; ++k) {
        const bool kin = k >= 0 && k < b.nz;
        const bool ownk = own && kin;
        const bool ringred = tid < NRING && ring && kin && ((ri + rj + k) & 1) == 0;
        // raw coefficients of plane k: own point (c*) and red ring point (a*)
        R cW = 0, cE = 0, cS = 0, cN = 0, cB = 0, cT = 0, cr = 0;
        R aW = 0, aE = 0, aS = 0, aN = 0, aB = 0, aT = 0, ar = 0;
        auto load_own = [&]() {
            if (ownk) {
                const int q = box_index(b, i, j, k);
                cW = bx[q]; cE = bx[q + 1]; cS = by[q]; cN = by[q + sy];
                if (!have_carry) cB = bz[q];
                cT = bz[q + sz]; cr = r[q];
            }
        };
        auto load_ring = [&]() {
            if (ringred) {
                const int q = box_index(b, ri, rj, k);
                aW = bx[q]; aE = bx[q + 1]; aS = by[q]; aN = by[q + sy]; aB = bz[q]; aT = bz[q + sz]; ar = r[q];
            }
        };
        if constexpr (EARLY) {
            // all of the step's global loads before the barrier, so that their
            // latencies overlap: old plane k+1 first (its LDS stores wait only
            // for it), then the coefficients (used after the barrier)
            auto old_at = [&](int t) -> R {
                int ii = i0 + (t % EX2) - 2, jj = j0 + (t / EX2) - 2;
                R v = R(0);
                const int kn = k + 1;
                if (!zero_guess && kn >= 0 && kn < b.nz && ii >= 0 && ii < b.nx && jj >= 0 && jj < b.ny) {
                    int q = box_index(b, ii, jj, kn);
                    v = ein[q];
                    if (ec) v += prolong_value<3, R, false>(cb, ec, ii, jj, kn, lin);
                }
                return v;
            };
            const R v0 = old_at(tid);
            const R v1 = two ? old_at(tid + NT) : R(0);
            load_own();
            load_ring();
            R *d = oldp[slot(k + 1)];
            d[tid] = v0;
            if (two) d[tid + NT] = v1;
        } else {
            load_old(k + 1);
        }
        __syncthreads();
        const R *om = oldp[slot(k - 1)], *oc = oldp[slot(k)], *op = oldp[slot(k + 1)];
        R *dst = newp[slot(k)];
        // red half-sweep of plane k: own tile point
        {
            if constexpr (!EARLY) load_own();
            R v = R(0);
            if (ownk) {
                const R wW = cW * ix2, wE = cE * ix2, wS = cS * iy2, wN = cN * iy2;
                const R wB = have_carry ? carryB : cB * iz2;
                const R wT = cT * iz2;
                carryB = wT;
                have_carry = true;
                if (((i + j + k) & 1) == 0) {
                    const R dg = wW + wE + wS + wN + wB + wT;
                    const R off = wW * oc[o2 - 1] + wE * oc[o2 + 1] + wS * oc[o2 - EX2] + wN * oc[o2 + EX2]
                                + wB * om[o2] + wT * op[o2];
                    v = dg > R(0) ? sor(oc[o2], (cr + off) / dg, omega) : R(0);
                } else {
                    kW = wW; kE = wE; kS = wS; kN = wN; kB = wB; kT = wT; kr = cr;
                    v = oc[o2];
                }
            }
            dst[o1] = v;
        }
        // red half-sweep of plane k: own ring point
        if (tid < NRING) {
            if constexpr (!EARLY) load_ring();
            R v = R(0);
            if (ring && kin) {
                if (ringred) {
                    const R wW = aW * ix2, wE = aE * ix2, wS = aS * iy2, wN = aN * iy2;
                    const R wB = aB * iz2, wT = aT * iz2;
                    const R dg = wW + wE + wS + wN + wB + wT;
                    const R off = wW * oc[ro2 - 1] + wE * oc[ro2 + 1] + wS * oc[ro2 - EX2] + wN * oc[ro2 + EX2]
                                + wB * om[ro2] + wT * op[ro2];
                    v = dg > R(0) ? sor(oc[ro2], (ar + off) / dg, omega) : R(0);
                } else {
                    v = oc[ro2];
                }
            }
            dst[ro1] = v;
        }
        __syncthreads();
        // black half-sweep of plane k-1 on the tile, written out with the red values
        const int kk = k - 1;
        if (kk >= k0 && kk < k1 && own) {
            const R *nm = newp[slot(kk - 1)], *nc = newp[slot(kk)], *np = newp[slot(kk + 1)];
            const int q = box_index(b, i, j, kk);
            R v;
            if (((i + j + kk) & 1) == 1) {
                const R dg = kW + kE + kS + kN + kB + kT;
                const R off = kW * nc[o1 - 1] + kE * nc[o1 + 1] + kS * nc[o1 - EX1] + kN * nc[o1 + EX1]
                            + kB * nm[o1] + kT * np[o1];
                v = dg > R(0) ? sor(nc[o1], (kr + off) / dg, omega) : R(0);
            } else {
                v = nc[o1];
            }
            eout[q] = v;
        }
    }
}

// ---------------------------------------------------------------- coefficients
// Coarse cell viscosity: harmonic mean of the 2^d children.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_coarsen_mu(Box fb, Box cb, const R *__restrict__ f, R *__restrict__ c) {
    int idx = box_thread_index();
    if (idx >= cb.nb) return;
    int I, J, K;
    decompose(cb, idx, I, J, K);
    if (!is_cell(cb, I, J, K)) { c[idx] = R(0); return; }
    double s = 0.0;
    const int n2 = DIM == 3 ? 2 : 1;
    for (int dk = 0; dk < n2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di)
                s += 1.0 / (double)f[box_index(fb, 2 * I + di, 2 * J + dj, DIM == 3 ? 2 * K + dk : 0)];
    c[idx] = (R)((DIM == 3 ? 8.0 : 4.0) / s);
}

// Coarse Poisson coefficient on the faces normal to comp: arithmetic mean of the
// coincident fine beta (the harmonic mean of rho); wall faces stay zero.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_coarsen_beta(Box fb, Box cb, int comp, const R *__restrict__ f, R *__restrict__ c) {
    int idx = box_thread_index();
    if (idx >= cb.nb) return;
    int I, J, K;
    decompose(cb, idx, I, J, K);
    bool inner = comp == 0 ? is_ux(cb, I, J, K) : comp == 1 ? is_vy(cb, I, J, K) : is_wz(cb, I, J, K);
    if (!inner) { c[idx] = R(0); return; }
    const int s[3] = {1, fb.px, fb.plane};
    const int t1 = comp == 0 ? s[1] : s[0];
    const int t2 = comp == 2 ? s[1] : s[2];
    int base = box_index(fb, 2 * I, 2 * J, DIM == 3 ? 2 * K : 0);
    double acc = (double)f[base] + (double)f[base + t1];
    if (DIM == 3) acc += (double)f[base + t2] + (double)f[base + t1 + t2];
    c[idx] = (R)(acc * (DIM == 3 ? 0.25 : 0.5));
}

// Edge viscosities of a level: harmonic mean of the 4 cells around each edge,
// out-of-domain cells mirrored (wrapped along a periodic axis).  mxy at (x-face i, y-face j, cell k), mxz at
// (x-face i, cell j, z-face k), myz at (cell i, y-face j, z-face k).
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_edge_mu(Box b, const R *__restrict__ mu, R *__restrict__ mxy,
        R *__restrict__ mxz, R *__restrict__ myz) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    // out-of-domain cells: mirrored at a wall, wrapped on a periodic axis
    auto cl = [](int a, int n, int per) { return per ? (a + n) % n : (a < 0 ? 0 : (a > n - 1 ? n - 1 : a)); };
    int i0 = cl(i - 1, b.nx, b.per[0]), i1 = cl(i, b.nx, b.per[0]);
    int j0 = cl(j - 1, b.ny, b.per[1]), j1 = cl(j, b.ny, b.per[1]);
    if (k < b.nz) {
        double s = 1.0 / (double)mu[box_index(b, i0, j0, k)] + 1.0 / (double)mu[box_index(b, i1, j0, k)]
                 + 1.0 / (double)mu[box_index(b, i0, j1, k)] + 1.0 / (double)mu[box_index(b, i1, j1, k)];
        mxy[idx] = (R)(4.0 / s);
    } else {
        mxy[idx] = R(0);
    }
    if (DIM == 3) {
        int k0 = cl(k - 1, b.nz, b.per[2]), k1 = cl(k, b.nz, b.per[2]);
        if (j < b.ny) {
            double s = 1.0 / (double)mu[box_index(b, i0, j, k0)] + 1.0 / (double)mu[box_index(b, i1, j, k0)]
                     + 1.0 / (double)mu[box_index(b, i0, j, k1)] + 1.0 / (double)mu[box_index(b, i1, j, k1)];
            mxz[idx] = (R)(4.0 / s);
        } else {
            mxz[idx] = R(0);
        }
        if (i < b.nx) {
            double s = 1.0 / (double)mu[box_index(b, i, j0, k0)] + 1.0 / (double)mu[box_index(b, i, j1, k0)]
                     + 1.0 / (double)mu[box_index(b, i, j0, k1)] + 1.0 / (double)mu[box_index(b, i, j1, k1)];
            myz[idx] = (R)(4.0 / s);
        } else {
            myz[idx] = R(0);
        }
    }
}

// ---------------------------------------------------------------- layout conversion
// Caller layout (C order, x fastest, per-field shape) <-> padded box.
// comp 0,1,2: face arrays normal to x,y,z; comp 3: cell array.
// mode 0: copy, 1: reciprocal (beta = 1/rho), 2: multiply by s.
// Only interior unknowns are copied (faces: interior faces; with keep_walls the
// wall faces too); everything else in the box is written as 0.  With flag, the
// values read are checked on the way (one vector store per block at most, after
// a block-wide OR; the flags are read first so that later blocks mostly skip the
// store): check 0, flag[0] = 1 if one is not finite and flag[1] = 1 if one is
// nonzero; check 1 (a viscosity), flag[0] = 1 if one is negative or not finite.
// Row form: a block of 64 x kPackRows threads takes kPackRows rows (j, k) of the
// box, one wavefront per row, each lane stepping over x in strides of 64, so no
// thread divides a flat point index.
constexpr int kPackRows = 4;

// Face rows (j, k) of component comp (1: y-faces, 2: z-faces) that are not
// unknowns: the walls (and, on a periodic axis, face n, the slot that repeats
// face 0).  x-faces: the same along x.
__device__ inline bool face_row_wall(const Box &b, int comp, int j, int k) {
    if (comp == 1) return (j == 0 && !b.per[1]) || (j == b.ny && !(b.open_top && b.dim == 2));
    if (comp == 2) return (k == 0 && !b.per[2]) || (k == b.nz && !(b.open_top && b.dim == 3));
    return false;
}
__device__ inline bool x_wall_face(const Box &b, int i) { return (i == 0 && !b.per[0]) || i == b.nx; }

__global__ void __launch_bounds__(64 * kPackRows) k_pack(Box b, int comp, int mode, int keep_walls, double s,
        const double *__restrict__ src, double *__restrict__ dst, int *__restrict__ flag, int check) {
    const int r = blockIdx.x * kPackRows + threadIdx.y;     // row j + py k
    bool bad = false, nz = false;
    if (r < b.py * b.pz) {
        const int k = r / b.py, j = r - k * b.py;
        const int ex = b.nx + (comp == 0), ey = b.ny + (comp == 1), ez = b.nz + (comp == 2);
        const bool row_in = j < ey && k < ez;
        const bool row_wall = face_row_wall(b, comp, j, k);
        const double *sr = src + (row_in ? ex * (j + ey * k) : 0);
        double *dr = dst + r * b.px;
        for (int i = threadIdx.x; i < b.px; i += 64) {
            double val = 0.0;
            if (row_in && i < ex && (keep_walls || !(row_wall || (comp == 0 && x_wall_face(b, i))))) {
                const double x = sr[i];
                bad |= check ? !(x >= 0.0) || !isfinite(x) : !isfinite(x);
                nz |= x != 0.0;
                val = mode == 0 ? x : mode == 1 ? 1.0 / x : s * x;
            }
            dr[i] = val;
        }
    }
    if (flag) {                       // uniform: every thread of the block takes both barriers
        const bool any_bad = __syncthreads_or(bad), any_nz = __syncthreads_or(nz);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            if (any_bad && flag[0] == 0) flag[0] = 1;
            if (!check && any_nz && flag[1] == 0) flag[1] = 1;
        }
    }
}

// Box -> caller layout for every point of the caller's array (wall faces included;
// along a periodic axis the caller's last face, which repeats face 0, gets face 0).
__global__ void __launch_bounds__(64 * kPackRows) k_unpack(Box b, int comp, const double *__restrict__ src,
        double *__restrict__ dst) {
    const int r = blockIdx.x * kPackRows + threadIdx.y;
    if (r >= b.py * b.pz) return;
    const int k = r / b.py, j = r - k * b.py;
    const int ex = b.nx + (comp == 0), ey = b.ny + (comp == 1), ez = b.nz + (comp == 2);
    if (j >= ey || k >= ez) return;
    double *dr = dst + ex * (j + ey * k);
    // on a periodic axis the caller's face n repeats face 0
    const int js = (comp == 1 && b.per[1] && j == b.ny) ? 0 : j;
    const int ks = (comp == 2 && b.per[2] && k == b.nz) ? 0 : k;
    const double *sr = src + (js + b.py * ks) * b.px;
    for (int i = threadIdx.x; i < ex; i += 64) dr[i] = sr[(comp == 0 && b.per[0] && i == b.nx) ? 0 : i];
}

// Face densities of one component -> mass = rho/dt and beta = 1/rho in one pass
// over rho, in the row form of k_pack: interior faces (and the open top's, where
// beta = 2/rho) only, everything else in the box written as 0.  flag[0] = 1 if an interior mass value is not > 0 or not
// finite (one vector store per block at most, after a block-wide OR).
__global__ void __launch_bounds__(64 * kPackRows) k_pack_rho(Box b, int comp, double inv_dt,
        const double *__restrict__ src, double *__restrict__ mass, double *__restrict__ beta,
        int *__restrict__ flag) {
    const int r = blockIdx.x * kPackRows + threadIdx.y;     // row j + py k
    bool bad = false;
    if (r < b.py * b.pz) {
        const int k = r / b.py, j = r - k * b.py;
        const int ex = b.nx + (comp == 0), ey = b.ny + (comp == 1), ez = b.nz + (comp == 2);
        const bool row_in = j < ey && k < ez;
        const bool row_wall = face_row_wall(b, comp, j, k);
        const double *sr = src + (row_in ? ex * (j + ey * k) : 0);
        double *mr = mass + r * b.px, *br = beta + r * b.px;
        for (int i = threadIdx.x; i < b.px; i += 64) {
            double m = 0.0, be = 0.0;
            if (row_in && i < ex && !(row_wall || (comp == 0 && x_wall_face(b, i)))) {
                const double x = sr[i];
                m = inv_dt * x;
                // the open top's faces: zero pressure on the face, half a cell from the
                // centre below, so the Poisson flux through them carries a factor 2
                const bool topf = (comp == 2 && b.dim == 3 && k == b.nz) || (comp == 1 && b.dim == 2 && j == b.ny);
                be = (topf ? 2.0 : 1.0) / x;
                bad |= !(m > 0.0) || !isfinite(m);
            }
            mr[i] = m;
            br[i] = be;
        }
    }
    const bool any_bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && threadIdx.y == 0 && any_bad && flag[0] == 0) flag[0] = 1;
}

// ---------------------------------------------------------------- preconditioner glue
// q = r_p + D u~ (FP64), s = -q/dt (right-hand side of -L_rho phi = -s_paper).
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_precond_div(Box b, const R *__restrict__ eu, const R *__restrict__ ev,
        const R *__restrict__ ew, const double *__restrict__ rp, double dt, double *__restrict__ q,
        R *__restrict__ s) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    double qq = 0.0;
    if (is_cell(b, i, j, k)) {
        const Nbr o = nbr(b, i, j, k);
        double dv = ((double)eu[idx + o.xp] - (double)eu[idx]) * b.ihx + ((double)ev[idx + o.yp] - (double)ev[idx]) * b.ihy;
        if (DIM == 3) dv += ((double)ew[idx + o.zp] - (double)ew[idx]) * b.ihz;
        qq = rp[idx] + dv;
    }
    q[idx] = qq;
    s[idx] = (R)(-qq / dt);
}

// z_u = u~ - dt beta G phi on interior faces; z_p = phi - 2 theta mu q on cells.
// eu/ev/ew may alias zu/zv/zw (FP64 multigrid): each point is read, then written,
// by the same thread.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_precond_update(Box b, const R *eu, const R *ev, const R *ew,
        const R *__restrict__ phi, const double *__restrict__ bx, const double *__restrict__ by,
        const double *__restrict__ bz, const double *__restrict__ mu, const double *__restrict__ q,
        double dt, double theta, double *zu, double *zv, double *zw, double *__restrict__ zp) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    const double ph = (double)phi[idx];
    const Nbr o = nbr(b, i, j, k);
    double z = 0.0;
    if (is_ux(b, i, j, k)) z = (double)eu[idx] - dt * bx[idx] * (ph - (double)phi[idx + o.xm]) * b.ihx;
    zu[idx] = z;
    z = 0.0;
    if (is_vy(b, i, j, k)) z = (double)ev[idx] - dt * by[idx] * (ph - (double)phi[idx + o.ym]) * b.ihy;
    zv[idx] = z;
    if (DIM == 3) {
        z = 0.0;
        if (is_wz(b, i, j, k)) z = (double)ew[idx] - dt * bz[idx] * (ph - (double)phi[idx + o.zm]) * b.ihz;
        zw[idx] = z;
    }
    z = 0.0;
    if (is_cell(b, i, j, k)) z = ph - 2.0 * theta * mu[idx] * q[idx];
    zp[idx] = z;
}

// Diagonal (point-Jacobi) form of step 1 folded into the glue kernels: when the
// velocity operator is mass dominated, u~ = D_A^{-1} v_u with dinv the inverse
// diagonal of A.  Same formulas as k_precond_div / k_precond_update otherwise.
// The input vector is vs * (vu, vv, vw, rp): the Krylov basis is stored
// unnormalised with its scale kept aside.
template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_precond_div_jac(Box b, const double *__restrict__ vu,
        const double *__restrict__ vv, const double *__restrict__ vw, const double *__restrict__ du,
        const double *__restrict__ dv, const double *__restrict__ dw, const double *__restrict__ rp, double vs,
        double dt, double *__restrict__ q, R *__restrict__ s) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    double qq = 0.0;
    if (is_cell(b, i, j, k)) {
        const Nbr o = nbr(b, i, j, k);
        double d = (vu[idx + o.xp] * du[idx + o.xp] - vu[idx] * du[idx]) * b.ihx
                 + (vv[idx + o.yp] * dv[idx + o.yp] - vv[idx] * dv[idx]) * b.ihy;
        if (DIM == 3) d += (vw[idx + o.zp] * dw[idx + o.zp] - vw[idx] * dw[idx]) * b.ihz;
        qq = vs * (rp[idx] + d);
    }
    q[idx] = qq;
    s[idx] = (R)(-qq / dt);
}

template <int DIM, class R>
__global__ void __launch_bounds__(kBlock) k_precond_update_jac(Box b, const double *__restrict__ vu,
        const double *__restrict__ vv, const double *__restrict__ vw, const double *__restrict__ du,
        const double *__restrict__ dv, const double *__restrict__ dw, double vs, const R *__restrict__ phi,
        const double *__restrict__ bx, const double *__restrict__ by, const double *__restrict__ bz,
        const double *__restrict__ mu, const double *__restrict__ q, double dt, double theta,
        double *__restrict__ zu, double *__restrict__ zv, double *__restrict__ zw, double *__restrict__ zp) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    const double ph = (double)phi[idx];
    const Nbr o = nbr(b, i, j, k);
    double z = 0.0;
    if (is_ux(b, i, j, k)) z = vs * vu[idx] * du[idx] - dt * bx[idx] * (ph - (double)phi[idx + o.xm]) * b.ihx;
    zu[idx] = z;
    z = 0.0;
    if (is_vy(b, i, j, k)) z = vs * vv[idx] * dv[idx] - dt * by[idx] * (ph - (double)phi[idx + o.ym]) * b.ihy;
    zv[idx] = z;
    if (DIM == 3) {
        z = 0.0;
        if (is_wz(b, i, j, k)) z = vs * vw[idx] * dw[idx] - dt * bz[idx] * (ph - (double)phi[idx + o.zm]) * b.ihz;
        zw[idx] = z;
    }
    z = 0.0;
    if (is_cell(b, i, j, k)) z = ph - 2.0 * theta * mu[idx] * q[idx];
    zp[idx] = z;
}

// Inverse diagonal of the fine velocity operator (0 off the interior faces).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_vel_inv_diag(Box b, VelCoef<double> c, double *__restrict__ du,
        double *__restrict__ dv, double *__restrict__ dw) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    double off, dg, v = 0.0;
    if (is_ux(b, i, j, k)) { row_u<DIM, double>(b, idx, i, j, k, nullptr, nullptr, nullptr, 0, c, off, dg); v = 1.0 / dg; }
    du[idx] = v;
    v = 0.0;
    if (is_vy(b, i, j, k)) { row_v<DIM, double>(b, idx, i, j, k, nullptr, nullptr, nullptr, 0, c, off, dg); v = 1.0 / dg; }
    dv[idx] = v;
    if (DIM == 3) {
        v = 0.0;
        if (is_wz(b, i, j, k)) { row_w<double>(b, idx, i, j, k, nullptr, nullptr, nullptr, 0, c, off, dg); v = 1.0 / dg; }
        dw[idx] = v;
    }
}

// ---------------------------------------------------------------- learned stage glue
// Coarse cell = mean of its 8 children (3D).
template <class R>
__global__ void __launch_bounds__(kBlock) k_restrict_avg3(Box fb, Box cb, const R *__restrict__ f, R *__restrict__ c) {
    int idx = box_thread_index();
    if (idx >= cb.nb) return;
    int I, J, K;
    decompose(cb, idx, I, J, K);
    if (!is_cell(cb, I, J, K)) { c[idx] = R(0); return; }
    R acc = 0;
    for (int d = 0; d < 8; ++d)
        acc += f[box_index(fb, 2 * I + (d & 1), 2 * J + ((d >> 1) & 1), 2 * K + (d >> 2))];
    c[idx] = acc * R(0.125);
}

// y = -L_rho e on the cells of one level (0 elsewhere)
template <class R>
__global__ void __launch_bounds__(kBlock) k_p_apply3(Box b, const R *__restrict__ e, const R *__restrict__ bx,
        const R *__restrict__ by, const R *__restrict__ bz, R *__restrict__ y) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    R v = 0;
    if (is_cell(b, i, j, k)) {
        R off, dg;
        prow<3, R>(b, idx, i, j, k, e, bx, by, bz, off, dg);
        v = dg * e[idx] - off;
    }
    y[idx] = v;
}

// Static features on a level of n^3 cells (planar, x fastest): f0 = log10(rho)/3 - 1/2
// with rho the harmonic mean of the interior face densities (from beta), and
// f1 = log10(mu)/2 + 2.
template <class R>
__global__ void __launch_bounds__(kBlock) k_learned_static(Box b, const R *__restrict__ bx, const R *__restrict__ by,
        const R *__restrict__ bz, const R *__restrict__ mu, float *__restrict__ f0, float *__restrict__ f1) {
    int t = blockIdx.x * kBlock + threadIdx.x;
    const int nc = b.nx * b.ny * b.nz;
    if (t >= nc) return;
    const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
    const int q = box_index(b, i, j, k);
    double sb = 0.0;
    int cnt = 0;
    const double f[6] = {(double)bx[q], (double)bx[q + 1], (double)by[q], (double)by[q + b.px],
                         (double)bz[q], (double)bz[q + b.plane]};
    for (int a = 0; a < 6; ++a)
        if (f[a] > 0.0) { sb += f[a]; ++cnt; }
    const double rho = cnt > 0 ? cnt / sb : 1.0;
    f0[t] = (float)(log10(rho) / 3.0 - 0.5);
    f1[t] = (float)(log10(fmax((double)mu[q], 1e-30)) / 2.0 + 2.0);
}

// One block: rms of the level's cell values, then dst = src / rms (planar FP32,
// zero mean removed first when `center`).  rms (and the mean) go to stat[0..1].
template <class R>
__global__ void __launch_bounds__(1024) k_normalise_planar(Box b, const R *__restrict__ src, int center,
        float *__restrict__ dst, double *__restrict__ stat) {
    __shared__ double sh[1024];
    const int nc = b.nx * b.ny * b.nz;
    double s1 = 0.0;
    for (int t = threadIdx.x; t < nc; t += 1024) {
        const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
        s1 += (double)src[box_index(b, i, j, k)];
    }
    sh[threadIdx.x] = s1;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double mean = center ? sh[0] / nc : 0.0;
    __syncthreads();
    double s2 = 0.0;
    for (int t = threadIdx.x; t < nc; t += 1024) {
        const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
        const double v = (double)src[box_index(b, i, j, k)] - mean;
        s2 += v * v;
    }
    sh[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double rms = sqrt(sh[0] / nc);
    const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
    for (int t = threadIdx.x; t < nc; t += 1024) {
        const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
        dst[t] = (float)(((double)src[box_index(b, i, j, k)] - mean) * inv);
    }
    if (threadIdx.x == 0) {
        stat[0] = rms;
        stat[1] = mean;
    }
}

// planar FP32 -> the cells of a level's box array (other slots untouched)
template <class R>
__global__ void __launch_bounds__(kBlock) k_planar_to_box(Box b, const float *__restrict__ src, R *__restrict__ dst) {
    int t = blockIdx.x * kBlock + threadIdx.x;
    const int nc = b.nx * b.ny * b.nz;
    if (t >= nc) return;
    const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
    dst[box_index(b, i, j, k)] = (R)src[t];
}

// One block: alpha = <y, s> / <y, y> over the level's cells (the least-squares
// amplitude of the prediction e for -L e = s), then e *= alpha (alpha = 0 if
// not finite).
template <class R>
__global__ void __launch_bounds__(1024) k_fit_amplitude(Box b, const R *__restrict__ y, const R *__restrict__ s,
        R *__restrict__ e, double *__restrict__ stat) {
    __shared__ double a[1024], c[1024];
    const int nc = b.nx * b.ny * b.nz;
    double ys = 0.0, yy = 0.0;
    for (int t = threadIdx.x; t < nc; t += 1024) {
        const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
        const int q = box_index(b, i, j, k);
        ys += (double)y[q] * (double)s[q];
        yy += (double)y[q] * (double)y[q];
    }
    a[threadIdx.x] = ys;
    c[threadIdx.x] = yy;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            a[threadIdx.x] += a[threadIdx.x + o];
            c[threadIdx.x] += c[threadIdx.x + o];
        }
        __syncthreads();
    }
    double alpha = c[0] > 0.0 ? a[0] / c[0] : 0.0;
    if (!isfinite(alpha)) alpha = 0.0;
    for (int t = threadIdx.x; t < nc; t += 1024) {
        const int i = t % b.nx, j = (t / b.nx) % b.ny, k = t / (b.nx * b.ny);
        const int q = box_index(b, i, j, k);
        e[q] = (R)(alpha * (double)e[q]);
    }
    if (threadIdx.x == 0) stat[2] = alpha;
}

// ---------------------------------------------------------------- BLAS-1
template <class A, class B>
__global__ void __launch_bounds__(kBlock) k_cast(long long n, const A *__restrict__ x, B *__restrict__ y) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long st = (long long)gridDim.x * kBlock;
    for (; t < n; t += st) y[t] = (B)x[t];
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_fill(long long n, R *__restrict__ x, R v) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long st = (long long)gridDim.x * kBlock;
    for (; t < n; t += st) x[t] = v;
}

// wave64 + LDS block reduction of NV partial sums; the result is in lane 0 of
// warp 0 for each of the NV values.
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], double *lds /* [NV][kBlock/64] */) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double x = v[m];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) lds[m * (kBlock / 64) + wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            double x = threadIdx.x < kBlock / 64 ? lds[m * (kBlock / 64) + threadIdx.x] : 0.0;
            for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
            v[m] = x;
        }
    }
}

// The Krylov BLAS kernels stream whole vectors (n even, every vector 16-byte
// aligned) as element pairs with 16-byte non-temporal accesses.  Each block owns
// a contiguous chunk of kBlock * P pairs, thread t the pairs t, t + kBlock, ...
// of it (coalesced), and issues all of its loads before the arithmetic: with P
// chosen so that about two dozen pairs (multidot) or 8-12 (maxpy, which also
// stores) are in flight per thread this reaches 6.0-6.4 and 5.7 TB/s at the
// 256^3 vector length, where grid-stride loops over 2048-16384 blocks reach
// 5.1-5.4 and 4.5 TB/s.
typedef double dpair __attribute__((ext_vector_type(2)));

// partial[m * gridDim.x + block] = sum over this block's pairs of
// wgt * V_m[t] * w[t], m < NV; wgt = w2 for pair index >= pstart2 (pstart even).
// SELF (NV = 1, V = w): the weighted squared norm, each pair loaded once.
template <int NV, int P, bool SELF = false>
__global__ void __launch_bounds__(kBlock) k_multidot(long long n2, long long pstart2, double w2,
        const dpair *__restrict__ V, long long ldv2, const dpair *__restrict__ w, double *__restrict__ partial) {
    static_assert(!SELF || NV == 1, "a self product has one vector");
    __shared__ double lds[NV * (kBlock / 64)];
    const long long base = (long long)blockIdx.x * (kBlock * P) + threadIdx.x;
    dpair x[P], v[NV][P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const long long u = base + (long long)p * kBlock;
        const dpair z = {0.0, 0.0};
        x[p] = u < n2 ? __builtin_nontemporal_load(w + u) : z;
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m][p] = SELF ? x[p] : u < n2 ? __builtin_nontemporal_load(V + m * ldv2 + u) : z;
    }
    double acc[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) acc[m] = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        dpair xp = x[p];
        if (base + (long long)p * kBlock >= pstart2) xp *= w2;
#pragma unroll
        for (int m = 0; m < NV; ++m) acc[m] += v[m][p].x * xp.x + v[m][p].y * xp.y;
    }
    block_reduce<NV>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) partial[m * gridDim.x + blockIdx.x] = acc[m];
    }
}

// out[m] (=, or += if accumulate) sum over blocks of partial[m * nblk + .], in a
// fixed order: the result is bitwise reproducible.  One block per m.  With
// mscale != nullptr the sum is multiplied by mscale[m] first.
__global__ void __launch_bounds__(kBlock) k_reduce_partials(int nblk, const double *__restrict__ partial,
        double *__restrict__ out, int accumulate, const double *__restrict__ mscale) {
    __shared__ double lds[kBlock / 64];
    const int m = blockIdx.x;
    double v[1] = {0.0};
#pragma unroll 8
    for (int t = threadIdx.x; t < nblk; t += kBlock) v[0] += partial[(size_t)m * nblk + t];
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) {
        const double r = mscale ? v[0] * mscale[m] : v[0];
        out[m] = accumulate ? out[m] + r : r;
    }
}

// p[0] = v (one thread; a device scalar set in stream order)
__global__ void k_set_scalar(double *__restrict__ p, double v) {
    if (threadIdx.x == 0) p[0] = v;
}

// w[t] += sign * sum_m c[m] * s[m] * V_m[t], m < NV (c and the optional per-vector
// scales s on the device; s = 1 when vscale is nullptr), over element pairs as
// k_multidot.  With partial != nullptr also the weighted squared norm of the
// updated w (weight w2 from pair index pstart2 on), one partial sum per block.
template <int NV, int P>
__global__ void __launch_bounds__(kBlock) k_maxpy(long long n2, double sign, const dpair *__restrict__ V,
        long long ldv2, const double *__restrict__ c, const double *__restrict__ vscale, dpair *__restrict__ w,
        long long pstart2, double w2, double *__restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    double cc[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) cc[m] = sign * c[m] * (vscale ? vscale[m] : 1.0);
    const long long base = (long long)blockIdx.x * (kBlock * P) + threadIdx.x;
    dpair x[P], v[NV][P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const long long u = base + (long long)p * kBlock;
        if (u < n2) {
            x[p] = __builtin_nontemporal_load(w + u);
#pragma unroll
            for (int m = 0; m < NV; ++m) v[m][p] = __builtin_nontemporal_load(V + m * ldv2 + u);
        }
    }
    double nrm[1] = {0.0};
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const long long u = base + (long long)p * kBlock;
        if (u < n2) {
            dpair y = x[p];
#pragma unroll
            for (int m = 0; m < NV; ++m) y += cc[m] * v[m][p];
            __builtin_nontemporal_store(y, w + u);
            nrm[0] += (u >= pstart2 ? w2 : 1.0) * (y.x * y.x + y.y * y.y);
        }
    }
    if (partial) {
        block_reduce<1>(nrm, lds);
        if (threadIdx.x == 0) partial[blockIdx.x] = nrm[0];
    }
}

// x[t] *= 1/sqrt(nrm2[0]) (nothing if the norm is zero)
__global__ void __launch_bounds__(kBlock) k_scale_inv_sqrt(long long n, const double *__restrict__ nrm2,
        double *__restrict__ x) {
    double s2 = nrm2[0];
    if (!(s2 > 0.0)) return;
    double s = 1.0 / sqrt(s2);
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long st = (long long)gridDim.x * kBlock;
    for (; t < n; t += st) x[t] *= s;
}

// dst[t] = src[t]: the streaming reference (one read and one write per element).
// With vec2, 16-byte non-temporal accesses (both arrays 16-byte aligned); one
// element pair per thread over a full grid measured fastest (6.6 TB/s against
// 4.7-5.6 TB/s for grid-stride loops over 2048-16384 blocks).
typedef double stream_d2 __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(kBlock) k_stream_copy(long long n, const double *__restrict__ src,
        double *__restrict__ dst, int vec2) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long st = (long long)gridDim.x * kBlock;
    if (vec2) {
        const long long n2 = n / 2;
        const stream_d2 *s2 = reinterpret_cast<const stream_d2 *>(src);
        stream_d2 *d2 = reinterpret_cast<stream_d2 *>(dst);
        for (long long u = t; u < n2; u += st) __builtin_nontemporal_store(__builtin_nontemporal_load(s2 + u), d2 + u);
        if (t == 0 && (n & 1)) dst[n - 1] = src[n - 1];
    } else {
        for (; t < n; t += st) dst[t] = src[t];
    }
}

// x[0, n) = 0 (x 16-byte aligned) with 16-byte non-temporal stores, one pair per
// thread of a full grid (grid stride beyond it).
__global__ void __launch_bounds__(kBlock) k_zero(long long n, double *__restrict__ x) {
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long st = (long long)gridDim.x * kBlock;
    stream_d2 *x2 = reinterpret_cast<stream_d2 *>(x);
    const stream_d2 z = {0.0, 0.0};
    for (long long u = t; u < n / 2; u += st) __builtin_nontemporal_store(z, x2 + u);
    if (t == 0 && (n & 1)) x[n - 1] = 0.0;
}

// x[t] *= s
__global__ void __launch_bounds__(kBlock) k_scale(long long n, double s, double *__restrict__ x) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long st = (long long)gridDim.x * kBlock;
    for (; t < n; t += st) x[t] *= s;
}

// subtract mean = sum[0] / ncell on the cells of a cell array
__global__ void __launch_bounds__(kBlock) k_sub_mean(Box b, const double *__restrict__ sum, double *__restrict__ p) {
    int idx = box_thread_index();
    if (idx >= b.nb) return;
    int i, j, k;
    decompose(b, idx, i, j, k);
    if (!is_cell(b, i, j, k)) return;
    p[idx] -= sum[0] / ((double)b.nx * b.ny * b.nz);
}

// Partial sums of the squared residual r - (-L_rho) e and of r^2 over the cells of
// one 3D level (grid-stride; block b writes partial[b] and partial[gridDim.x + b]).
template <class R>
__global__ void __launch_bounds__(kBlock) k_p_res_partial(Box b, const R *__restrict__ e, const R *__restrict__ r,
        const R *__restrict__ bx, const R *__restrict__ by, const R *__restrict__ bz, double *__restrict__ partial) {
    __shared__ double lds[2 * (kBlock / 64)];
    double v[2] = {0.0, 0.0};
    for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < b.nb; idx += gridDim.x * kBlock) {
        int i, j, k;
        decompose(b, idx, i, j, k);
        if (!is_cell(b, i, j, k)) continue;
        R off, dg;
        prow<3, R>(b, idx, i, j, k, e, bx, by, bz, off, dg);
        const double res = (double)r[idx] - ((double)dg * (double)e[idx] - (double)off);
        v[0] += res * res;
        v[1] += (double)r[idx] * (double)r[idx];
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = v[0];
        partial[gridDim.x + blockIdx.x] = v[1];
    }
}

// partial sums (plain) of a range; used for means and norms of sub-blocks
__global__ void __launch_bounds__(kBlock) k_partial_sum(long long n, const double *__restrict__ x, int squared,
        double *__restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    double v[1] = {0.0};
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long st = (long long)gridDim.x * kBlock;
    for (; t < n; t += st) {
        double a = x[t];
        v[0] += squared ? a * a : a;
    }
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

}  // namespace stk
