// Padded-box layout shared by every staggered field of one multigrid level.
//
// A level with Nx x Ny x Nz cells stores every field -- cell (p, mu), face
// (u, v, w, rho, beta) and edge (mu_xy, mu_xz, mu_yz) -- in one index space of
// (Nx+1) x (Ny+1) x (Nz+1) points (Nz+1 -> 1 in 2D; rows may be widened to Px >
// Nx+1 points, see pad_rows), x fastest.  Point (i,j,k)
// holds cell (i,j,k), the x-face at x = i*hx, the y-face at y = j*hy, the
// z-face at z = k*hz and the edges through the lower corner of that cell, so
// that every stencil uses the same neighbour offsets (1, px, px*py) whatever
// the field.  Slots that are not an unknown (wall-normal faces, padding) hold
// zero.  Each field is surrounded by a zero guard of at least one plane, so a
// +-1 neighbour of any box point is a valid address; stencils whose weight
// vanishes there (beta = 0 on wall faces) need no branch.  Along a periodic
// axis the flat kernels wrap the neighbour offsets instead (see Nbr).
#pragma once
#include <hip/hip_runtime.h>

namespace stk {

struct Box {
    int dim;                 // 2 or 3
    int nx, ny, nz;          // cells (nz = 1 in 2D)
    int px, py, pz;          // padded extents: nx+1, ny+1, nz+1 (1 in 2D)
    int plane;               // px * py
    int nb;                  // px * py * pz points
    int guard;               // zero elements before and after each field
    int stride;              // nb + 2*guard: field-to-field distance in a vector
    double hx, hy, hz;
    double ihx, ihy, ihz;    // 1/h
    int open_top;            // 1: the upper end of the vertical axis (y in 2D, z in 3D) is open
                             // (zero pressure, zero tangential velocity); the vertical velocity on
                             // its faces (index ny / nz) is an unknown
    int per[3];              // 1: the axis is periodic (cells and faces 0 .. n-1 wrap; face n is
                             // face 0 and its slot is padding), 0: walls at both ends
};

inline Box make_box(int dim, int nx, int ny, int nz, double hx, double hy, double hz) {
    Box b;
    b.dim = dim;
    b.nx = nx; b.ny = ny; b.nz = dim == 3 ? nz : 1;
    b.px = nx + 1; b.py = ny + 1; b.pz = dim == 3 ? nz + 1 : 1;
    b.plane = b.px * b.py;
    b.nb = b.plane * b.pz;
    b.guard = ((b.plane + 1 + 63) / 64) * 64;    // keeps each field 512-byte aligned
    b.stride = b.nb + 2 * b.guard;
    b.stride = ((b.stride + 63) / 64) * 64;
    b.hx = hx; b.hy = hy; b.hz = dim == 3 ? hz : hx;
    b.ihx = 1.0 / b.hx; b.ihy = 1.0 / b.hy; b.ihz = 1.0 / b.hz;
    b.open_top = 0;
    b.per[0] = b.per[1] = b.per[2] = 0;
    return b;
}

// Widens the rows of a box to a multiple of `mult` points (the slots past x = nx
// are padding, holding zero like slot nx).  With mult = 16 an FP64 row starts on a
// 128-byte boundary, so the row segments the z-marching kernels read per tile are
// whole cache lines; the guard and the field stride follow the wider plane.
inline void pad_rows(Box &b, int mult) {
    b.px = ((b.nx + 1 + mult - 1) / mult) * mult;
    b.plane = b.px * b.py;
    b.nb = b.plane * b.pz;
    b.guard = ((b.plane + 1 + 63) / 64) * 64;
    b.stride = b.nb + 2 * b.guard;
    b.stride = ((b.stride + 63) / 64) * 64;
}

__host__ __device__ inline int box_index(const Box &b, int i, int j, int k) {
    return i + b.px * (j + b.py * k);
}

}  // namespace stk
