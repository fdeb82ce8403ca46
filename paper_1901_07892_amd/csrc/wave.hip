// Inflow data of the wave tank (Sec. 7.1): the second-order Stokes wave of eqs.
// eq_stokes_eta, eq_stokes_u and eq_stokes_v evaluated on the x = 0 side and
// restricted to the liquid by the boundary Heaviside of eq.
// eq_heaviside_normal_bdry.  The vertical axis is y in 2D and z in 3D, with the
// tank bottom at 0 and the still level at the depth d; the wave travels along x.
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace {

constexpr int kWaveBlock = 256;

struct WaveArgs {
    double H, d, k, omega, g, eps, t;
    double c2;         // second-harmonic amplitude of the elevation
    double a1, a2;     // first- and second-order velocity amplitudes
    double eta0;       // elevation at x = 0
};

__device__ inline double heaviside(double phi, double eps) {
    if (phi < -eps) return 0.0;
    if (phi > eps) return 1.0;
    return 0.5 * (1.0 + phi / eps + sin(M_PI * phi / eps) / M_PI);
}

// horizontal (x) and vertical velocity of the wave at x = 0, height y above the still level
__device__ inline double wave_u(const WaveArgs &w, double y) {
    return w.a1 * cosh(w.k * (w.d + y)) * cos(-w.omega * w.t) + w.a2 * cosh(2.0 * w.k * (w.d + y)) * cos(-2.0 * w.omega * w.t);
}
__device__ inline double wave_v(const WaveArgs &w, double y) {
    return w.a1 * sinh(w.k * (w.d + y)) * sin(-w.omega * w.t) + w.a2 * sinh(2.0 * w.k * (w.d + y)) * sin(-2.0 * w.omega * w.t);
}

// thread t: u_n at (vertical cell index a, lateral index l) and u_t at (vertical node index a, l)
__global__ void __launch_bounds__(kWaveBlock) k_wave_inflow(WaveArgs w, int nvert, int nlat, double hv,
                                                            double *__restrict__ un, double *__restrict__ ut) {
    const int t = blockIdx.x * kWaveBlock + threadIdx.x;
    if (t >= (nvert + 1) * nlat) return;
    const int l = t % nlat, a = t / nlat;
    if (a < nvert) {
        const double y = (a + 0.5) * hv - w.d;
        un[l + nlat * a] = (1.0 - heaviside(-w.eta0 + y, w.eps)) * wave_u(w, y);
    }
    const double yn = a * hv - w.d;
    ut[l + nlat * a] = (1.0 - heaviside(-w.eta0 + yn, w.eps)) * wave_v(w, yn);
}

}  // namespace

extern "C" stokes_status stokes_wave_inflow(const stokes_grid *grid, const stokes_wave *wave, double t,
                                            double *u_n, double *u_t, void *stream) {
    if (!grid || !wave || !u_n || !u_t) return STOKES_EINVAL;
    const int dim = grid->dim;
    if (dim != 2 && dim != 3) return STOKES_EINVAL;
    for (int a = 0; a < dim; ++a) {
        if (grid->periodic[a]) return STOKES_EINVAL;     // the wave tank has walls
        if (grid->n[a] < 2) return STOKES_ESHAPE;
        if (!(grid->h[a] > 0.0) || !std::isfinite(grid->h[a])) return STOKES_EINVAL;
    }
    const double H = wave->height, d = wave->depth, lam = wave->wavelength, om = wave->omega, g = wave->gravity;
    if (!(H >= 0.0) || !(d > 0.0) || !(lam > 0.0) || !(om > 0.0) || !(g > 0.0) || !(wave->n_cells > 0.0) ||
        !std::isfinite(H + d + lam + om + g + wave->n_cells + t))
        return STOKES_EINVAL;
    const int v = dim - 1;
    const int nvert = grid->n[v], nlat = dim == 3 ? grid->n[1] : 1;
    if (((long long)nvert + 1) * nlat >= (1LL << 31)) return STOKES_ESHAPE;
    WaveArgs w{};
    w.H = H;
    w.d = d;
    w.k = 2.0 * M_PI / lam;
    w.omega = om;
    w.g = g;
    w.t = t;
    w.eps = wave->n_cells * std::sqrt(grid->h[0] * grid->h[v]);
    const double kd = w.k * d;
    w.c2 = M_PI * H * H / (8.0 * lam) * std::cosh(kd) * (2.0 + std::cosh(2.0 * kd)) / std::pow(std::sinh(kd), 3);
    w.a1 = H * g * w.k / (2.0 * om) / std::cosh(kd);
    w.a2 = 3.0 * H * H * om * w.k / 16.0 / std::pow(std::sinh(kd), 4);
    w.eta0 = 0.5 * H * std::cos(-om * t) + w.c2 * std::cos(-2.0 * om * t);
    const long long n = (long long)(nvert + 1) * nlat;
    k_wave_inflow<<<(unsigned)((n + kWaveBlock - 1) / kWaveBlock), kWaveBlock, 0,
                    reinterpret_cast<hipStream_t>(stream)>>>(w, nvert, nlat, grid->h[v], u_n, u_t);
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}
