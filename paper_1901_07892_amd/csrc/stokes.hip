// Host side of the MI355X Stokes solver: workspace layout, coefficient setup and
// multigrid hierarchy, V-cycles, the projection preconditioner, FGMRES and the
// C-ABI declared in include/stokes.h.
//
// Everything the solver keeps lives in the caller's workspace; no device memory
// is allocated here.  All work is queued on the context's stream; the host
// synchronises once per FGMRES iteration to read the new Hessenberg column.
#include "../../include/stokes.h"
#include "kernels.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace stk;

extern "C" void *stokes_unet_stream_internal(const stokes_unet *u);

namespace {

constexpr int kMaxLev = 24;
constexpr int kDenseMax = 2048;     // largest coarsest pressure level solved densely
constexpr long long kSmallPostCells = 16 * 16 * 16;   // "small" pressure levels (lighter post-smoothing)
constexpr int kRedBlocks = 2048;    // blocks of the streaming reduction kernels
constexpr int kGroup = 8;           // vectors per multidot / maxpy launch
static_assert(kGroup >= 3, "c.partial holds the 3 partials per block of the setup min/max");
constexpr int kLearnedMaxCells = 1 << 18;   // largest level (64^3) the learned stage may run on
constexpr int kSmallMaxOps = 4096;          // passes of one small-level cycle

thread_local std::string g_setup_error;

struct HipError {
    hipError_t e;
    const char *what;
};

#define HIPCHK(call)                                                  \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) throw HipError{e_, #call};              \
    } while (0)

// ---------------------------------------------------------------- workspace carving
struct Carver {
    char *base;        // nullptr: only count
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    // nf consecutive fields of one box; returns the pointer of field 0's origin
    template <class T>
    T *fields(const Box &b, int nf) {
        T *p = take<T>((size_t)b.stride * nf);
        return p ? p + b.guard : nullptr;
    }
};

template <class R>
struct Level {
    Box b;
    R *mass[3] = {nullptr, nullptr, nullptr};
    R *beta[3] = {nullptr, nullptr, nullptr};
    R *mu = nullptr, *mxy = nullptr, *mxz = nullptr, *myz = nullptr;
    R *eu[3] = {nullptr, nullptr, nullptr}, *ru[3] = {nullptr, nullptr, nullptr}, *tu[3] = {nullptr, nullptr, nullptr};
    R *ep = nullptr, *ep2 = nullptr, *rp = nullptr;   // ep2: second buffer of the fused 3D sweep
};

template <class R>
struct MG {
    int nlev = 0;      // pressure levels
    int nvlev = 0;     // velocity levels
    Level<R> L[kMaxLev];
    R *dense = nullptr;
    int *dmap = nullptr;
    int ndense = 0;
    bool use_dense = false;
    // single-workgroup cycle of the small levels (k_p_small_cycle), from level small_l0 down
    int small_l0 = -1;
    SmallMG<R> small{};
    SmallOp *ops = nullptr;
    int nops = 0;
    size_t small_lds = 0;
};

bool can_coarsen(const Box &b) {
    bool ok = b.nx % 2 == 0 && b.ny % 2 == 0 && b.nx >= 4 && b.ny >= 4;
    if (b.dim == 3) ok = ok && b.nz % 2 == 0 && b.nz >= 4;
    long long cells = (long long)b.nx * b.ny * b.nz;
    return ok && cells > 64;
}

Box coarse_of(const Box &f) {
    Box c = make_box(f.dim, f.nx / 2, f.ny / 2, f.dim == 3 ? f.nz / 2 : 1, 2 * f.hx, 2 * f.hy, 2 * f.hz);
    c.open_top = f.open_top;
    for (int a = 0; a < 3; ++a) c.per[a] = f.per[a];
    return c;
}

}  // namespace

struct stokes_ctx {
    stokes_grid grid;
    stokes_options opt;
    double dt = 0, theta = 1, sigma = 1;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0, ws_need = 0, ws_used = 0;
    int v_clear = 0, z_clear = 0;       // leading Krylov vectors V, Z zero-filled since setup
    int dim = 3, nf = 4;
    Box fine;
    // fine-level FP64 operator
    double *mass[3] = {nullptr, nullptr, nullptr}, *beta[3] = {nullptr, nullptr, nullptr};
    double *mu = nullptr, *mxy = nullptr, *mxz = nullptr, *myz = nullptr;
    double *dinv[3] = {nullptr, nullptr, nullptr};   // inverse velocity diagonal (diagonal step)
    MG<double> mgd;
    MG<float> mgf;
    // Krylov storage: V (m+1 vectors), Z (m vectors), each nf fields of fine.stride
    int m = 30;
    long long vlen = 0;
    double unknowns = 0;        // interior unknowns (velocity faces + cells)
    double *V = nullptr, *Z = nullptr, *xk = nullptr, *bk = nullptr, *q = nullptr;
    double *partial = nullptr, *dsc = nullptr;
    double *vs = nullptr;        // scales of the unnormalised Krylov basis (m + 1)
    int *dflag = nullptr;
    int vcycles = 0;
    int cyc_first = 3, cyc_next = 3;   // pressure cycles: first / later applications of a restart cycle
    int cyc_now = 3;                    // cycles of the current application
    double p_omega = 1.0;               // pressure smoother over-relaxation (resolved p_omega)
    int nu_sec1 = 2, nu_sec2 = 2;       // pre-/post-smoothing sweeps on the second pressure level
    int nu_mid1 = 2;                    // pre-smoothing sweeps on the third and fourth pressure levels
    int nu_small2 = 2;                  // post-smoothing sweeps on the 3D levels of at most 16^3 cells
    double visc_ratio = -1.0;   // max viscous/mass diagonal ratio (automatic velocity levels)
    bool diag_vel = false;      // velocity subsolve is one diagonal step (see stokes_options.vel_smoother)
    // learned stage: network, the level it runs on, feature/prediction buffers
    stokes_unet *net = nullptr;
    int lc = -1;
    bool learned_active = false;
    double stall_ratio = 0.9;
    float *lf[4] = {nullptr, nullptr, nullptr, nullptr};   // f0, f1, f2, prediction (planar, <= 64^3)
    double *lstat = nullptr;
    // measurement: HIP events around every finest-level launch of one kernel class
    int prof_kind = -1;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double prof_ms = 0.0, prof_bytes = 0.0;
    long long prof_launches = 0;
    ~stokes_ctx() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    std::string err;

    double *vec(double *base, int j) const { return base + (size_t)j * vlen; }
    double *fld(double *vbase, int f) const { return vbase + (size_t)f * fine.stride + fine.guard; }
};

namespace {

// ---------------------------------------------------------------- layout
template <class R>
void carve_mg(Carver &cv, stokes_ctx &c, MG<R> &mg, bool alias_level0) {
    Box b = c.fine;
    int nl = 0;
    for (;;) {
        Level<R> &L = mg.L[nl];
        L.b = b;
        const int d = b.dim;
        if (nl == 0 && alias_level0) {
            // FP64 multigrid: level 0 uses the fine operator's own arrays
            for (int a = 0; a < d; ++a) {
                L.mass[a] = reinterpret_cast<R *>(c.mass[a]);
                L.beta[a] = reinterpret_cast<R *>(c.beta[a]);
            }
            L.mu = reinterpret_cast<R *>(c.mu);
            L.mxy = reinterpret_cast<R *>(c.mxy);
            L.mxz = reinterpret_cast<R *>(c.mxz);
            L.myz = reinterpret_cast<R *>(c.myz);
        } else {
            for (int a = 0; a < d; ++a) L.mass[a] = cv.fields<R>(b, 1);
            for (int a = 0; a < d; ++a) L.beta[a] = cv.fields<R>(b, 1);
            L.mu = cv.fields<R>(b, 1);
            L.mxy = cv.fields<R>(b, 1);
            if (d == 3) {
                L.mxz = cv.fields<R>(b, 1);
                L.myz = cv.fields<R>(b, 1);
            }
        }
        R *e = cv.fields<R>(b, d), *r = cv.fields<R>(b, d), *t = cv.fields<R>(b, d);
        for (int a = 0; a < d; ++a) {
            L.eu[a] = e ? e + (size_t)a * b.stride : nullptr;
            L.ru[a] = r ? r + (size_t)a * b.stride : nullptr;
            L.tu[a] = t ? t + (size_t)a * b.stride : nullptr;
        }
        L.ep = cv.fields<R>(b, 1);
        L.ep2 = cv.fields<R>(b, 1);
        L.rp = cv.fields<R>(b, 1);
        ++nl;
        if (nl >= kMaxLev || !can_coarsen(b)) break;
        b = coarse_of(b);
    }
    mg.nlev = nl;
    int vl = c.opt.vel_levels;
    mg.nvlev = (vl <= 0 || vl > nl) ? nl : vl;   // auto (vl == 0) is settled in setup
    const Box &cb = mg.L[nl - 1].b;
    mg.ndense = cb.nx * cb.ny * cb.nz;
    mg.use_dense = mg.ndense <= kDenseMax;
    if (mg.use_dense) {
        mg.dense = cv.take<R>((size_t)mg.ndense * mg.ndense);
        mg.dmap = cv.take<int>(mg.ndense);
    }
    if (b.dim == 3 && c.opt.p_small) mg.ops = cv.take<SmallOp>(kSmallMaxOps);
}

// Pairs per thread of the Krylov BLAS kernels for NV vectors: about two dozen
// pairs in flight per thread for multidot, 8-12 for maxpy (larger maxpy chunks
// take all 256 registers of a lane and leave one wave per SIMD).
constexpr int dot_pairs(int nv) { return nv == 1 ? 12 : nv == 2 ? 8 : nv == 3 ? 6 : nv <= 5 ? 4 : nv <= 7 ? 3 : 2; }
constexpr int kSelfPairs = 16;   // a squared norm: one load per pair
constexpr int axpy_pairs(int nv) { return nv == 1 ? 4 : nv == 2 ? 4 : nv == 3 ? 3 : nv <= 5 ? 2 : 1; }
inline unsigned chunk_blocks(long long n2, int pairs) {
    return (unsigned)((n2 + (long long)kBlock * pairs - 1) / ((long long)kBlock * pairs));
}
// doubles of c.partial: the per-block partials of the largest BLAS launch
// (kGroup vectors) and of the streaming reductions
inline size_t partial_doubles(long long vlen) {
    size_t need = (size_t)kRedBlocks * kGroup;
    for (int nv = 1; nv <= kGroup; ++nv) {
        need = std::max(need, (size_t)nv * chunk_blocks(vlen / 2, dot_pairs(nv)));
        need = std::max(need, (size_t)chunk_blocks(vlen / 2, axpy_pairs(nv)));
    }
    need = std::max(need, (size_t)chunk_blocks(vlen / 2, kSelfPairs));
    return need;
}

void carve_all(Carver &cv, stokes_ctx &c) {
    const Box &b = c.fine;
    const int d = c.dim;
    for (int a = 0; a < d; ++a) c.mass[a] = cv.fields<double>(b, 1);
    for (int a = 0; a < d; ++a) c.beta[a] = cv.fields<double>(b, 1);
    c.mu = cv.fields<double>(b, 1);
    c.mxy = cv.fields<double>(b, 1);
    if (d == 3) {
        c.mxz = cv.fields<double>(b, 1);
        c.myz = cv.fields<double>(b, 1);
    }
    for (int a = 0; a < d; ++a) c.dinv[a] = cv.fields<double>(b, 1);
    if (c.opt.precision == 1) carve_mg<float>(cv, c, c.mgf, false);
    else carve_mg<double>(cv, c, c.mgd, true);
    c.vlen = (long long)b.stride * c.nf;
    c.V = cv.take<double>((size_t)c.vlen * (c.m + 1));
    c.Z = cv.take<double>((size_t)c.vlen * c.m);
    c.xk = cv.take<double>((size_t)c.vlen);
    c.bk = cv.take<double>((size_t)c.vlen);
    c.q = cv.fields<double>(b, 1);
    c.partial = cv.take<double>(partial_doubles(c.vlen));
    c.dsc = cv.take<double>(4 * (size_t)(c.m + 8));
    c.vs = cv.take<double>((size_t)c.m + 2);
    if (d == 3)
        for (int a = 0; a < 4; ++a) c.lf[a] = cv.take<float>((size_t)kLearnedMaxCells);
    c.lstat = cv.take<double>(8);
    c.dflag = cv.take<int>(64);
    c.ws_used = cv.off;
    c.ws_need = cv.off + 256;   // room to start the carving at a 256-byte boundary
}

// The z-marching kernels assume walls on every side; a level with a periodic
// axis takes the flat kernels, which wrap.
inline bool any_periodic(const Box &b) { return b.per[0] || b.per[1] || b.per[2]; }

// ---------------------------------------------------------------- launch helpers
template <int DIM, class R>
void prolong_add(stokes_ctx &c, const Box &fb, const Box &cb, int lin, const R *ec, R *f);
inline unsigned nblocks_box(const Box &b) { return (unsigned)((b.nb + kBlock - 1) / kBlock); }
inline unsigned nblocks_stream(long long n) {
    long long g = (n + kBlock - 1) / kBlock;
    return (unsigned)std::max<long long>(1, std::min<long long>(g, kRedBlocks));
}

// Records a pair of HIP events around one launch when that kernel class is
// being measured (finest level only); the bytes are the launch's algorithmic
// traffic.
struct ProfScope {
    stokes_ctx &c;
    bool on;
    ProfScope(stokes_ctx &cc, int kind, double bytes, bool finest = true) : c(cc) {
        on = finest && c.prof_kind == kind && c.ev_used + 2 <= c.ev.size();
        if (on) {
            HIPCHK(hipEventRecord(c.ev[c.ev_used], c.stream));
            c.prof_bytes += bytes;
            c.prof_launches++;
        }
    }
    ~ProfScope() {
        if (on) {
            (void)hipEventRecord(c.ev[c.ev_used + 1], c.stream);
            c.ev_used += 2;
        }
    }
};

void prof_collect(stokes_ctx &c) {
    for (size_t t = 0; t + 1 < c.ev_used; t += 2) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, c.ev[t], c.ev[t + 1]));
        c.prof_ms += ms;
    }
    c.ev_used = 0;
}

template <class R>
VelCoef<R> vcoef(const Level<R> &L, double theta) {
    VelCoef<R> c;
    for (int a = 0; a < 3; ++a) c.mass[a] = L.mass[a];
    c.mu = L.mu;
    c.mxy = L.mxy;
    c.mxz = L.mxz;
    c.myz = L.myz;
    c.theta = (R)theta;
    return c;
}

VelCoef<double> fine_coef(const stokes_ctx &c) {
    VelCoef<double> v;
    for (int a = 0; a < 3; ++a) v.mass[a] = c.mass[a];
    v.mu = c.mu;
    v.mxy = c.mxy;
    v.mxz = c.mxz;
    v.myz = c.myz;
    v.theta = c.theta;
    return v;
}

// blocks of the row-form layout conversion kernels (kPackRows box rows each)
inline unsigned nblocks_rows(const Box &b) { return (unsigned)((b.py * b.pz + kPackRows - 1) / kPackRows); }

// dst[0, n) = src[0, n) (n > 0) with the streaming-copy kernel: 16-byte
// non-temporal accesses when both are 16-byte aligned, one pair per thread.
inline void stream_copy(const double *src, double *dst, long long n, hipStream_t stream) {
    const bool vec2 = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    const long long work = vec2 ? (n + 1) / 2 : n;
    const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>((work + kBlock - 1) / kBlock, 1 << 22));
    k_stream_copy<<<g, kBlock, 0, stream>>>(n, src, dst, vec2 ? 1 : 0);
}

template <class R>
void fill(stokes_ctx &c, R *p, long long n, R v) {
    k_fill<R><<<nblocks_stream(n), kBlock, 0, c.stream>>>(n, p, v);
}

// V[0, nv) and Z[0, nz) zero-filled before their first use after setup.  The
// workspace clear at setup leaves the Krylov vectors out (they are most of the
// workspace: 2 m + 1 vectors for restart length m), and a solve that converges
// in a few iterations touches only the first few of them.
void touch_krylov(stokes_ctx &c, int nv, int nz) {
    auto zero = [&](double *x, long long n) {
        if (reinterpret_cast<uintptr_t>(x) & 15) { fill<double>(c, x, n, 0.0); return; }
        const long long work = (n + 1) / 2;
        const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>((work + kBlock - 1) / kBlock, 1 << 22));
        k_zero<<<g, kBlock, 0, c.stream>>>(n, x);
    };
    nv = std::min(nv, c.m + 1);
    nz = std::min(nz, c.m);
    if (nv > c.v_clear) {
        zero(c.vec(c.V, c.v_clear), (long long)(nv - c.v_clear) * c.vlen);
        c.v_clear = nv;
    }
    if (nz > c.z_clear) {
        zero(c.vec(c.Z, c.z_clear), (long long)(nz - c.z_clear) * c.vlen);
        c.z_clear = nz;
    }
}

// ---------------------------------------------------------------- velocity multigrid
template <int DIM, class R>
void vel_smooth(stokes_ctx &c, Level<R> &L, R *const e[3], R *const r[3], int sweeps, bool zero_guess) {
    VelCoef<R> co = vcoef(L, c.theta);
    for (int s = 0; s < sweeps; ++s) {
        for (int comp = 0; comp < DIM; ++comp) {
            for (int colour = 0; colour < 2; ++colour) {
                int valid = VALID_U | VALID_V | VALID_W;
                if (zero_guess && s == 0) {
                    valid = 0;
                    for (int a = 0; a < comp; ++a) valid |= 1 << a;
                    if (colour == 1) valid |= 1 << comp;
                }
                k_vel_gs<DIM, R><<<nblocks_box(L.b), kBlock, 0, c.stream>>>(
                    L.b, co, comp, colour, valid, e[0], e[1], e[2], r[0], r[1], r[2]);
            }
        }
    }
}

template <int DIM, class R>
void vel_vcycle(stokes_ctx &c, MG<R> &mg, int l, R *const e[3], R *const r[3], bool zero_guess) {
    Level<R> &L = mg.L[l];
    const int nu1 = c.opt.nu1, nu2 = c.opt.nu2;
    if (l == mg.nvlev - 1) {
        int sw = l == 0 ? c.opt.vel_sweeps : std::max(1, c.opt.coarse_sweeps);
        vel_smooth<DIM, R>(c, L, e, r, sw, zero_guess);
        return;
    }
    if (zero_guess && nu1 == 0)
        for (int a = 0; a < DIM; ++a) fill<R>(c, e[a] - L.b.guard, L.b.stride, R(0));
    vel_smooth<DIM, R>(c, L, e, r, nu1, zero_guess);
    Level<R> &C = mg.L[l + 1];
    k_vel_residual<DIM, R><<<nblocks_box(L.b), kBlock, 0, c.stream>>>(
        L.b, vcoef(L, c.theta), e[0], e[1], e[2], r[0], r[1], r[2], L.tu[0], L.tu[1], L.tu[2]);
    for (int a = 0; a < DIM; ++a)
        k_face_restrict<DIM, R><<<nblocks_box(C.b), kBlock, 0, c.stream>>>(L.b, C.b, a, L.tu[a], C.ru[a]);
    vel_vcycle<DIM, R>(c, mg, l + 1, C.eu, C.ru, true);
    for (int a = 0; a < DIM; ++a)
        k_face_prolong_add<DIM, R><<<nblocks_box(L.b), kBlock, 0, c.stream>>>(L.b, C.b, a, C.eu[a], e[a]);
    vel_smooth<DIM, R>(c, L, e, r, nu2, false);
}

// ---------------------------------------------------------------- pressure multigrid
// Coarse cycles per visit of level l: p_gamma on the p_wdepth finest levels (all
// when p_wdepth = 0), one below; one when the coarse level is solved exactly.
template <class R>
int gamma_at(const stokes_ctx &c, const MG<R> &mg, int l) {
    if (l + 1 >= mg.nlev - 1) return 1;
    return (c.opt.p_wdepth == 0 || l < c.opt.p_wdepth) ? c.opt.p_gamma : 1;
}

// f += the prolonged coarse correction on the cells of level fb
template <int DIM, class R>
void prolong_add(stokes_ctx &c, const Box &fb, const Box &cb, int lin, const R *ec, R *f) {
    if (any_periodic(fb))
        k_p_prolong_add<DIM, R, true><<<nblocks_box(fb), kBlock, 0, c.stream>>>(fb, cb, lin, ec, f);
    else
        k_p_prolong_add<DIM, R, false><<<nblocks_box(fb), kBlock, 0, c.stream>>>(fb, cb, lin, ec, f);
}

// Pre- and post-smoothing sweeps of pressure level l.
inline int p_nu_pre(const stokes_ctx &c, int l) { return l == 1 ? c.nu_sec1 : (l == 2 || l == 3) ? c.nu_mid1 : c.opt.nu1; }
inline int p_nu_post(const stokes_ctx &c, int l) {
    if (l == 1) return c.nu_sec2;
    // the small levels (at most 16^3 cells, coarsened from the fine box by 2 per axis)
    if (c.dim == 3 && l >= 2 &&
        (long long)(c.fine.nx >> l) * (c.fine.ny >> l) * (c.fine.nz >> l) <= kSmallPostCells)
        return c.nu_small2;
    return c.opt.nu2;
}

// The first sweep after a coarse correction on a flat level with walls: the
// prolongation folded into its two colour passes (k_p_gs_ec), the values of
// prolong_add + p_smooth with one launch less.
template <int DIM, class R>
void p_sweep_flat_ec(stokes_ctx &c, Level<R> &L, R *e, const R *r, const R *ec, const Box &cb) {
    const R *bz = DIM == 3 ? L.beta[2] : L.beta[1];
    for (int colour = 0; colour < 2; ++colour)
        k_p_gs_ec<DIM, R><<<nblocks_box(L.b), kBlock, 0, c.stream>>>(L.b, colour, R(c.p_omega), e, r, L.beta[0],
                                                                      L.beta[1], bz, cb, c.opt.p_prolong, ec);
}

template <int DIM, class R>
void p_smooth(stokes_ctx &c, Level<R> &L, R *e, const R *r, int sweeps, bool zero_guess) {
    const bool per = any_periodic(L.b);
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            const int zg = (zero_guess && s == 0 && colour == 0) ? 1 : 0;
            const R *bz = DIM == 3 ? L.beta[2] : L.beta[1];
            if (per)
                k_p_gs<DIM, R, true><<<nblocks_box(L.b), kBlock, 0, c.stream>>>(L.b, colour, zg, R(c.p_omega), e, r, L.beta[0], L.beta[1], bz);
            else
                k_p_gs<DIM, R, false><<<nblocks_box(L.b), kBlock, 0, c.stream>>>(L.b, colour, zg, R(c.p_omega), e, r, L.beta[0], L.beta[1], bz);
        }
}

// One fused 3D sweep from `in` into `out` (optionally adding the prolonged coarse
// correction `ec` to the old values first).  Levels of at least 2^20 cells use
// the two-barrier kernel on 64x16 tiles (1024 threads, low halo fraction);
// smaller ones the one-barrier pipelined kernel on 32x16 or 32x8 tiles.
template <class R, int TX, int TY, bool PIPE>
void p_sweep3_launch(stokes_ctx &c, Level<R> &L, const R *in, R *out, const R *r, bool zero_guess,
                     const R *ec, const Box *cb, int min_blocks) {
    const Box &b = L.b;
    int gx = (b.nx + TX - 1) / TX, gy = (b.ny + TY - 1) / TY;
    // z chunks: enough blocks to fill the chip, at least 8 planes per chunk
    int kc = b.nz;
    while (kc > 8 && (long long)gx * gy * ((b.nz + kc - 1) / kc) < min_blocks) kc = (kc + 1) / 2;
    int gz = (b.nz + kc - 1) / kc;
    const double cells = (double)b.nx * b.ny * b.nz;
    // new iterate, right-hand side, three face coefficients, the old iterate unless
    // the sweep starts from zero (+ 1/8 field for a folded coarse correction)
    ProfScope ps(c, STOKES_PROF_P_SWEEP, cells * sizeof(R) * ((zero_guess ? 5.0 : 6.0) + (ec ? 0.125 : 0.0)),
                 b.nx == c.fine.nx);
    if (PIPE)
        k_p_sweep3<R, TX, TY><<<dim3(gx, gy, gz), TX * TY, 0, c.stream>>>(
            b, kc, zero_guess ? 1 : 0, R(c.p_omega), in, ec, cb ? *cb : b, c.opt.p_prolong, out, r, L.beta[0], L.beta[1], L.beta[2]);
    else
        k_p_sweep3c<R, TX, TY, sizeof(R) == 4><<<dim3(gx, gy, gz), TX * TY, 0, c.stream>>>(
            b, kc, zero_guess ? 1 : 0, R(c.p_omega), in, ec, cb ? *cb : b, c.opt.p_prolong, out, r, L.beta[0], L.beta[1], L.beta[2]);
}

template <class R>
void p_sweep3(stokes_ctx &c, Level<R> &L, const R *in, R *out, const R *r, bool zero_guess,
              const R *ec, const Box *cb) {
    const long long cells = (long long)L.b.nx * L.b.ny * L.b.nz;
    if (cells >= (1LL << 20) && L.b.nx >= 64 && L.b.ny >= 16)
        p_sweep3_launch<R, 64, 16, false>(c, L, in, out, r, zero_guess, ec, cb, 512);
    else if (L.b.nx >= 32 && L.b.ny >= 16)
        p_sweep3_launch<R, 32, 16, true>(c, L, in, out, r, zero_guess, ec, cb, 1024);
    else
        p_sweep3_launch<R, 32, 8, true>(c, L, in, out, r, zero_guess, ec, cb, 2048);
}

// Coarse right-hand side rc = average over the 2^d children of r - (-L_rho) e,
// from level L to the next-coarser level C.  3D levels of at least 2^21 cells
// use the z-marching kernel (each fine plane read once), the others (or all
// with flat_only) the per-cell kernel; same formulas and summation order.
template <int DIM, class R>
void p_residual_restrict(stokes_ctx &c, const Level<R> &L, const Level<R> &C, const R *e, const R *r, R *rc,
                         bool flat_only) {
    const R *bz = DIM == 3 ? L.beta[2] : L.beta[1];
    if (DIM == 3 && !flat_only && !any_periodic(L.b) && (long long)L.b.nx * L.b.ny * L.b.nz >= (1LL << 21)) {
        constexpr int TX = 64, TY = 4;
        const int gx = (C.b.nx + TX - 1) / TX, gy = (C.b.ny + TY - 1) / TY;
        int kc = C.b.nz;
        while (kc > 2 && (long long)gx * gy * ((C.b.nz + kc - 1) / kc) < 1024) kc = (kc + 1) / 2;
        const int gz = (C.b.nz + kc - 1) / kc;
        k_p_residual_restrict3_z<R, TX, TY><<<dim3(gx, gy, gz), TX * TY, 0, c.stream>>>(
            L.b, C.b, kc, e, r, L.beta[0], L.beta[1], bz, rc);
    } else {
        if (any_periodic(L.b))
            k_p_residual_restrict<DIM, R, true><<<nblocks_box(C.b), kBlock, 0, c.stream>>>(L.b, C.b, e, r, L.beta[0], L.beta[1], bz, rc);
        else
            k_p_residual_restrict<DIM, R, false><<<nblocks_box(C.b), kBlock, 0, c.stream>>>(L.b, C.b, e, r, L.beta[0], L.beta[1], bz, rc);
    }
}

// One red-black Gauss-Seidel sweep of -L_rho e = r on level L, starting from
// *cur (zero when zg; plus the prolonged coarse correction ec of level cb when
// ec != nullptr).  Levels of at most 64^3 cells (and every 2D level, or all
// with flat_only) take two flat colour passes in place; larger 3D levels the
// fused z-marching kernel from *cur into *spare, after which the two pointers
// are swapped, so *cur always names the array that holds the new iterate.
template <int DIM, class R>
void p_level_sweep(stokes_ctx &c, Level<R> &L, R *&cur, R *&spare, const R *r, bool zg, const R *ec, const Box *cb,
                   bool flat_only) {
    // levels of at most 64^3 cells are latency-bound: two flat colour passes beat
    // a z-marching launch there
    const bool flat = DIM == 2 || flat_only || any_periodic(L.b) || (long long)L.b.nx * L.b.ny * L.b.nz <= (1LL << 18);
    if (flat) {
        if (ec && !flat_only && !any_periodic(L.b)) {
            p_sweep_flat_ec<DIM, R>(c, L, cur, r, ec, *cb);
            return;
        }
        if (ec) prolong_add<DIM, R>(c, L.b, *cb, c.opt.p_prolong, ec, cur);
        p_smooth<DIM, R>(c, L, cur, r, 1, zg);
        return;
    }
    p_sweep3<R>(c, L, cur, spare, r, zg, ec, cb);
    std::swap(cur, spare);
}

// V-cycle on -L_rho e = r at level l.  Returns the array that holds the new
// iterate: e itself, or (3D, after an odd number of fused sweeps) the level's
// other buffer.
template <int DIM, class R>
R *p_vcycle(stokes_ctx &c, MG<R> &mg, int l, R *e, R *r, bool zero_guess) {
    if (DIM == 3 && l == mg.small_l0) {
        auto kern = any_periodic(mg.small.b[0]) ? k_p_small_cycle<R, true> : k_p_small_cycle<R, false>;
        kern<<<1, kSmallThreads, mg.small_lds, c.stream>>>(mg.small, mg.ops, mg.nops,
                                                                       zero_guess ? 1 : 0, e, r);
        return e;
    }
    Level<R> &L = mg.L[l];
    R *cur = e;
    R *spare = (e == L.ep) ? L.ep2 : L.ep;
    auto sweep = [&](bool zg, const R *ec, const Box *cb) {
        p_level_sweep<DIM, R>(c, L, cur, spare, r, zg, ec, cb, false);
    };
    if (l == mg.nlev - 1) {
        if (mg.use_dense) {
            k_dense_solve<R><<<1, 1024, mg.ndense * sizeof(R), c.stream>>>(mg.ndense, mg.dense, mg.dmap, r, e);
        } else if (DIM == 3) {
            for (int s = 0; s < std::max(1, c.opt.coarse_sweeps); ++s) sweep(zero_guess && s == 0, nullptr, nullptr);
        } else {
            p_smooth<DIM, R>(c, L, e, r, std::max(1, c.opt.coarse_sweeps), zero_guess);
        }
        return cur;
    }
    const int nu1 = p_nu_pre(c, l), nu2 = p_nu_post(c, l);
    if (zero_guess && nu1 == 0) fill<R>(c, cur - L.b.guard, L.b.stride, R(0));
    if (DIM == 3) {
        for (int s = 0; s < nu1; ++s) sweep(zero_guess && s == 0, nullptr, nullptr);
    } else {
        p_smooth<DIM, R>(c, L, cur, r, nu1, zero_guess);
    }
    Level<R> &C = mg.L[l + 1];
    p_residual_restrict<DIM, R>(c, L, C, cur, r, C.rp, false);
    R *ce = p_vcycle<DIM, R>(c, mg, l + 1, C.ep, C.rp, true);
    // W-cycle (p_gamma = 2): a second coarse cycle on the same coarse equation
    // (pointless above the exactly solved coarsest level)
    for (int g = 1; g < gamma_at(c, mg, l); ++g) ce = p_vcycle<DIM, R>(c, mg, l + 1, ce, C.rp, false);
    if (DIM == 3 && nu2 > 0) {
        sweep(false, ce, &C.b);                    // prolongation folded into the first post-sweep
        for (int s = 1; s < nu2; ++s) sweep(false, nullptr, nullptr);
    } else if (DIM == 2 && nu2 > 0 && !any_periodic(L.b)) {
        p_sweep_flat_ec<DIM, R>(c, L, cur, r, ce, C.b);   // prolongation folded into the first post-sweep
        p_smooth<DIM, R>(c, L, cur, r, nu2 - 1, false);
    } else {
        prolong_add<DIM, R>(c, L.b, C.b, c.opt.p_prolong, ce, cur);
        if (DIM == 3) {
            for (int s = 0; s < nu2; ++s) sweep(false, nullptr, nullptr);
        } else {
            p_smooth<DIM, R>(c, L, cur, r, nu2, false);
        }
    }
    return cur;
}

// ---------------------------------------------------------------- learned stage
// Initial guess for the pressure cycles from the network: the pressure
// right-hand side is restricted to the learned level, scaled to unit RMS and
// fed with the static features; the prediction's amplitude is fitted by least
// squares against that level's operator, and the result is prolonged
// (trilinearly, level by level) to the finest level.
template <class R>
void restrict_rhs_to(stokes_ctx &c, MG<R> &mg, int lc) {
    const R *src = mg.L[0].rp;
    for (int l = 0; l < lc; ++l) {
        k_restrict_avg3<R><<<nblocks_box(mg.L[l + 1].b), kBlock, 0, c.stream>>>(mg.L[l].b, mg.L[l + 1].b, src, mg.L[l + 1].rp);
        src = mg.L[l + 1].rp;
    }
}

// A coarse prediction in mg.L[lc].ep2 (with the restricted right-hand side in
// that level's rp) -> fitted amplitude, prolonged trilinearly to phi0.
template <class R>
void guess_from_coarse(stokes_ctx &c, MG<R> &mg, int lc, R *phi0) {
    Level<R> &C = mg.L[lc];
    k_p_apply3<R><<<nblocks_box(C.b), kBlock, 0, c.stream>>>(C.b, C.ep2, C.beta[0], C.beta[1], C.beta[2], C.ep);
    k_fit_amplitude<R><<<1, 1024, 0, c.stream>>>(C.b, C.ep, C.rp, C.ep2, c.lstat);
    R *cur = C.ep2;
    for (int l = lc - 1; l >= 0; --l) {
        R *dst = l == 0 ? phi0 : mg.L[l].ep2;
        fill<R>(c, dst - mg.L[l].b.guard, mg.L[l].b.stride, R(0));
        prolong_add<3, R>(c, mg.L[l].b, mg.L[l + 1].b, 1, cur, dst);
        cur = dst;
    }
}

template <class R>
void learned_guess(stokes_ctx &c, MG<R> &mg, R *phi0) {
    const int lc = c.lc;
    restrict_rhs_to<R>(c, mg, lc);
    Level<R> &C = mg.L[lc];
    const int nc = C.b.nx * C.b.ny * C.b.nz;
    k_normalise_planar<R><<<1, 1024, 0, c.stream>>>(C.b, C.rp, 0, c.lf[2], c.lstat);
    stokes_status st = stokes_unet_forward(c.net, c.lf[0], c.lf[1], c.lf[2], c.lf[3]);
    if (st != STOKES_OK) throw HipError{hipErrorUnknown, "stokes_unet_forward"};
    k_planar_to_box<R><<<(nc + kBlock - 1) / kBlock, kBlock, 0, c.stream>>>(C.b, c.lf[3], C.ep2);
    guess_from_coarse<R>(c, mg, lc, phi0);
}

// Pressure subsolve of the preconditioner: cyc_now cycles on -L_rho phi = r
// (level 0 right-hand side already in L0.rp), from zero or from the learned
// guess.  Returns the array holding phi.
template <int DIM, class R>
R *pressure_cycles(stokes_ctx &c, MG<R> &mg) {
    Level<R> &L0 = mg.L[0];
    R *phi = L0.ep;
    bool zero = true;
    if (DIM == 3 && c.net && c.learned_active) {
        learned_guess<R>(c, mg, phi);
        zero = false;
    }
    for (int cyc = 0; cyc < c.cyc_now; ++cyc) {
        phi = p_vcycle<DIM, R>(c, mg, 0, phi, L0.rp, zero && cyc == 0);
        c.vcycles++;
    }
    return phi;
}

// ---------------------------------------------------------------- preconditioner
// z = P^{-1} v:
//   1. u~ ~= A^{-1} v_u                      (velocity V-cycles)
//   2. q = v_p + D u~,  s = q / dt
//   3. phi ~= L_rho^{-1} s, L_rho = D beta G (pressure V-cycles on -L_rho)
//   4. z_u = u~ - dt beta G phi
//   5. z_p = phi - 2 theta mu q              (local-viscosity pressure update)
// Its derivation: with constant coefficients A (dt beta G phi) = G p exactly
// when p = phi - 2 theta mu dt beta Lap(phi), and beta Lap(phi) ~= s.
template <int DIM, class R>
void precond(stokes_ctx &c, MG<R> &mg, double *v, double vs, double *z) {
    Level<R> &L0 = mg.L[0];
    double *vu[3] = {c.fld(v, 0), c.fld(v, 1), DIM == 3 ? c.fld(v, 2) : nullptr};
    double *zu[3] = {c.fld(z, 0), c.fld(z, 1), DIM == 3 ? c.fld(z, 2) : nullptr};
    double *vp = c.fld(v, DIM), *zp = c.fld(z, DIM);
    if (c.diag_vel) {
        // step 1 as one diagonal step, folded into the divergence and update kernels
        double *d2 = DIM == 3 ? c.dinv[2] : c.dinv[1];
        k_precond_div_jac<DIM, R><<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(
            c.fine, vu[0], vu[1], DIM == 3 ? vu[2] : vu[1], c.dinv[0], c.dinv[1], d2, vp, vs, c.dt, c.q, L0.rp);
        R *phi = pressure_cycles<DIM, R>(c, mg);
        k_precond_update_jac<DIM, R><<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(
            c.fine, vu[0], vu[1], DIM == 3 ? vu[2] : vu[1], c.dinv[0], c.dinv[1], d2, vs, phi, c.beta[0], c.beta[1],
            DIM == 3 ? c.beta[2] : c.beta[1], c.mu, c.q, c.dt, c.theta, zu[0], zu[1], DIM == 3 ? zu[2] : zu[1], zp);
        return;
    }
    // the multigrid velocity path reads v as it is (the caller passes vs = 1)
    R *eu[3], *ru[3];
    if (sizeof(R) == sizeof(double)) {
        for (int a = 0; a < 3; ++a) {
            eu[a] = reinterpret_cast<R *>(zu[a]);
            ru[a] = reinterpret_cast<R *>(vu[a]);
        }
    } else {
        long long n = (long long)DIM * c.fine.stride;
        k_cast<double, R><<<nblocks_stream(n), kBlock, 0, c.stream>>>(n, v, L0.ru[0] - L0.b.guard);
        for (int a = 0; a < 3; ++a) {
            eu[a] = L0.eu[a];
            ru[a] = L0.ru[a];
        }
    }
    if (c.opt.vel_cycles <= 0) {
        for (int a = 0; a < DIM; ++a) fill<R>(c, eu[a] - L0.b.guard, L0.b.stride, R(0));
    }
    for (int cyc = 0; cyc < c.opt.vel_cycles; ++cyc) {
        vel_vcycle<DIM, R>(c, mg, 0, eu, ru, cyc == 0);
        c.vcycles++;
    }
    k_precond_div<DIM, R><<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(c.fine, eu[0], eu[1], eu[2], vp, c.dt, c.q, L0.rp);
    R *phi = pressure_cycles<DIM, R>(c, mg);
    k_precond_update<DIM, R><<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(
        c.fine, eu[0], eu[1], eu[2], phi, c.beta[0], c.beta[1], DIM == 3 ? c.beta[2] : c.beta[1], c.mu, c.q,
        c.dt, c.theta, zu[0], zu[1], DIM == 3 ? zu[2] : zu[1], zp);
}

// ---------------------------------------------------------------- BLAS helpers
template <int NV, bool SELF = false>
unsigned launch_multidot(stokes_ctx &c, const double *V, const double *w, double w2) {
    constexpr int P = SELF ? kSelfPairs : dot_pairs(NV);
    const long long n2 = c.vlen / 2;
    const unsigned g = chunk_blocks(n2, P);
    k_multidot<NV, P, SELF><<<g, kBlock, 0, c.stream>>>(n2, (long long)c.dim * c.fine.stride / 2, w2,
                                                   reinterpret_cast<const dpair *>(V), n2,
                                                   reinterpret_cast<const dpair *>(w), c.partial);
    return g;
}

template <int NV>
unsigned launch_maxpy(stokes_ctx &c, double sign, const double *V, const double *coef, const double *vscale,
                      double *w, double w2, double *partial) {
    constexpr int P = axpy_pairs(NV);
    const long long n2 = c.vlen / 2;
    const unsigned g = chunk_blocks(n2, P);
    k_maxpy<NV, P><<<g, kBlock, 0, c.stream>>>(n2, sign, reinterpret_cast<const dpair *>(V), n2, coef, vscale,
                                                reinterpret_cast<dpair *>(w), (long long)c.dim * c.fine.stride / 2,
                                                w2, partial);
    return g;
}

// The vectors of the Krylov BLAS: vlen even (a multiple of 64) and every
// vector 16-byte aligned (carved at 256-byte boundaries, vlen * 8 bytes apart).
inline void check_pairs(const stokes_ctx &c, const double *p) {
    if ((c.vlen & 1) || (reinterpret_cast<uintptr_t>(p) & 15)) throw HipError{hipErrorInvalidValue, "Krylov vector alignment"};
}

// out[0..nv) = scale[m] * <V_m, w>_W for m < nv (W: pressure block weighted by w2;
// scale = 1 when nullptr)
void multidot(stokes_ctx &c, const double *V, int nv, const double *w, double w2, double *out,
              const double *scale = nullptr) {
    check_pairs(c, V);
    check_pairs(c, w);
    for (int m0 = 0; m0 < nv; m0 += kGroup) {
        int cnt = std::min(kGroup, nv - m0);
        const double *Vm = V + (size_t)m0 * c.vlen;
        // a squared norm (V_0 = w) reads one vector
        ProfScope ps(c, STOKES_PROF_MULTIDOT, (double)(cnt == 1 && Vm == w ? 1 : cnt + 1) * c.unknowns * 8.0);
        unsigned g = 0;
        switch (cnt) {
        case 1: g = Vm == w ? launch_multidot<1, true>(c, Vm, w, w2) : launch_multidot<1>(c, Vm, w, w2); break;
        case 2: g = launch_multidot<2>(c, Vm, w, w2); break;
        case 3: g = launch_multidot<3>(c, Vm, w, w2); break;
        case 4: g = launch_multidot<4>(c, Vm, w, w2); break;
        case 5: g = launch_multidot<5>(c, Vm, w, w2); break;
        case 6: g = launch_multidot<6>(c, Vm, w, w2); break;
        case 7: g = launch_multidot<7>(c, Vm, w, w2); break;
        default: g = launch_multidot<8>(c, Vm, w, w2); break;
        }
        k_reduce_partials<<<cnt, kBlock, 0, c.stream>>>((int)g, c.partial, out + m0, 0, scale ? scale + m0 : nullptr);
    }
}

// w += sign * sum_m coef[m] vscale[m] V_m   (coef and vscale on the device;
// vscale = 1 when nullptr).  With nrm2 != nullptr the weighted squared norm of
// the result is reduced into nrm2[0].
void maxpy(stokes_ctx &c, double sign, const double *V, int nv, const double *coef, double *w,
           double w2 = 1.0, double *nrm2 = nullptr, const double *vscale = nullptr) {
    check_pairs(c, V);
    check_pairs(c, w);
    unsigned g = 0;
    for (int m0 = 0; m0 < nv; m0 += kGroup) {
        int cnt = std::min(kGroup, nv - m0);
        bool last = m0 + kGroup >= nv;
        ProfScope ps(c, STOKES_PROF_MAXPY, (double)(cnt + 2) * c.unknowns * 8.0);
        const double *Vm = V + (size_t)m0 * c.vlen;
        const double *cm = coef + m0, *sm = vscale ? vscale + m0 : nullptr;
        double *part = (last && nrm2) ? c.partial : nullptr;
        switch (cnt) {
        case 1: g = launch_maxpy<1>(c, sign, Vm, cm, sm, w, w2, part); break;
        case 2: g = launch_maxpy<2>(c, sign, Vm, cm, sm, w, w2, part); break;
        case 3: g = launch_maxpy<3>(c, sign, Vm, cm, sm, w, w2, part); break;
        case 4: g = launch_maxpy<4>(c, sign, Vm, cm, sm, w, w2, part); break;
        case 5: g = launch_maxpy<5>(c, sign, Vm, cm, sm, w, w2, part); break;
        case 6: g = launch_maxpy<6>(c, sign, Vm, cm, sm, w, w2, part); break;
        case 7: g = launch_maxpy<7>(c, sign, Vm, cm, sm, w, w2, part); break;
        default: g = launch_maxpy<8>(c, sign, Vm, cm, sm, w, w2, part); break;
        }
    }
    if (nrm2) k_reduce_partials<<<1, kBlock, 0, c.stream>>>((int)g, c.partial, nrm2, 0, nullptr);
}

void sync_read(stokes_ctx &c, const double *dsrc, double *hdst, int n) {
    HIPCHK(hipMemcpyAsync(hdst, dsrc, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
}

template <int DIM>
void apply_fine(stokes_ctx &c, double *x, double *f, double *y) {
    const double cells = (double)c.fine.nx * c.fine.ny * c.fine.nz;
    // x: 4 unknown fields, coefficients: DIM mass + mu + edges; y: 4 fields; f: 4 more
    const int nedge = DIM == 3 ? 3 : 1;
    ProfScope ps(c, STOKES_PROF_MATVEC, cells * 8.0 * ((DIM + 1) * (f ? 3 : 2) + DIM + 1 + nedge));
    if (DIM == 3 && c.opt.matvec_z && !any_periodic(c.fine)) {
        constexpr int TX = 64, TY = 8;
        const Box &b = c.fine;
        int gx = (b.nx + TX - 1) / TX, gy = (b.ny + TY - 1) / TY;
        int kc = b.nz;
        while (kc > 8 && (long long)gx * gy * ((b.nz + kc - 1) / kc) < 2048) kc = (kc + 1) / 2;
        int gz = (b.nz + kc - 1) / kc;
        k_apply3_z<TX, TY><<<dim3(gx, gy, gz), TX * TY, 0, c.stream>>>(
            b, kc, fine_coef(c), c.fld(x, 0), c.fld(x, 1), c.fld(x, 2), c.fld(x, 3),
            f ? c.fld(f, 0) : nullptr, f ? c.fld(f, 1) : nullptr, f ? c.fld(f, 2) : nullptr,
            f ? c.fld(f, 3) : nullptr, c.fld(y, 0), c.fld(y, 1), c.fld(y, 2), c.fld(y, 3));
        if (b.open_top)
            k_apply_top3<<<(unsigned)((b.nx * b.ny + kBlock - 1) / kBlock), kBlock, 0, c.stream>>>(
                b, fine_coef(c), c.fld(x, 0), c.fld(x, 1), c.fld(x, 2), c.fld(x, 3), f ? c.fld(f, 2) : nullptr,
                c.fld(y, 2));
        return;
    }
    k_apply<DIM><<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(
        c.fine, fine_coef(c), c.fld(x, 0), c.fld(x, 1), DIM == 3 ? c.fld(x, 2) : nullptr, c.fld(x, DIM),
        f ? c.fld(f, 0) : nullptr, f ? c.fld(f, 1) : nullptr, (f && DIM == 3) ? c.fld(f, 2) : nullptr,
        f ? c.fld(f, DIM) : nullptr, c.fld(y, 0), c.fld(y, 1), DIM == 3 ? c.fld(y, 2) : nullptr, c.fld(y, DIM));
}

void remove_p_mean(stokes_ctx &c, double *x) {
    double *p = c.fld(x, c.dim) - c.fine.guard;
    const long long n = c.fine.stride;
    const unsigned g = nblocks_stream(n);
    k_partial_sum<<<g, kBlock, 0, c.stream>>>(n, p, 0, c.partial);
    k_reduce_partials<<<1, kBlock, 0, c.stream>>>((int)g, c.partial, c.dsc, 0, nullptr);
    k_sub_mean<<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(c.fine, c.dsc, c.fld(x, c.dim));
}

// ---------------------------------------------------------------- FGMRES
template <int DIM, class R>
stokes_status fgmres(stokes_ctx &c, MG<R> &mg, double tol, bool zero_guess, stokes_stats &st) {
    const int m = c.m;
    const double w2 = c.sigma * c.sigma;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m), hbuf(2 * m + 4);
    // The Krylov basis is kept unnormalised: v_j = hs[j] * V_j, with the scales
    // also on the device (c.vs) for the Gram-Schmidt kernels.  This saves one
    // pass over every new basis vector; the preconditioner is positively
    // homogeneous, so it takes the scale as an argument.
    std::vector<double> hs(m + 1, 1.0);
    auto set_scale = [&](int j, double v) {
        hs[j] = v;
        k_set_scalar<<<1, 64, 0, c.stream>>>(c.vs + j, v);
    };
    auto HH = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    double *dh = c.dsc, *dh2 = c.dsc + (m + 2), *dy = c.dsc + 2 * (m + 2);

    multidot(c, c.bk, 1, c.bk, w2, dh);
    double bn2;
    sync_read(c, dh, &bn2, 1);
    if (!std::isfinite(bn2)) { c.err = "non-finite right-hand side"; return STOKES_ENAN; }
    const double bnorm = std::sqrt(bn2);
    st.iters = 0;
    st.restarts = 0;
    if (bnorm == 0.0) {
        fill<double>(c, c.xk, c.vlen, 0.0);
        fill<double>(c, c.vec(c.V, 0), c.vlen, 0.0);   // its residual
        st.rel_res_est = st.rel_res_true = 0.0;
        return STOKES_OK;
    }
    double prev = INFINITY;
    stokes_status status = STOKES_NOT_CONVERGED;
    bool first = true;
    touch_krylov(c, 1, 0);
    for (;;) {
        double *v0 = c.vec(c.V, 0);
        double be2;
        if (first && zero_guess) {
            // x0 = 0: the residual is b itself
            stream_copy(c.bk, v0, c.vlen, c.stream);
            be2 = bn2;
        } else {
            apply_fine<DIM>(c, c.xk, c.bk, v0);
            multidot(c, v0, 1, v0, w2, dh);
            sync_read(c, dh, &be2, 1);
        }
        first = false;
        if (!std::isfinite(be2)) { c.err = "non-finite residual"; return STOKES_ENAN; }
        const double beta = std::sqrt(be2);
        st.rel_res_true = beta / bnorm;
        if (beta <= tol * bnorm) { status = STOKES_OK; break; }
        if (st.iters >= c.opt.max_iters) { status = STOKES_NOT_CONVERGED; break; }
        if (beta >= 0.999 * prev) { status = STOKES_NOT_CONVERGED; break; }   // stagnation across a restart
        prev = beta;
        if (st.iters > 0) st.restarts++;
        set_scale(0, 1.0 / beta);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int nj = 0;
        bool breakdown = false;
        for (int j = 0; j < m && st.iters < c.opt.max_iters; ++j) {
            touch_krylov(c, j + 2, j + 1);
            double *vj = c.vec(c.V, j), *zj = c.vec(c.Z, j), *w = c.vec(c.V, j + 1);
            if (!c.diag_vel && hs[j] != 1.0) {
                // the multigrid velocity path reads v_j in many kernels: normalise it
                k_scale<<<nblocks_stream(c.vlen), kBlock, 0, c.stream>>>(c.vlen, hs[j], vj);
                set_scale(j, 1.0);
            }
            c.cyc_now = j == 0 ? c.cyc_first : c.cyc_next;
            precond<DIM, R>(c, mg, vj, hs[j], zj);
            apply_fine<DIM>(c, zj, nullptr, w);
            // classical Gram-Schmidt: one pass (orth 1) or two (orth 2); the last
            // update pass also reduces the norm of the new vector
            multidot(c, c.V, j + 1, w, w2, dh, c.vs);
            if (c.opt.orth >= 2) {
                maxpy(c, -1.0, c.V, j + 1, dh, w, 1.0, nullptr, c.vs);
                multidot(c, c.V, j + 1, w, w2, dh2, c.vs);
                maxpy(c, -1.0, c.V, j + 1, dh2, w, w2, dh2 + (j + 1), c.vs);
            } else {
                maxpy(c, -1.0, c.V, j + 1, dh, w, w2, dh2 + (j + 1), c.vs);
            }
            HIPCHK(hipMemcpyAsync(hbuf.data(), dh, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, c.stream));
            HIPCHK(hipMemcpyAsync(hbuf.data() + (m + 2), dh2, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, c.stream));
            HIPCHK(hipStreamSynchronize(c.stream));
            for (int i = 0; i <= j; ++i) HH(i, j) = hbuf[i] + (c.opt.orth >= 2 ? hbuf[m + 2 + i] : 0.0);
            double hn2 = hbuf[m + 2 + j + 1];
            if (!std::isfinite(hn2)) { c.err = "non-finite Arnoldi vector"; return STOKES_ENAN; }
            double hn = std::sqrt(std::max(hn2, 0.0));
            HH(j + 1, j) = hn;
            if (hn > 0.0) set_scale(j + 1, 1.0 / hn);
            for (int i = 0; i < j; ++i) {
                double t = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                HH(i + 1, j) = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
                HH(i, j) = t;
            }
            double a = HH(j, j), bb = HH(j + 1, j);
            double den = std::hypot(a, bb);
            cs[j] = den > 0.0 ? a / den : 1.0;
            sn[j] = den > 0.0 ? bb / den : 0.0;
            HH(j, j) = den;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            st.iters++;
            nj = j + 1;
            const double prev_est = j == 0 ? 1.0 : st.rel_res_est;
            st.rel_res_est = std::fabs(g[j + 1]) / bnorm;
            if (c.net && c.learned_active && st.rel_res_est > c.stall_ratio * prev_est) {
                // the learned guess stopped helping: plain multigrid from here on
                c.learned_active = false;
                st.fell_back = 1;
            }
            if (std::fabs(g[j + 1]) <= tol * bnorm) break;
            if (hn == 0.0) { breakdown = true; break; }
        }
        for (int i = nj - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < nj; ++k) s -= HH(i, k) * y[k];
            y[i] = HH(i, i) != 0.0 ? s / HH(i, i) : 0.0;
        }
        HIPCHK(hipMemcpyAsync(dy, y.data(), sizeof(double) * nj, hipMemcpyHostToDevice, c.stream));
        maxpy(c, 1.0, c.Z, nj, dy, c.xk);
        // zero-mean pressure before the true residual is formed, so that the
        // residual left in V[0] on return belongs to the returned iterate (with an
        // open top the pressure is fixed by its zero value there)
        if (!c.fine.open_top) remove_p_mean(c, c.xk);
        if (breakdown) {
            apply_fine<DIM>(c, c.xk, c.bk, v0);
            multidot(c, v0, 1, v0, w2, dh);
            sync_read(c, dh, &be2, 1);
            st.rel_res_true = std::sqrt(be2) / bnorm;
            status = st.rel_res_true <= tol ? STOKES_OK : STOKES_BREAKDOWN;
            break;
        }
    }
    return status;
}

// ---------------------------------------------------------------- setup helpers
// Dense inverse of the coarsest pressure operator -D beta G: the pseudo-inverse
// of the singular all-walls (Neumann) operator, or the inverse with the open top.
template <class R>
void build_dense(stokes_ctx &c, MG<R> &mg) {
    Level<R> &L = mg.L[mg.nlev - 1];
    const Box &b = L.b;
    const int n = mg.ndense, d = b.dim;
    std::vector<R> bt[3];
    for (int a = 0; a < d; ++a) {
        bt[a].resize(b.nb);
        HIPCHK(hipMemcpyAsync(bt[a].data(), L.beta[a], sizeof(R) * b.nb, hipMemcpyDeviceToHost, c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    std::vector<int> map(n);
    std::vector<double> A((size_t)n * n, 0.0);
    auto cid = [&](int i, int j, int k) { return i + b.nx * (j + b.ny * k); };
    const double ih2[3] = {b.ihx * b.ihx, b.ihy * b.ihy, b.ihz * b.ihz};
    for (int k = 0; k < b.nz; ++k)
        for (int j = 0; j < b.ny; ++j)
            for (int i = 0; i < b.nx; ++i) {
                int r = cid(i, j, k);
                map[r] = box_index(b, i, j, k);
                int pos[3] = {i, j, k}, ext[3] = {b.nx, b.ny, b.nz};
                for (int a = 0; a < d; ++a) {
                    for (int side = 0; side < 2; ++side) {
                        int nb[3] = {i, j, k};
                        nb[a] += side ? 1 : -1;
                        int f[3] = {i, j, k};
                        if (side) f[a] += 1;
                        if (nb[a] < 0 || nb[a] >= ext[a]) {
                            if (b.per[a]) {
                                // periodic: the neighbour and the face wrap
                                nb[a] = (nb[a] + ext[a]) % ext[a];
                                f[a] %= ext[a];
                            } else {
                                // the open top: zero pressure on the face (its beta carries the
                                // factor 2 of the half-cell distance); walls carry no flux
                                if (b.open_top && side == 1 && a == d - 1)
                                    A[(size_t)r * n + r] += (double)bt[a][box_index(b, f[0], f[1], f[2])] * ih2[a];
                                continue;
                            }
                        }
                        double w = (double)bt[a][box_index(b, f[0], f[1], f[2])] * ih2[a];
                        A[(size_t)r * n + r] += w;
                        A[(size_t)r * n + cid(nb[0], nb[1], nb[2])] -= w;
                    }
                }
                (void)pos;
            }
    // walls everywhere: the operator is singular (constants); with
    // B = L + (s/n) 1 1^T (s the mean diagonal) nonsingular, L^+ = B^{-1} - 1 1^T/(s n).
    // With the open top it is nonsingular and M is its inverse.
    const bool neumann = !b.open_top;
    double sdiag = 0.0;
    for (int r = 0; r < n; ++r) sdiag += A[(size_t)r * n + r];
    sdiag /= n;
    if (neumann)
        for (auto &x : A) x += sdiag / n;
    // Gauss-Jordan inverse with partial pivoting
    std::vector<double> Inv((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) Inv[(size_t)r * n + r] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
        if (piv != col)
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)piv * n + k], A[(size_t)col * n + k]);
                std::swap(Inv[(size_t)piv * n + k], Inv[(size_t)col * n + k]);
            }
        double p = A[(size_t)col * n + col];
        double ip = 1.0 / p;
        for (int k = 0; k < n; ++k) {
            A[(size_t)col * n + k] *= ip;
            Inv[(size_t)col * n + k] *= ip;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = A[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)col * n + k];
                Inv[(size_t)r * n + k] -= f * Inv[(size_t)col * n + k];
            }
        }
    }
    std::vector<R> M((size_t)n * n);
    const double corr = neumann ? 1.0 / (sdiag * n) : 0.0;
    for (size_t t = 0; t < M.size(); ++t) M[t] = (R)(Inv[t] - corr);
    HIPCHK(hipMemcpyAsync(mg.dense, M.data(), sizeof(R) * M.size(), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(mg.dmap, map.data(), sizeof(int) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
}

// Passes of the cycle on level l (relative index l - l0 in the pass list), in
// the order p_vcycle launches them on flat levels.  zg: zero-guess flag of the
// level's first smoothing pass (0 no, 1 yes, 2 the launch's).
template <class R>
void gen_small_ops(const stokes_ctx &c, const MG<R> &mg, int l0, int l, int zg, std::vector<SmallOp> &ops) {
    const int rel = l - l0;
    auto sweeps = [&](int n, int z) {
        for (int s = 0; s < n; ++s)
            for (int colour = 0; colour < 2; ++colour)
                ops.push_back({SOP_GS, rel, colour, (s == 0 && colour == 0) ? z : 0});
    };
    if (l == mg.nlev - 1) {
        if (mg.use_dense) ops.push_back({SOP_DENSE, rel, 0, 0});
        else sweeps(std::max(1, c.opt.coarse_sweeps), zg);
        return;
    }
    // with a zero guess and no pre-smoothing the iterate must read as zero (at
    // the first level the launch leaves it zero by not loading it)
    if (zg == 1 && p_nu_pre(c, l) == 0) ops.push_back({SOP_ZERO, rel, 0, 0});
    sweeps(p_nu_pre(c, l), zg);
    ops.push_back({SOP_RESTRICT, rel, 0, 0});
    gen_small_ops<R>(c, mg, l0, l + 1, 1, ops);
    for (int g = 1; g < gamma_at(c, mg, l); ++g) gen_small_ops<R>(c, mg, l0, l + 1, 0, ops);
    ops.push_back({SOP_PROLONG, rel, 0, 0});
    sweeps(p_nu_post(c, l), 0);
}

// Picks the finest level (below the finest) from which the whole 3D cycle fits
// in the LDS of one workgroup, lays out that LDS and uploads the pass list.
template <class R>
void plan_small(stokes_ctx &c, MG<R> &mg) {
    mg.small_l0 = -1;
    if (c.dim != 3 || !c.opt.p_small || !mg.ops || mg.nlev < 3) return;
    int dev = 0, lds_max = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    size_t budget = std::min<size_t>((size_t)lds_max, 160 * 1024);
    for (int l0 = 1; l0 <= mg.nlev - 2; ++l0) {
        const Box &f = mg.L[l0].b;
        if ((long long)f.nx * f.ny * f.nz > (1LL << 18) || mg.nlev - l0 > kSmallMaxLev) continue;
        SmallMG<R> s{};
        s.nl = mg.nlev - l0;
        size_t off = 0;
        for (int k = 0; k < s.nl; ++k) {
            const Level<R> &L = mg.L[l0 + k];
            const Box &b = L.b;
            const size_t nl = (size_t)b.nb + b.plane;     // one zero plane below the box
            s.b[k] = b;
            s.off_e[k] = (int)(off + b.plane);
            off += nl;
            s.off_r[k] = (int)(off + b.plane);
            off += nl;
            s.stride_b[k] = (int)nl;
            s.off_b[k] = -1;
            if (k >= 1) {
                s.off_b[k] = (int)(off + b.plane);
                off += 3 * nl;
            }
            for (int a = 0; a < 3; ++a) s.gbeta[k][a] = L.beta[a];
        }
        s.ndense = mg.use_dense ? mg.ndense : 0;
        s.dense = mg.dense;
        s.off_rs = (int)off;
        off += s.ndense;
        if (off * sizeof(R) > budget) continue;
        s.off_dense = -1;
        const size_t nd2 = (size_t)s.ndense * s.ndense;
        if (s.ndense > 0 && (off + nd2) * sizeof(R) <= budget) {
            s.off_dense = (int)off;
            off += nd2;
        }
        s.lin = c.opt.p_prolong;
        s.omega = R(c.p_omega);
        s.lds_elems = (int)off;
        std::vector<SmallOp> ops;
        gen_small_ops<R>(c, mg, l0, l0, 2, ops);
        if (ops.size() > (size_t)kSmallMaxOps) continue;
        if (off * sizeof(R) > 64 * 1024 &&
            (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_p_small_cycle<R, false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)(off * sizeof(R))) != hipSuccess ||
             hipFuncSetAttribute(reinterpret_cast<const void *>(&k_p_small_cycle<R, true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)(off * sizeof(R))) != hipSuccess)) {
            // the runtime refuses more than 64 KiB: plan again within that
            (void)hipGetLastError();
            budget = 64 * 1024;
            l0 = 0;
            continue;
        }
        HIPCHK(hipMemcpyAsync(mg.ops, ops.data(), sizeof(SmallOp) * ops.size(), hipMemcpyHostToDevice, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        mg.small = s;
        mg.nops = (int)ops.size();
        mg.small_lds = off * sizeof(R);
        mg.small_l0 = l0;
        return;
    }
}

template <int DIM, class R>
void build_hierarchy(stokes_ctx &c, MG<R> &mg, bool cast_level0) {
    Level<R> &L0 = mg.L[0];
    if (cast_level0) {
        const long long n = c.fine.stride;
        auto cast = [&](const double *src, R *dst) {
            k_cast<double, R><<<nblocks_stream(n), kBlock, 0, c.stream>>>(n, src - c.fine.guard, dst - L0.b.guard);
        };
        for (int a = 0; a < DIM; ++a) {
            cast(c.mass[a], L0.mass[a]);
            cast(c.beta[a], L0.beta[a]);
        }
        cast(c.mu, L0.mu);
        cast(c.mxy, L0.mxy);
        if (DIM == 3) {
            cast(c.mxz, L0.mxz);
            cast(c.myz, L0.myz);
        }
    }
    for (int l = 1; l < mg.nlev; ++l) {
        Level<R> &F = mg.L[l - 1], &C = mg.L[l];
        unsigned gb = nblocks_box(C.b);
        k_coarsen_mu<DIM, R><<<gb, kBlock, 0, c.stream>>>(F.b, C.b, F.mu, C.mu);
        k_edge_mu<DIM, R><<<gb, kBlock, 0, c.stream>>>(C.b, C.mu, C.mxy, C.mxz, C.myz);
        for (int a = 0; a < DIM; ++a) {
            k_face_restrict<DIM, R><<<gb, kBlock, 0, c.stream>>>(F.b, C.b, a, F.mass[a], C.mass[a]);
            k_coarsen_beta<DIM, R><<<gb, kBlock, 0, c.stream>>>(F.b, C.b, a, F.beta[a], C.beta[a]);
        }
    }
    if (mg.use_dense) build_dense<R>(c, mg);
    plan_small<R>(c, mg);
}

__global__ void k_minmax(Box b, const double *__restrict__ m0, const double *__restrict__ m1,
                         const double *__restrict__ m2, const double *__restrict__ mu, double *__restrict__ out) {
    // out: [min mass, max mass, max mu] per block -> out[3*block + .]
    __shared__ double s0[kBlock], s1[kBlock], s2[kBlock];
    double mn = INFINITY, mx = 0.0, mm = 0.0;
    for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < b.nb; idx += gridDim.x * kBlock) {
        int i, j, k;
        decompose(b, idx, i, j, k);
        if (is_ux(b, i, j, k)) { mn = fmin(mn, m0[idx]); mx = fmax(mx, m0[idx]); }
        if (is_vy(b, i, j, k)) { mn = fmin(mn, m1[idx]); mx = fmax(mx, m1[idx]); }
        if (b.dim == 3 && is_wz(b, i, j, k)) { mn = fmin(mn, m2[idx]); mx = fmax(mx, m2[idx]); }
        if (is_cell(b, i, j, k)) mm = fmax(mm, mu[idx]);
    }
    s0[threadIdx.x] = mn; s1[threadIdx.x] = mx; s2[threadIdx.x] = mm;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s0[threadIdx.x] = fmin(s0[threadIdx.x], s0[threadIdx.x + o]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + o]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = s0[0];
        out[3 * blockIdx.x + 1] = s1[0];
        out[3 * blockIdx.x + 2] = s2[0];
    }
}

// Largest ratio (viscous part of a momentum diagonal) / (its mass term rho/dt)
// over the interior faces; per-block maxima in out[block].
template <int DIM>
__global__ void k_visc_ratio(Box b, VelCoef<double> c, double *__restrict__ out) {
    __shared__ double sm[kBlock];
    double mx = 0.0;
    for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < b.nb; idx += gridDim.x * kBlock) {
        int i, j, k;
        decompose(b, idx, i, j, k);
        double off, dg;
        if (is_ux(b, i, j, k)) { row_u<DIM, double>(b, idx, i, j, k, nullptr, nullptr, nullptr, 0, c, off, dg); mx = fmax(mx, dg / c.mass[0][idx] - 1.0); }
        if (is_vy(b, i, j, k)) { row_v<DIM, double>(b, idx, i, j, k, nullptr, nullptr, nullptr, 0, c, off, dg); mx = fmax(mx, dg / c.mass[1][idx] - 1.0); }
        if (DIM == 3 && is_wz(b, i, j, k)) { row_w<double>(b, idx, i, j, k, nullptr, nullptr, nullptr, 0, c, off, dg); mx = fmax(mx, dg / c.mass[2][idx] - 1.0); }
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

stokes_options defaults() {
    stokes_options o;
    o.precision = 0;
    o.visc_scale = 1.0;
    o.cont_scale = 0.0;
    o.restart = 30;
    o.max_iters = 200;
    o.nu1 = 2;
    o.nu2 = 2;
    o.vel_cycles = 1;
    o.p_cycles = 0;
    o.coarse_sweeps = 40;
    o.vel_levels = 0;
    o.vel_sweeps = 1;
    o.p_prolong = 0;
    o.vel_smoother = 1;
    o.orth = 1;
    o.matvec_z = 1;
    o.p_gamma = 2;
    o.p_small = 1;
    o.p_wdepth = 2;
    o.p_cycles_next = 0;
    o.p_nu_second = 0;
    o.open_top = 0;
    o.p_omega = 0.0;
    return o;
}

const char *check_grid_opts(const stokes_grid *g, const stokes_options &o) {
    if (!g) return "grid is NULL";
    if (g->dim != 2 && g->dim != 3) return "grid.dim must be 2 or 3";
    for (int a = 0; a < g->dim; ++a) {
        if (g->n[a] < 2) return "every axis needs at least 2 cells";
        if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a])) return "grid spacings must be positive";
    }
    // box points with the rows as fine_box pads them
    // (in double: a product of three 32-bit extents can exceed 64 bits)
    const long long nx1 = (long long)g->n[0] + 1;
    const long long px = (g->dim == 3 && g->n[0] >= 256) ? ((nx1 + 15) / 16) * 16 : nx1;
    const double pts = (double)px * ((double)g->n[1] + 1) * (g->dim == 3 ? (double)g->n[2] + 1 : 1.0);
    if (pts * (g->dim + 1) > 1073741824.0) return "grid too large for 32-bit vector indexing";
    if (o.precision != 0 && o.precision != 1) return "precision must be 0 (FP64) or 1 (FP32 multigrid)";
    if (!(o.visc_scale >= 0.0) || !std::isfinite(o.visc_scale)) return "visc_scale must be >= 0";
    if (!(o.cont_scale >= 0.0) || !std::isfinite(o.cont_scale)) return "cont_scale must be >= 0";
    if (o.restart < 1 || o.restart > 200) return "restart must be in [1, 200]";
    if (o.max_iters < 1) return "max_iters must be >= 1";
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1) return "nu1, nu2 >= 0 with nu1 + nu2 >= 1";
    if (o.vel_cycles < 0 || o.p_cycles < 0 || o.p_cycles_next < 0) return "vel_cycles, p_cycles and p_cycles_next must be >= 0";
    if (o.coarse_sweeps < 1) return "coarse_sweeps must be >= 1";
    if (o.vel_levels < 0) return "vel_levels must be >= 0";
    if (o.vel_sweeps < 1) return "vel_sweeps must be >= 1";
    if (o.p_prolong != 0 && o.p_prolong != 1) return "p_prolong must be 0 or 1";
    if (o.vel_smoother != 0 && o.vel_smoother != 1) return "vel_smoother must be 0 or 1";
    if (o.orth != 1 && o.orth != 2) return "orth must be 1 or 2";
    if (o.matvec_z != 0 && o.matvec_z != 1) return "matvec_z must be 0 or 1";
    if (o.p_gamma != 1 && o.p_gamma != 2) return "p_gamma must be 1 (V-cycle) or 2 (W-cycle)";
    if (o.p_small != 0 && o.p_small != 1) return "p_small must be 0 or 1";
    if (o.p_nu_second < 0) return "p_nu_second must be >= 0";
    if (o.p_wdepth < 0) return "p_wdepth must be >= 0";
    if (o.open_top != 0 && o.open_top != 1) return "open_top must be 0 or 1";
    if (!(o.p_omega == 0.0 || (o.p_omega > 0.0 && o.p_omega < 2.0))) return "p_omega must be 0 (automatic) or in (0, 2)";
    for (int a = 0; a < g->dim; ++a) {
        if (g->periodic[a] != 0 && g->periodic[a] != 1) return "periodic[a] must be 0 or 1";
        // red-black colouring stays a colouring across the wrap only for even counts
        if (g->periodic[a] && g->n[a] % 2 != 0) return "a periodic axis needs an even number of cells";
    }
    if (o.open_top && g->periodic[g->dim - 1]) return "open_top needs walls, not a periodic vertical axis";
    return nullptr;
}

// The finest level's box.  Large 3D grids (at least 256 cells along x) get rows
// padded to 16 points: a 64-point tile row is then four whole 128-byte lines, and
// the finest fused sweep runs 5% faster (the extra slots cost the contiguous
// Krylov vector kernels 6% more bytes at 256 cells).
Box fine_box(const stokes_grid *g) {
    Box b = make_box(g->dim, g->n[0], g->n[1], g->dim == 3 ? g->n[2] : 1, g->h[0], g->h[1],
                     g->dim == 3 ? g->h[2] : g->h[0]);
    if (g->dim == 3 && g->n[0] >= 256) pad_rows(b, 16);
    return b;
}

void init_ctx_shape(stokes_ctx &c, const stokes_grid *g, const stokes_options &o) {
    c.grid = *g;
    c.opt = o;
    c.dim = g->dim;
    c.nf = g->dim + 1;
    c.m = o.restart;
    c.theta = o.visc_scale;
    // automatic smoother relaxation: red-black SOR with omega = 1.1 on 3D grids
    // (the same or fewer FGMRES iterations than Gauss-Seidel on every 3D workload
    // measured, FP64 and FP32 multigrid), plain Gauss-Seidel in 2D (no gain there)
    const bool omega_auto = o.p_omega == 0.0;
    c.p_omega = !omega_auto ? o.p_omega : (g->dim == 3 ? 1.1 : 1.0);
    // automatic pressure-cycle schedule: in 3D FP64 a lighter first application
    // and stronger later ones reach the tolerance in two FGMRES iterations on the
    // density-ratio-1000 workloads (4 + 5 cycles with the automatic relaxation,
    // 4 + 6 with any other); the FP32 cycles cannot, nor do the 2D hierarchies,
    // and those keep three cycles per application
    const bool two_step = o.precision == 0 && g->dim == 3;
    c.cyc_first = o.p_cycles > 0 ? o.p_cycles : (two_step ? 4 : 3);
    c.cyc_next = o.p_cycles_next > 0 ? o.p_cycles_next
                                     : (o.p_cycles > 0 ? o.p_cycles : (two_step ? (omega_auto ? 5 : 6) : 3));
    c.cyc_now = c.cyc_first;
    // smoothing below the finest pressure level: with W-cycles on the two finest
    // levels the second is cycled twice and the third and fourth four times per visit
    // of the finest, and in FP64 one sweep on each side of the second and one
    // pre-smoothing sweep on the third and fourth are enough (same iteration counts,
    // fewer sweeps); FP32 multigrid keeps nu1/nu2
    const bool sec_auto = o.precision == 0 && o.p_gamma == 2;
    c.nu_sec1 = o.p_nu_second > 0 ? o.p_nu_second : (sec_auto ? std::min(o.nu1, 1) : o.nu1);
    c.nu_sec2 = o.p_nu_second > 0 ? o.p_nu_second : (sec_auto ? std::min(o.nu2, 1) : o.nu2);
    c.nu_mid1 = o.p_nu_second == 0 && sec_auto ? std::min(o.nu1, 1) : o.nu1;
    // and with the automatic relaxation one post-smoothing sweep on the small levels
    // (at most 16^3 cells, the single-workgroup cycle's) keeps every iteration count
    c.nu_small2 = o.p_nu_second == 0 && sec_auto && omega_auto ? std::min(o.nu2, 1) : o.nu2;
    c.fine = fine_box(g);
    c.fine.open_top = o.open_top;
    for (int a = 0; a < g->dim; ++a) c.fine.per[a] = g->periodic[a];
    {
        const Box &b = c.fine;
        double nc = (double)b.nx * b.ny * b.nz;
        c.unknowns = nc + (double)(b.nx - 1 + b.per[0]) * b.ny * b.nz + (double)b.nx * (b.ny - 1 + b.per[1]) * b.nz +
                     (g->dim == 3 ? (double)b.nx * b.ny * (b.nz - 1 + b.per[2]) : 0.0) +
                     (o.open_top ? (double)b.nx * (g->dim == 3 ? b.ny : 1) : 0.0);
    }
}

template <int DIM>
stokes_status setup_impl(stokes_ctx &c, const double *const rho[3], const double *mu) {
    const Box &b = c.fine;
    const unsigned gb = nblocks_box(b);
    // everything but the Krylov vectors (cleared on first use, touch_krylov)
    {
        const size_t vb = (size_t)(reinterpret_cast<char *>(c.V) - c.ws);
        const size_t ze = (size_t)(reinterpret_cast<char *>(c.Z + (size_t)c.vlen * c.m) - c.ws);
        HIPCHK(hipMemsetAsync(c.ws, 0, vb, c.stream));
        HIPCHK(hipMemsetAsync(c.ws + ze, 0, c.ws_used - ze, c.stream));
        c.v_clear = c.z_clear = 0;
    }
    for (int a = 0; a < DIM; ++a) {
        k_pack_rho<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, a, 1.0 / c.dt, rho[a], c.mass[a],
                                                                          c.beta[a], c.dflag);
    }
    k_pack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, 0, 0, 1.0, mu, c.mu, c.dflag, 1);
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, c.dflag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (flag) {
        c.err = "rho must be > 0 on interior faces and mu >= 0 on cells (finite)";
        return STOKES_EINVAL;
    }
    k_edge_mu<DIM, double><<<gb, kBlock, 0, c.stream>>>(b, c.mu, c.mxy, c.mxz, c.myz);
    if (c.opt.vel_levels == 0) {
        // automatic velocity hierarchy: smoother only when the operator is mass dominated
        const int nbk = kRedBlocks;
        k_visc_ratio<DIM><<<nbk, kBlock, 0, c.stream>>>(b, fine_coef(c), c.partial);
        std::vector<double> h(nbk);
        HIPCHK(hipMemcpyAsync(h.data(), c.partial, sizeof(double) * nbk, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        c.visc_ratio = *std::max_element(h.begin(), h.end());
        int nl = c.opt.precision == 1 ? c.mgf.nlev : c.mgd.nlev;
        int nv = c.visc_ratio < 1e-2 ? 1 : nl;
        c.mgf.nvlev = c.opt.precision == 1 ? nv : 0;
        c.mgd.nvlev = c.opt.precision == 1 ? 0 : nv;
    }
    if (c.opt.precision == 1) build_hierarchy<DIM, float>(c, c.mgf, true);
    else build_hierarchy<DIM, double>(c, c.mgd, false);
    k_vel_inv_diag<DIM><<<gb, kBlock, 0, c.stream>>>(b, fine_coef(c), c.dinv[0], c.dinv[1], DIM == 3 ? c.dinv[2] : c.dinv[1]);
    {
        int nv = c.opt.precision == 1 ? c.mgf.nvlev : c.mgd.nvlev;
        c.diag_vel = c.opt.vel_smoother == 1 && nv == 1 && c.opt.vel_sweeps == 1 && c.opt.vel_cycles == 1;
    }
    if (c.fine.open_top && !c.diag_vel) {
        c.err = "open_top needs the single-level diagonal velocity step (a mass-dominated operator, "
                "or vel_levels = 1 with the default vel_smoother, vel_sweeps and vel_cycles)";
        return STOKES_EINVAL;
    }
    // continuity weight
    if (c.opt.cont_scale > 0.0) {
        c.sigma = c.opt.cont_scale;
    } else {
        const int nbk = kRedBlocks;        // 3 partials per block: fits c.partial (kRedBlocks * kGroup)
        k_minmax<<<nbk, kBlock, 0, c.stream>>>(b, c.mass[0], c.mass[1], DIM == 3 ? c.mass[2] : c.mass[1], c.mu, c.partial);
        std::vector<double> h(3 * nbk);
        HIPCHK(hipMemcpyAsync(h.data(), c.partial, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        double mn = INFINITY, mx = 0.0, mm = 0.0;
        for (int t = 0; t < nbk; ++t) {
            mn = std::min(mn, h[3 * t]);
            mx = std::max(mx, h[3 * t + 1]);
            mm = std::max(mm, h[3 * t + 2]);
        }
        double l = std::max(b.nx * b.hx, b.ny * b.hy);
        if (DIM == 3) l = std::max(l, b.nz * b.hz);
        const double k = M_PI / l;
        const double aref = std::sqrt(mn * mx) + c.theta * mm * k * k;   // mass already holds rho/dt
        c.sigma = aref / k;
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    HIPCHK(hipGetLastError());
    return STOKES_OK;
}

// Packs (u, p) into the box vector vb; with flag, flag[0] is set if a value is
// not finite and flag[1] if one is nonzero (the caller clears both first).
template <int DIM>
void pack_vector(stokes_ctx &c, const double *const u[3], const double *p, double *vb, int *flag = nullptr) {
    const Box &b = c.fine;
    for (int a = 0; a < DIM; ++a)
        k_pack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, a, 0, 0, 1.0, u[a], c.fld(vb, a), flag, 0);
    k_pack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, 0, 0, 1.0, p, c.fld(vb, DIM), flag, 0);
}

template <int DIM>
void unpack_vector(stokes_ctx &c, double *vb, double *const u[3], double *p) {
    const Box &b = c.fine;
    for (int a = 0; a < DIM; ++a) k_unpack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, a, c.fld(vb, a), u[a]);
    k_unpack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, c.fld(vb, DIM), p);
}

template <int DIM>
stokes_status solve_impl(stokes_ctx &c, const double *const rhs_u[3], const double *rhs_p, double tol,
                         double *const x_u[3], double *x_p, stokes_stats &st) {
    c.vcycles = 0;
    c.learned_active = c.net != nullptr;
    // dflag[0..1]: right-hand side not finite / nonzero; dflag[2..3]: the same for x
    k_fill<int><<<1, kBlock, 0, c.stream>>>(4, c.dflag, 0);
    pack_vector<DIM>(c, rhs_u, rhs_p, c.bk, c.dflag);
    int flag = 0;
    // mean of rhs_p
    {
        double *p = c.fld(c.bk, DIM) - c.fine.guard;
        const unsigned g = nblocks_stream(c.fine.stride);
        k_partial_sum<<<g, kBlock, 0, c.stream>>>(c.fine.stride, p, 0, c.partial);
        k_reduce_partials<<<1, kBlock, 0, c.stream>>>((int)g, c.partial, c.dsc, 0, nullptr);
        double s;
        HIPCHK(hipMemcpyAsync(&flag, c.dflag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        sync_read(c, c.dsc, &s, 1);
        if (flag) { c.err = "non-finite right-hand side"; return STOKES_ENAN; }
        if (!c.fine.open_top) {            // walls everywhere: the mean of rhs_p is incompatible
            st.g_mean = s / ((double)c.fine.nx * c.fine.ny * c.fine.nz);
            k_sub_mean<<<nblocks_box(c.fine), kBlock, 0, c.stream>>>(c.fine, c.dsc, c.fld(c.bk, DIM));
        }
    }
    pack_vector<DIM>(c, x_u, x_p, c.xk, c.dflag + 2);
    int xflag[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(xflag, c.dflag + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (xflag[0]) { c.err = "non-finite initial guess"; return STOKES_ENAN; }
    const bool zero_guess = xflag[1] == 0;
    if (!zero_guess && !c.fine.open_top) remove_p_mean(c, c.xk);   // an all-zero guess has zero mean
    stokes_status s = c.opt.precision == 1 ? fgmres<DIM, float>(c, c.mgf, tol, zero_guess, st)
                                           : fgmres<DIM, double>(c, c.mgd, tol, zero_guess, st);
    if (s < 0) return s;
    // final residual split into its blocks (plain 2-norm); fgmres leaves the
    // residual b - K x of the returned (zero-mean pressure) iterate in V[0]
    double *v0 = c.vec(c.V, 0);
    {
        const long long nvel = (long long)DIM * c.fine.stride;
        const unsigned g1 = nblocks_stream(nvel), g2 = nblocks_stream(c.fine.stride), g3 = nblocks_stream(c.vlen);
        k_partial_sum<<<g1, kBlock, 0, c.stream>>>(nvel, v0, 1, c.partial);
        k_reduce_partials<<<1, kBlock, 0, c.stream>>>((int)g1, c.partial, c.dsc, 0, nullptr);
        k_partial_sum<<<g2, kBlock, 0, c.stream>>>(c.fine.stride, c.fld(v0, DIM) - c.fine.guard, 1, c.partial);
        k_reduce_partials<<<1, kBlock, 0, c.stream>>>((int)g2, c.partial, c.dsc + 1, 0, nullptr);
        k_partial_sum<<<g3, kBlock, 0, c.stream>>>(c.vlen, c.bk, 1, c.partial);
        k_reduce_partials<<<1, kBlock, 0, c.stream>>>((int)g3, c.partial, c.dsc + 2, 0, nullptr);
        double h3[3];
        sync_read(c, c.dsc, h3, 3);
        double bn = std::sqrt(h3[2]);
        if (bn > 0) {
            st.rel_res_mom = std::sqrt(h3[0]) / bn;
            st.rel_res_cont = std::sqrt(h3[1]) / bn;
            st.rel_res_plain = std::sqrt(h3[0] + h3[1]) / bn;
        }
    }
    unpack_vector<DIM>(c, c.xk, x_u, x_p);
    HIPCHK(hipStreamSynchronize(c.stream));
    HIPCHK(hipGetLastError());
    prof_collect(c);
    return s;
}

}  // namespace

namespace {

template <class R>
int learned_level(const MG<R> &mg, int n) {
    for (int l = 0; l < mg.nlev; ++l) {
        const Box &b = mg.L[l].b;
        if (b.dim == 3 && b.nx == n && b.ny == n && b.nz == n && (long long)n * n * n <= kLearnedMaxCells) return l;
    }
    return -1;
}

template <class R>
void learned_static(stokes_ctx &c, MG<R> &mg, int lc, float *f0, float *f1) {
    Level<R> &C = mg.L[lc];
    const int nc = C.b.nx * C.b.ny * C.b.nz;
    k_learned_static<R><<<(nc + kBlock - 1) / kBlock, kBlock, 0, c.stream>>>(C.b, C.beta[0], C.beta[1], C.beta[2], C.mu, f0, f1);
}

// Training tuple on the level with n^3 cells: static features, the restricted
// pressure right-hand side of the first preconditioner application (unit RMS)
// and the restricted converged pressure solution (zero mean, unit RMS).
template <class R>
void first_p3_rhs(stokes_ctx &c, MG<R> &mg) {
    const Box &fb = c.fine;
    Level<R> &L0 = mg.L[0];
    double *v = c.bk;
    // steps 1-2 of the preconditioner on v = b: u~ and the Poisson right-hand side
    if (c.diag_vel) {
        k_precond_div_jac<3, R><<<nblocks_box(fb), kBlock, 0, c.stream>>>(
            fb, c.fld(v, 0), c.fld(v, 1), c.fld(v, 2), c.dinv[0], c.dinv[1], c.dinv[2], c.fld(v, 3), 1.0, c.dt, c.q,
            L0.rp);
    } else {
        touch_krylov(c, 0, 1);
        double *z = c.vec(c.Z, 0);
        R *eu[3], *ru[3];
        if (sizeof(R) == sizeof(double)) {
            for (int a = 0; a < 3; ++a) {
                eu[a] = reinterpret_cast<R *>(c.fld(z, a));
                ru[a] = reinterpret_cast<R *>(c.fld(v, a));
            }
        } else {
            long long n = 3LL * fb.stride;
            k_cast<double, R><<<nblocks_stream(n), kBlock, 0, c.stream>>>(n, v, L0.ru[0] - L0.b.guard);
            for (int a = 0; a < 3; ++a) {
                eu[a] = L0.eu[a];
                ru[a] = L0.ru[a];
            }
        }
        for (int cyc = 0; cyc < std::max(1, c.opt.vel_cycles); ++cyc) vel_vcycle<3, R>(c, mg, 0, eu, ru, cyc == 0);
        k_precond_div<3, R><<<nblocks_box(fb), kBlock, 0, c.stream>>>(fb, eu[0], eu[1], eu[2], c.fld(v, 3), c.dt, c.q, L0.rp);
    }
}

// Training tuple on the level with n^3 cells: static features, the restricted
// pressure right-hand side of the first preconditioner application (unit RMS)
// and the restricted converged pressure solution (zero mean, unit RMS).
template <class R>
void learned_tuple(stokes_ctx &c, MG<R> &mg, int lc, int cycles, float *f0, float *f1, float *s_c, float *phi_c) {
    Level<R> &L0 = mg.L[0];
    first_p3_rhs<R>(c, mg);
    R *phi = L0.ep;
    for (int cyc = 0; cyc < cycles; ++cyc) phi = p_vcycle<3, R>(c, mg, 0, phi, L0.rp, cyc == 0);
    const R *ss = L0.rp;
    const R *pp = phi;
    for (int l = 0; l < lc; ++l) {
        Level<R> &F = mg.L[l], &C = mg.L[l + 1];
        k_restrict_avg3<R><<<nblocks_box(C.b), kBlock, 0, c.stream>>>(F.b, C.b, ss, C.rp);
        k_restrict_avg3<R><<<nblocks_box(C.b), kBlock, 0, c.stream>>>(F.b, C.b, pp, C.ep);
        ss = C.rp;
        pp = C.ep;
    }
    Level<R> &C = mg.L[lc];
    k_normalise_planar<R><<<1, 1024, 0, c.stream>>>(C.b, ss, 0, s_c, c.lstat);
    k_normalise_planar<R><<<1, 1024, 0, c.stream>>>(C.b, pp, 1, phi_c, c.lstat + 3);
    learned_static<R>(c, mg, lc, f0, f1);
}

// What an initial guess is worth to the pressure cycles of the first
// preconditioner application (a measurement; the solve never calls it).  The
// reference solution phi* of that subsolve is ref_cycles cycles from zero.
// Row 0 starts from zero, row 1 from the attached network's guess, row 1 + l
// (l = 1 .. kStudyRows - 2) from the ideal guess a perfect predictor on level l
// could give: phi* averaged down to level l, then the same amplitude fit and
// trilinear prolongation the network's output takes.  out[row][k] = relative
// residual ||s - (-L_rho) phi_k|| / ||s|| after k = 0 .. max_cycles cycles;
// NaN for a row with no network or no such level.
constexpr int kStudyRows = STOKES_STUDY_ROWS;

template <class R>
double p_rel_residual(stokes_ctx &c, MG<R> &mg, const R *e) {
    Level<R> &L0 = mg.L[0];
    const int g = kRedBlocks;
    k_p_res_partial<R><<<g, kBlock, 0, c.stream>>>(L0.b, e, L0.rp, L0.beta[0], L0.beta[1], L0.beta[2], c.partial);
    k_reduce_partials<<<2, kBlock, 0, c.stream>>>(g, c.partial, c.dsc, 0, nullptr);
    double h[2];
    sync_read(c, c.dsc, h, 2);
    return h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
}

template <class R>
void learned_study(stokes_ctx &c, MG<R> &mg, int ref_cycles, int max_cycles, double *out) {
    Level<R> &L0 = mg.L[0];
    const int nk = max_cycles + 1;
    first_p3_rhs<R>(c, mg);
    // phi* into the first Krylov Z vector (scratch here; re-cleared before the next solve)
    R *star = reinterpret_cast<R *>(c.vec(c.Z, 0)) + L0.b.guard;
    R *phi = L0.ep;
    for (int k = 0; k < ref_cycles; ++k) phi = p_vcycle<3, R>(c, mg, 0, phi, L0.rp, k == 0);
    k_cast<R, R><<<nblocks_stream(L0.b.stride), kBlock, 0, c.stream>>>(L0.b.stride, phi - L0.b.guard, star - L0.b.guard);
    for (int row = 0; row < kStudyRows; ++row) {
        const int l = row - 1;
        const bool have = row == 0 || (row == 1 && c.net && c.lc >= 0) || (row >= 2 && l < mg.nlev);
        if (!have) {
            for (int k = 0; k < nk; ++k) out[row * nk + k] = std::nan("");
            continue;
        }
        bool zero = row == 0;
        if (zero) {
            fill<R>(c, L0.ep - L0.b.guard, L0.b.stride, R(0));
        } else if (row == 1) {
            learned_guess<R>(c, mg, L0.ep);
        } else {
            const R *src = star;
            for (int m = 0; m < l; ++m) {
                k_restrict_avg3<R><<<nblocks_box(mg.L[m + 1].b), kBlock, 0, c.stream>>>(mg.L[m].b, mg.L[m + 1].b, src,
                                                                                       mg.L[m + 1].ep);
                src = mg.L[m + 1].ep;
            }
            Level<R> &C = mg.L[l];
            k_cast<R, R><<<nblocks_stream(C.b.stride), kBlock, 0, c.stream>>>(C.b.stride, C.ep - C.b.guard, C.ep2 - C.b.guard);
            restrict_rhs_to<R>(c, mg, l);
            guess_from_coarse<R>(c, mg, l, L0.ep);
        }
        phi = L0.ep;
        out[row * nk] = p_rel_residual<R>(c, mg, phi);
        for (int k = 1; k < nk; ++k) {
            phi = p_vcycle<3, R>(c, mg, 0, phi, L0.rp, zero && k == 1);
            out[row * nk + k] = p_rel_residual<R>(c, mg, phi);
        }
    }
    c.z_clear = 0;
}

// Right-hand-side lift of Dirichlet inflow data on the x = 0 side: the rows next
// to that wall move the known boundary values to the right (see
// stokes_inflow_lift).  One thread per (j, k) of the wall plane; caller layouts
// for the right-hand side, box layout for the viscosities.
__global__ void __launch_bounds__(kBlock) k_inflow_lift(Box b, const double *__restrict__ mu,
        const double *__restrict__ mxy, const double *__restrict__ mxz, double theta,
        const double *__restrict__ un, const double *__restrict__ ut,
        double *__restrict__ fu, double *__restrict__ fv, double *__restrict__ fw, double *__restrict__ fp) {
    const int ny = b.ny, nz = b.nz, nx = b.nx;
    const int vert = b.dim - 1;                             // 1 in 2D, 2 in 3D
    const int nvert = vert == 1 ? ny : nz;
    // thread over (j, k) in [0, ny] x [0, nz] (2D: k = 0 only): cell rows and node rows
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int pj = ny + 1, pk = b.dim == 3 ? nz + 1 : 1;
    if (t >= pj * pk) return;
    const int j = t % pj, k = t / pj;
    const double ihx = b.ihx, ihy = b.ihy, ihz = b.ihz;
    const bool cell = j < ny && k < (b.dim == 3 ? nz : 1);
    // un is (Nz, Ny) (2D: Ny); ut (Nz+1, Ny) (2D: Ny+1)
    auto UN = [&](int jj, int kk) { return un[jj + ny * kk]; };
    if (cell) {
        const double u0 = UN(j, k);
        fp[nx * (j + ny * k)] -= u0 * ihx;                                  // continuity of cell (0, j, k)
        fu[1 + (nx + 1) * (j + ny * k)] += theta * 2.0 * mu[box_index(b, 0, j, k)] * u0 * ihx * ihx;
    }
    // vertical component on the faces (0, .) next to the wall: its wall edge's shear
    // stress has the known parts -2 u_t / h_x and d u_n / d(vertical)
    const int iv = vert == 1 ? j : k;                        // face index along the vertical
    const bool vfaces = vert == 1 ? (k == 0 && j >= 1 && (j < ny || (b.open_top && j == ny)))
                                  : (j < ny && k >= 1 && (k < nz || (b.open_top && k == nz)));
    if (vfaces) {
        double dun;
        if (iv < nvert) {
            dun = vert == 1 ? (UN(j, 0) - UN(j - 1, 0)) * ihy : (UN(j, k) - UN(j, k - 1)) * ihz;
        } else {                                            // open top: u above = -u below
            dun = vert == 1 ? -2.0 * UN(j - 1, 0) * ihy : -2.0 * UN(j, k - 1) * ihz;
        }
        const double utv = vert == 1 ? ut[j] : ut[j + ny * k];
        const double me = vert == 1 ? mxy[box_index(b, 0, j, 0)] : mxz[box_index(b, 0, j, k)];
        const double tau = me * (-2.0 * utv * ihx + dun);
        if (vert == 1) fv[nx * (j + (ny + 1) * k)] -= theta * tau * ihx;
        else fw[nx * (j + ny * k)] -= theta * tau * ihx;
    }
    // 3D lateral component v on the faces (0, j, k), 1 <= j < ny: d u_n / d y on the wall edge
    if (b.dim == 3 && k < nz && j >= 1 && j < ny) {
        const double tau = mxy[box_index(b, 0, j, k)] * (UN(j, k) - UN(j - 1, k)) * ihy;
        fv[nx * (j + (ny + 1) * k)] -= theta * tau * ihx;
    }
}

// One pressure-multigrid kernel of the finest level on caller data (the test
// hook stokes_pressure_op): the caller's cell arrays are packed into the level's
// arrays (through an FP64 staging field and a cast with FP32 multigrid), the
// kernel runs as the cycle launches it (or in its flat form), and the result is
// unpacked into the caller's cell layout.
template <int DIM, class R>
void pressure_op(stokes_ctx &c, MG<R> &mg, int op, const double *e_in, const double *r_in, const double *ec_in,
                 double *out) {
    Level<R> &L = mg.L[0];
    double *stage = c.q - c.fine.guard;     // one FP64 field of the fine box, guards included
    auto load = [&](const Box &b, const double *src, R *dst) {
        if constexpr (sizeof(R) == sizeof(double)) {
            k_pack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, 0, 0, 1.0, src,
                                                                          reinterpret_cast<double *>(dst), nullptr, 0);
        } else {
            fill<double>(c, stage, b.stride, 0.0);
            k_pack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, 0, 0, 1.0, src, stage + b.guard,
                                                                          nullptr, 0);
            k_cast<double, R><<<nblocks_stream(b.stride), kBlock, 0, c.stream>>>(b.stride, stage, dst - b.guard);
        }
    };
    auto store = [&](const Box &b, const R *src, double *dst) {
        if constexpr (sizeof(R) == sizeof(double)) {
            k_unpack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, reinterpret_cast<const double *>(src), dst);
        } else {
            k_cast<R, double><<<nblocks_stream(b.stride), kBlock, 0, c.stream>>>(b.stride, src - b.guard, stage);
            k_unpack<<<nblocks_rows(b), dim3(64, kPackRows), 0, c.stream>>>(b, 3, stage + b.guard, dst);
        }
    };
    const bool flat = op == STOKES_POP_SWEEP_FLAT || op == STOKES_POP_RESTRICT_FLAT;
    load(L.b, r_in, L.rp);
    if (e_in) load(L.b, e_in, L.ep);
    if (op == STOKES_POP_SWEEP || op == STOKES_POP_SWEEP_FLAT) {
        const R *ec = nullptr;
        const Box *cb = nullptr;
        if (ec_in) {
            Level<R> &C = mg.L[1];
            load(C.b, ec_in, C.ep);
            ec = C.ep;
            cb = &C.b;
        }
        R *cur = L.ep, *spare = L.ep2;
        p_level_sweep<DIM, R>(c, L, cur, spare, L.rp, e_in == nullptr, ec, cb, flat);
        store(L.b, cur, out);
    } else {
        Level<R> &C = mg.L[1];
        p_residual_restrict<DIM, R>(c, L, C, L.ep, L.rp, C.rp, flat);
        store(C.b, C.rp, out);
    }
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

void stokes_default_options(stokes_options *opts) {
    if (opts) *opts = defaults();
}

size_t stokes_workspace_size(const stokes_grid *grid, const stokes_options *opts) {
    stokes_options o = opts ? *opts : defaults();
    if (check_grid_opts(grid, o)) return 0;
    stokes_ctx c;
    init_ctx_shape(c, grid, o);
    Carver cv{nullptr};
    carve_all(cv, c);
    return c.ws_need;
}

stokes_status stokes_setup(const double *const rho_face[3], const double *mu_cell, double dt,
                           const stokes_grid *grid, const stokes_options *opts, void *workspace,
                           size_t ws_bytes, void *stream, stokes_ctx **out) {
    g_setup_error.clear();
    if (!out) { g_setup_error = "out is NULL"; return STOKES_EINVAL; }
    *out = nullptr;
    stokes_options o = opts ? *opts : defaults();
    if (const char *msg = check_grid_opts(grid, o)) {
        g_setup_error = msg;
        return (grid && (grid->dim == 2 || grid->dim == 3)) && (std::strstr(msg, "cells") || std::strstr(msg, "too large"))
                   ? STOKES_ESHAPE : STOKES_EINVAL;
    }
    if (!(dt > 0.0) || !std::isfinite(dt)) { g_setup_error = "dt must be > 0"; return STOKES_EINVAL; }
    if (!rho_face || !rho_face[0] || !rho_face[1] || (grid->dim == 3 && !rho_face[2]) || !mu_cell) {
        g_setup_error = "coefficient pointer is NULL";
        return STOKES_EINVAL;
    }
    if (!workspace) { g_setup_error = "workspace is NULL"; return STOKES_EINVAL; }
    stokes_ctx *c = new stokes_ctx();
    init_ctx_shape(*c, grid, o);
    c->dt = dt;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    {
        Carver dry{nullptr};
        carve_all(dry, *c);
    }
    if (ws_bytes < c->ws_need) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "workspace too small: %zu bytes given, %zu needed", ws_bytes, c->ws_need);
        g_setup_error = buf;
        delete c;
        return STOKES_ENOMEM;
    }
    // carve from the first 256-byte boundary (the 16-byte vector accesses of the
    // BLAS kernels need aligned vectors; ws_need holds the slack)
    const size_t shift = (size_t)(-reinterpret_cast<uintptr_t>(workspace) & 255);
    c->ws = reinterpret_cast<char *>(workspace) + shift;
    c->ws_bytes = ws_bytes - shift;
    Carver cv{c->ws};
    carve_all(cv, *c);
    stokes_status s;
    try {
        s = c->dim == 3 ? setup_impl<3>(*c, rho_face, mu_cell) : setup_impl<2>(*c, rho_face, mu_cell);
    } catch (const HipError &e) {
        g_setup_error = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        delete c;
        return STOKES_EHIP;
    }
    if (s != STOKES_OK) {
        g_setup_error = c->err;
        delete c;
        return s;
    }
    *out = c;
    return STOKES_OK;
}

stokes_status stokes_apply(stokes_ctx *ctx, const double *const x_u[3], const double *x_p,
                           double *const y_u[3], double *y_p) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    const int d = ctx->dim;
    if (!x_u || !y_u || !x_p || !y_p || !x_u[0] || !x_u[1] || !y_u[0] || !y_u[1] ||
        (d == 3 && (!x_u[2] || !y_u[2]))) {
        ctx->err = "NULL array pointer";
        return STOKES_EINVAL;
    }
    try {
        touch_krylov(*ctx, 2, 0);
        double *vin = ctx->vec(ctx->V, 0), *vout = ctx->vec(ctx->V, 1 % (ctx->m + 1));
        if (d == 3) {
            pack_vector<3>(*ctx, x_u, x_p, vin);
            apply_fine<3>(*ctx, vin, nullptr, vout);
            unpack_vector<3>(*ctx, vout, y_u, y_p);
        } else {
            pack_vector<2>(*ctx, x_u, x_p, vin);
            apply_fine<2>(*ctx, vin, nullptr, vout);
            unpack_vector<2>(*ctx, vout, y_u, y_p);
        }
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

stokes_status stokes_solve(stokes_ctx *ctx, const double *const rhs_u[3], const double *rhs_p, double tol,
                           double *const x_u[3], double *x_p, stokes_stats *stats) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    const int d = ctx->dim;
    if (!rhs_u || !x_u || !rhs_p || !x_p || !rhs_u[0] || !rhs_u[1] || !x_u[0] || !x_u[1] ||
        (d == 3 && (!rhs_u[2] || !x_u[2]))) {
        ctx->err = "NULL array pointer";
        return STOKES_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        ctx->err = "tol must be > 0";
        return STOKES_EINVAL;
    }
    stokes_stats st;
    std::memset(&st, 0, sizeof st);
    auto t0 = std::chrono::steady_clock::now();
    stokes_status s;
    try {
        s = d == 3 ? solve_impl<3>(*ctx, rhs_u, rhs_p, tol, x_u, x_p, st)
                   : solve_impl<2>(*ctx, rhs_u, rhs_p, tol, x_u, x_p, st);
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        s = STOKES_EHIP;
    }
    auto t1 = std::chrono::steady_clock::now();
    st.ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    st.vcycles = ctx->vcycles;
    st.levels = ctx->opt.precision == 1 ? ctx->mgf.nlev : ctx->mgd.nlev;
    st.small_level = ctx->opt.precision == 1 ? ctx->mgf.small_l0 : ctx->mgd.small_l0;
    st.sigma = ctx->sigma;
    if (stats) *stats = st;
    return s;
}

stokes_status stokes_profile_kernel(stokes_ctx *ctx, int kernel) {
    if (!ctx) return STOKES_EINVAL;
    if (kernel < -1 || kernel > STOKES_PROF_MAXPY) {
        ctx->err = "unknown kernel class";
        return STOKES_EINVAL;
    }
    try {
        if (kernel >= 0 && ctx->ev.empty()) {
            ctx->ev.resize(8192);
            for (auto &e : ctx->ev) HIPCHK(hipEventCreate(&e));
        }
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return STOKES_EHIP;
    }
    ctx->prof_kind = kernel;
    ctx->ev_used = 0;
    ctx->prof_ms = ctx->prof_bytes = 0.0;
    ctx->prof_launches = 0;
    return STOKES_OK;
}

stokes_status stokes_profile_read(stokes_ctx *ctx, double *ms_total, long long *launches, double *bytes) {
    if (!ctx) return STOKES_EINVAL;
    if (ms_total) *ms_total = ctx->prof_ms;
    if (launches) *launches = ctx->prof_launches;
    if (bytes) *bytes = ctx->prof_bytes;
    ctx->prof_ms = ctx->prof_bytes = 0.0;
    ctx->prof_launches = 0;
    return STOKES_OK;
}

stokes_status stokes_stream_copy(const double *src, double *dst, long long n, void *stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) return STOKES_EINVAL;
    if (n == 0) return STOKES_OK;
    stream_copy(src, dst, n, reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}

stokes_status stokes_attach_learned(stokes_ctx *ctx, stokes_unet *net, double stall_ratio) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    if (!net) {
        ctx->net = nullptr;
        ctx->lc = -1;
        return STOKES_OK;
    }
    if (ctx->dim != 3) { ctx->err = "the learned stage needs a 3D grid"; return STOKES_EINVAL; }
    if (stokes_unet_stream_internal(net) != reinterpret_cast<void *>(ctx->stream)) {
        ctx->err = "network and solver must use the same stream";
        return STOKES_EINVAL;
    }
    const int n = stokes_unet_size(net);
    int lc = ctx->opt.precision == 1 ? learned_level(ctx->mgf, n) : learned_level(ctx->mgd, n);
    if (lc < 0) { ctx->err = "no multigrid level has n^3 cells for this network (n <= 64)"; return STOKES_EINVAL; }
    if (!(stall_ratio >= 0.0)) { ctx->err = "stall_ratio must be >= 0"; return STOKES_EINVAL; }
    try {
        if (ctx->opt.precision == 1) learned_static<float>(*ctx, ctx->mgf, lc, ctx->lf[0], ctx->lf[1]);
        else learned_static<double>(*ctx, ctx->mgd, lc, ctx->lf[0], ctx->lf[1]);
        HIPCHK(hipStreamSynchronize(ctx->stream));
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return STOKES_EHIP;
    }
    ctx->net = net;
    ctx->lc = lc;
    ctx->stall_ratio = stall_ratio;
    return STOKES_OK;
}

stokes_status stokes_learned_tuple(stokes_ctx *ctx, const double *const rhs_u[3], const double *rhs_p, int n,
                                   int cycles, float *f0, float *f1, float *s_c, float *phi_c) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    if (ctx->dim != 3 || !rhs_u || !rhs_u[0] || !rhs_u[1] || !rhs_u[2] || !rhs_p || !f0 || !f1 || !s_c || !phi_c ||
        cycles < 1) {
        ctx->err = "bad argument";
        return STOKES_EINVAL;
    }
    int lc = ctx->opt.precision == 1 ? learned_level(ctx->mgf, n) : learned_level(ctx->mgd, n);
    if (lc < 0) { ctx->err = "no multigrid level has n^3 cells (n <= 64)"; return STOKES_EINVAL; }
    try {
        pack_vector<3>(*ctx, rhs_u, rhs_p, ctx->bk);
        if (ctx->opt.precision == 1) learned_tuple<float>(*ctx, ctx->mgf, lc, cycles, f0, f1, s_c, phi_c);
        else learned_tuple<double>(*ctx, ctx->mgd, lc, cycles, f0, f1, s_c, phi_c);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

stokes_status stokes_learned_study(stokes_ctx *ctx, const double *const rhs_u[3], const double *rhs_p, int ref_cycles,
                                   int max_cycles, double *res) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    if (ctx->dim != 3 || !rhs_u || !rhs_u[0] || !rhs_u[1] || !rhs_u[2] || !rhs_p || !res || ref_cycles < 1 ||
        max_cycles < 0 || max_cycles > 64) {
        ctx->err = "bad argument";
        return STOKES_EINVAL;
    }
    try {
        pack_vector<3>(*ctx, rhs_u, rhs_p, ctx->bk);
        if (ctx->opt.precision == 1) learned_study<float>(*ctx, ctx->mgf, ref_cycles, max_cycles, res);
        else learned_study<double>(*ctx, ctx->mgd, ref_cycles, max_cycles, res);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

stokes_status stokes_inflow_lift(stokes_ctx *ctx, const double *u_n, const double *u_t, double *const rhs_u[3],
                                 double *rhs_p) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    const int d = ctx->dim;
    if (!u_n || !u_t || !rhs_u || !rhs_u[0] || !rhs_u[1] || (d == 3 && !rhs_u[2]) || !rhs_p) {
        ctx->err = "NULL array pointer";
        return STOKES_EINVAL;
    }
    const Box &b = ctx->fine;
    if (b.per[0]) {
        ctx->err = "inflow data needs a wall at x = 0, not a periodic x axis";
        return STOKES_EINVAL;
    }
    const long long pts = (long long)(b.ny + 1) * (d == 3 ? b.nz + 1 : 1);
    k_inflow_lift<<<(unsigned)((pts + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        b, ctx->mu, ctx->mxy, ctx->mxz, ctx->theta, u_n, u_t, rhs_u[0], rhs_u[1], d == 3 ? rhs_u[2] : nullptr, rhs_p);
    if (hipGetLastError() != hipSuccess) {
        ctx->err = "k_inflow_lift launch failed";
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

stokes_status stokes_pressure_op(stokes_ctx *ctx, int op, const double *e_in, const double *r, const double *ec,
                                 double *out) {
    if (!ctx) return STOKES_EINVAL;
    ctx->err.clear();
    if (op < STOKES_POP_SWEEP || op > STOKES_POP_RESTRICT_FLAT) { ctx->err = "unknown op"; return STOKES_EINVAL; }
    const bool restrict_op = op == STOKES_POP_RESTRICT || op == STOKES_POP_RESTRICT_FLAT;
    if (!r || !out || (restrict_op && (!e_in || ec)) || (ec && !e_in)) {
        ctx->err = "bad array pointers for this op";
        return STOKES_EINVAL;
    }
    const int nlev = ctx->opt.precision == 1 ? ctx->mgf.nlev : ctx->mgd.nlev;
    if ((restrict_op || ec) && nlev < 2) { ctx->err = "the grid has no coarser level"; return STOKES_EINVAL; }
    try {
        if (ctx->dim == 3) {
            if (ctx->opt.precision == 1) pressure_op<3, float>(*ctx, ctx->mgf, op, e_in, r, ec, out);
            else pressure_op<3, double>(*ctx, ctx->mgd, op, e_in, r, ec, out);
        } else {
            if (ctx->opt.precision == 1) pressure_op<2, float>(*ctx, ctx->mgf, op, e_in, r, ec, out);
            else pressure_op<2, double>(*ctx, ctx->mgd, op, e_in, r, ec, out);
        }
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

void stokes_destroy(stokes_ctx *ctx) { delete ctx; }

const char *stokes_last_error(const stokes_ctx *ctx) {
    if (!ctx) return g_setup_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"

// Message for stokes_last_error(NULL) from the other source files of the library.
void stk_set_thread_error(const char *msg) { g_setup_error = msg ? msg : ""; }
