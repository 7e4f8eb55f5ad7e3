/*
 * mhlp.hip -- HIP kernels and C ABI of the modified-Helmholtz layer-potential
 * library (declarations and contracts: include/mhlp.h).
 *
 * Data layout in device memory
 *   geometry : node SoA x, y, dx, dy, d2x, d2y (copy of the caller's [6][N]),
 *              derived per-node weight w, unit normal nx, ny, curvature;
 *              per panel the Legendre coefficients of its position (16
 *              complex), arclength h and a bounding circle.
 *   plan     : targets tx, ty; CSR near list by target (row_ptr, panel index
 *              ascending, target index, complex preimage) and 16 SLP + 16 DLP
 *              correction weights per listed (target, panel) pair.
 *
 * Kernels
 *   geom_prep        one thread per panel: weights, normals, curvature, Legendre
 *                    coefficients, arclength, bounding circle.
 *   near_list        one thread per target, run twice (count, then fill): candidate
 *                    panels (some node within 1.2 h), Newton preimage, Bernstein
 *                    radius < 3.5 (Sec. 4.5.1).
 *   near_weights     one thread per listed pair: correction weights (nearfield.h).
 *   far_eval_fp64    one thread per target, sources streamed through LDS in tiles
 *                    of 16 panels; listed panels are skipped and their corrected
 *                    contribution added in the epilogue (no add-then-subtract).
 *   gmres_*          BLAS-1 pieces of the Arnoldi process.
 */
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <map>
#include <mutex>
#include <numeric>

#include "mhlp.h"
#include "nearfield.h"

using namespace mhlp;

/* ------------------------------------------------------------------------ */
/* error handling                                                            */
/* ------------------------------------------------------------------------ */
static thread_local std::string g_err;

static mhlp_status fail(mhlp_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIPCHECK(x)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) return fail(MHLP_HIP_ERROR, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *mhlp_last_error(void) { return g_err.c_str(); }

/* error setter shared with the other translation units of the library */
__attribute__((visibility("hidden"))) mhlp_status mhlp_set_error(mhlp_status s, const char *msg)
{
    g_err = msg;
    return s;
}

/* ------------------------------------------------------------------------ */
/* handles                                                                   */
/* ------------------------------------------------------------------------ */
struct mhlp_geometry {
    int device = 0;
    int64_t N = 0, Np = 0;
    double *soa = nullptr;                       /* [6][N] */
    double *w = nullptr, *nx = nullptr, *ny = nullptr, *kappa = nullptr;
    double *pa = nullptr; /* [Np][16] complex Legendre coefficients of the panel relative to its node 7 */
    double *ph = nullptr, *pcx = nullptr, *pcy = nullptr, *prad = nullptr;
    std::vector<int32_t> curve_off; /* host: first panel of each curve, then Np */
};

/* Device state of one GMRES cycle (see the GMRES section). */
struct GState {
    int32_t j;     /* current Arnoldi column                               */
    int32_t kmax;  /* columns allowed in this cycle                        */
    int32_t done;  /* converged, broken down or kmax reached               */
    int32_t steps; /* Arnoldi steps taken in this cycle                    */
    double thresh; /* stop when the residual estimate |g_{j+1}| <= thresh  */
    double inv;    /* 1 / h_{j+1,j}: scaling of the next basis vector      */
    double resest; /* |g_{j+1}| after the last step                        */
    double bnorm;  /* ||b|| when the solve left it on the device (first cycle) */
    double rn2;    /* ||b - A x||^2 after the end of the cycle (its last chunk) */
    double *xout;  /* caller's array that receives x at the end of each cycle (or NULL) */
};
static_assert(sizeof(GState) <= 64, "the state and the tail state share the first 128 bytes of gdev");

namespace mhlp {
struct FmmTree;
}

struct mhlp_plan {
    const mhlp_geometry *g = nullptr;
    double alpha = 0.0;
    int64_t M = 0;
    bool onsurf = false;
    double *tx = nullptr, *ty = nullptr; /* owned unless onsurf; off-surface: Morton order */
    int32_t *perm = nullptr;             /* off-surface: caller index of internal target i */
    int32_t *near_ptr = nullptr;         /* [M+1] */
    int32_t *near_panel = nullptr;       /* [nnz] */
    int32_t *near_tgt = nullptr;         /* [nnz] */
    double *near_ts = nullptr;           /* [nnz][2] */
    double *wslp = nullptr, *wdlp = nullptr; /* [nnz][16] */
    double *wgrad = nullptr;  /* off-surface, built on first use: [4][nnz][16] gradient weights */
    bool stokes = false;      /* modified-Stokes (stresslet) plan: operator on [2][N] densities */
    double *wstk = nullptr;   /* stokes: [4][nnz][16] stresslet weights (D11, D12, D21, D22)   */
    mhlp::FmmTree *fmm = nullptr; /* off-surface scalar plans: FMM far field (mhlp_plan_set_fmm) */
    /* on-surface scalar plans up to SYM_NMAX nodes: the double layer's far sum
       with each unordered pair evaluated once (sym_far_kernel) */
    int2 *sym_tiles = nullptr;   /* (row block, column chunk) of each tile */
    int32_t sym_ntiles = 0;
    double *sym_p1 = nullptr;    /* [column chunks][N] row sums */
    double *sym_p2 = nullptr;    /* [row blocks][N] column sums */
    uint32_t *sym_bits = nullptr; /* [N][sym_nw] near panels of each node as bits */
    int32_t sym_nw = 0;
    uint8_t *sym_cls = nullptr;   /* [4 row blocks][Np] piece class of each (row wave, column panel) */
    double *wstkg = nullptr;  /* stokes, off-surface, built on first use: [8][nnz][16] stresslet
                                 gradient weights, block (2a + l) 2 + j = d u_a/d x_l per mu_j */
    double *stk_flux = nullptr; /* stokes: device scalar sum_j w_j mu_j.n_j / |Gamma|           */
    double inv_len = 0.0;     /* 1 / |Gamma| */
    int64_t nnz = 0;
    int32_t fill_mismatch = 0;
    int nsplit = 1;           /* source splits of the far field (small M)   */
    int32_t pps = 0;          /* panels per split                           */
    double *part = nullptr;   /* [2][nsplit][M] partial sums ([4][..] off-surface, for gradients) */
    /* FP64 far field as a stream of (target block, panel) units (far_eval_fp64) */
    uint8_t *wcls = nullptr;  /* [M/64 waves][Np] fine piece + 1 of each (wave, panel) */
    double *fqd = nullptr;    /* [2][KQ_NP] fine-piece scales at alpha (fine_scales) */
    int32_t sk_P[3] = {0, 0, 0}; /* blocks of the launch (resident blocks of the chip) for SLP+DLP, SLP, DLP */
    int32_t sk_S = 0;            /* partial slots per target block, the largest over the three */
    int32_t sk_stride = 1;       /* unit order within a target block (coprime to Np)            */
    double *skpart = nullptr;    /* [2][sk_S][M] */
    NearParams np{};
    double near_factor = 1.2;
    int64_t part_cap = 0;     /* capacity of part (doubles)                 */
    /* GMRES workspace (lazily allocated) */
    double *ws = nullptr;
    int64_t ws_cols = 0;
    double *hdev = nullptr;  /* small device scratch for dot products */
    double *hhost = nullptr; /* pinned host mirror                    */
    /* device-driven GMRES: state + Hessenberg data, captured step graphs */
    char *gdev = nullptr;       /* GState, H, cs, sn, gv, y, h1, h2, hn   */
    int gdev_R = 0;
    GState *gstate_host = nullptr; /* pinned mirror of the state          */
    hipStream_t cap_stream = nullptr;
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        const void *ws = nullptr, *part = nullptr, *gdev = nullptr, *x = nullptr, *b = nullptr;
        int R = 0, nsplit = 0;
    };
    /* keyed by (precision, chunk length S = 0..GMRES_MAX_CHUNK, steps m <= S
       whose Gram-Schmidt runs in one block, end-of-cycle tail or not) */
    std::map<int, StepGraph> graphs;
    int gm_first_steps[2] = {0, 0}; /* steps of the last solve's first cycle, per precision */
};

/* ------------------------------------------------------------------------ */
/* geometry preparation                                                      */
/* ------------------------------------------------------------------------ */
__host__ __device__ inline void geom_prep_body(int64_t p, const double *__restrict__ soa, int64_t N,
                                               double *__restrict__ w, double *__restrict__ nx,
                                               double *__restrict__ ny, double *__restrict__ kappa,
                                               double *__restrict__ pa, double *__restrict__ ph,
                                               double *__restrict__ pcx, double *__restrict__ pcy,
                                               double *__restrict__ prad)
{
    const double *x = soa, *y = soa + N, *dx = soa + 2 * N, *dy = soa + 3 * N, *ddx = soa + 4 * N,
                 *ddy = soa + 5 * N;
    double h = 0.0;
    for (int j = 0; j < 16; ++j) {
        const int64_t m = 16 * p + j;
        const double sp = hypot(dx[m], dy[m]);
        const double wm = GL16_W[j] * sp;
        w[m] = wm;
        nx[m] = -dy[m] / sp;
        ny[m] = dx[m] / sp;
        kappa[m] = (dx[m] * ddy[m] - dy[m] * ddx[m]) / (sp * sp * sp);
        h += wm;
    }
    /* Legendre coefficients of the panel polynomial relative to its node 7
       (an exact double): rounding then scales with the panel size instead of
       the distance from the origin.  Near-field routines add (node 7 - target)
       to the constant term and work in the target's frame (panel_local). */
    const cplx ref = mk(x[16 * p + 7], y[16 * p + 7]);
    cplx a[16];
    for (int mm = 0; mm < 16; ++mm) {
        cplx s = mk(0.0, 0.0);
        for (int j = 0; j < 16; ++j) s = s + LEGC[mm * 16 + j] * (mk(x[16 * p + j], y[16 * p + j]) - ref);
        a[mm] = s;
        pa[(16 * p + mm) * 2] = s.re;
        pa[(16 * p + mm) * 2 + 1] = s.im;
    }
    const cplx c0 = a[0]; /* panel centre relative to ref */
    double r = 0.0;
    for (int j = 0; j < 16; ++j) r = fmax(r, cabs((mk(x[16 * p + j], y[16 * p + j]) - ref) - c0));
    cplx e1 = mk(0.0, 0.0), e0 = mk(0.0, 0.0);
    for (int mm = 0; mm < 16; ++mm) {
        e1 = e1 + a[mm];
        e0 = e0 + ((mm & 1) ? -1.0 : 1.0) * a[mm];
    }
    r = fmax(r, fmax(cabs(e1 - c0), cabs(e0 - c0)));
    const cplx c = ref + c0;
    ph[p] = h;
    pcx[p] = c.re;
    pcy[p] = c.im;
    prad[p] = r;
}

/* given panel ends must lie within this fraction of the panel's arclength of
   the node polynomial's ends and of the next panel's start */
constexpr double PANEL_ENDS_TOL = 1e-6;

/* Checks given panel end points against the node data (Sec. 3.2: a panel is
   the degree-15 polynomial through its 16 nodes, so its ends are tau(-1) and
   tau(1)) and the chain of each closed curve (the end of a panel is the
   start of the next panel of its curve).  ends: [4][Np] xa, ya, xb, yb.
   flag[p]: bit 0 an end further than tol*h from the polynomial's end, bit 1
   the end of p further than tol*h from the start of next[p]. */
__global__ void panel_ends_kernel(const double *__restrict__ pa, const double *__restrict__ x,
                                  const double *__restrict__ y, const double *__restrict__ ph,
                                  const double *__restrict__ ends, const int32_t *__restrict__ next, int64_t Np,
                                  double tol, int32_t *__restrict__ flag)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= Np) return;
    double ax = x[16 * p + 7], ay = y[16 * p + 7], bx = ax, by = ay;
    for (int m = 0; m < 16; ++m) {
        const double cr = pa[(16 * p + m) * 2], ci = pa[(16 * p + m) * 2 + 1];
        bx += cr;
        by += ci;
        ax += (m & 1) ? -cr : cr;
        ay += (m & 1) ? -ci : ci;
    }
    const double lim = tol * ph[p];
    const double xa = ends[p], ya = ends[Np + p], xb = ends[2 * Np + p], yb = ends[3 * Np + p];
    int32_t f = 0;
    if (!(hypot(xa - ax, ya - ay) <= lim && hypot(xb - bx, yb - by) <= lim)) f |= 1;
    const int64_t q = next[p];
    if (!(hypot(xb - ends[q], yb - ends[Np + q]) <= lim)) f |= 2;
    flag[p] = f;
}

__global__ void geom_prep_kernel(const double *__restrict__ soa, int64_t N, int64_t Np, double *__restrict__ w,
                                 double *__restrict__ nx, double *__restrict__ ny, double *__restrict__ kappa,
                                 double *__restrict__ pa, double *__restrict__ ph, double *__restrict__ pcx,
                                 double *__restrict__ pcy, double *__restrict__ prad)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= Np) return;
    geom_prep_body(p, soa, N, w, nx, ny, kappa, pa, ph, pcx, pcy, prad);
}

/* ------------------------------------------------------------------------ */
/* near list                                                                 */
/* ------------------------------------------------------------------------ */
struct GeoView {
    const double *x, *y, *pa, *ph, *pcx, *pcy, *prad;
    int64_t N, Np;
};

/* Legendre coefficients of p(t) - z for panel p: the panel in the frame of
   the target z (the kernels depend on y - x only), so that tau - z near the
   target is formed without cancellation against |z|. */
__host__ __device__ inline void panel_local(const GeoView &G, int64_t p, cplx z, cplx *a)
{
    for (int m = 0; m < 16; ++m) a[m] = mk(G.pa[(16 * p + m) * 2], G.pa[(16 * p + m) * 2 + 1]);
    a[0] = a[0] + (mk(G.x[16 * p + 7], G.y[16 * p + 7]) - z);
}

/* Calls f(panel, self, tstar) for every panel needing a correction at target i
   (panel index ascending). */
template <class F>
__host__ __device__ inline void visit_near(const GeoView &G, int64_t i, cplx z, bool onsurf, double near_factor,
                                  double rho_direct, F &&f)
{
    const int64_t self_p = onsurf ? i / 16 : -1;
    for (int64_t p = 0; p < G.Np; ++p) {
        const double lim = near_factor * G.ph[p];
        const bool self = (p == self_p);
        if (!self) {
            const double dc = cabs(z - mk(G.pcx[p], G.pcy[p])) - G.prad[p];
            if (dc > lim) continue;
        }
        if (self) {
            f(p, (int)(i % 16), mk(GL16_T[i % 16], 0.0));
            continue;
        }
        double dmin = 1e300;
        int jb = 0;
        for (int j = 0; j < 16; ++j) {
            const double d = cabs2(z - mk(G.x[16 * p + j], G.y[16 * p + j]));
            if (d < dmin) {
                dmin = d;
                jb = j;
            }
        }
        if (dmin >= lim * lim) continue;
        cplx a[16];
        panel_local(G, p, z, a);
        cplx ts;
        if (!preimage(a, mk(0.0, 0.0), mk(GL16_T[jb], 0.0), ts)) continue;
        if (bernstein_rho(ts) >= rho_direct) continue;
        f(p, -1, ts);
    }
}

/* One traversal serves both passes of the CSR build (mode 0: count, mode 1:
   fill), so that the two passes run the same instructions and find the same
   pairs.  In fill mode, slots a target reserved but did not fill (which the
   shared code path rules out) are padded with panel -1, which every consumer
   skips, and the event is flagged. */
__host__ __device__ inline void near_list_body(int64_t i, int mode, const GeoView &G, const double *__restrict__ tx,
                                               const double *__restrict__ ty, int onsurf, double near_factor,
                                               double rho_direct, int32_t *__restrict__ cnt,
                                               const int32_t *__restrict__ ptr, int32_t *__restrict__ panel,
                                               int32_t *__restrict__ tgt, double *__restrict__ ts_out,
                                               int32_t *__restrict__ mismatch)
{
    int32_t q = mode ? ptr[i] : 0;
    const int32_t qend = mode ? ptr[i + 1] : INT_MAX;
    const int32_t q0 = q;
    visit_near(G, i, mk(tx[i], ty[i]), onsurf != 0, near_factor, rho_direct, [&](int64_t p, int, cplx ts) {
        if (mode && q < qend) {
            panel[q] = (int32_t)p;
            tgt[q] = (int32_t)i;
            ts_out[2 * q] = ts.re;
            ts_out[2 * q + 1] = ts.im;
        }
        ++q;
    });
    if (!mode) {
        cnt[i] = q - q0;
        return;
    }
    if (q != qend) mismatch[0] = 1;
    for (int32_t r = q; r < qend; ++r) {
        panel[r] = -1;
        tgt[r] = (int32_t)i;
        ts_out[2 * r] = 0.0;
        ts_out[2 * r + 1] = 0.0;
    }
}

__global__ void near_list_kernel(int mode, GeoView G, const double *__restrict__ tx, const double *__restrict__ ty,
                                 int64_t M, int onsurf, double near_factor, double rho_direct,
                                 int32_t *__restrict__ cnt, const int32_t *__restrict__ ptr,
                                 int32_t *__restrict__ panel, int32_t *__restrict__ tgt, double *__restrict__ ts_out,
                                 int32_t *__restrict__ mismatch)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    near_list_body(i, mode, G, tx, ty, onsurf, near_factor, rho_direct, cnt, ptr, panel, tgt, ts_out, mismatch);
}

/* exclusive scan of cnt[0..M) into ptr[0..M]; one block of 1024 threads */
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t *__restrict__ cnt, int64_t M,
                                                    int32_t *__restrict__ ptr)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (M + 1023) / 1024;
    const int64_t b = t * chunk, e = (b + chunk < M) ? b + chunk : M;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        ptr[i] = (int32_t)run;
        run += cnt[i];
    }
    if (t == 1023) ptr[M] = (int32_t)part[1023];
}

__host__ __device__ inline void near_weights_body(int64_t q, const GeoView &G, const double *__restrict__ tx,
                                                  const double *__restrict__ ty, int onsurf,
                                                  const int32_t *__restrict__ panel, const int32_t *__restrict__ tgt,
                                                  const double *__restrict__ ts, double alpha, const NearParams &P,
                                                  double *__restrict__ wsl, double *__restrict__ wdl)
{
    const int64_t p = panel[q], i = tgt[q];
    if (p < 0 || p >= G.Np) {
        for (int j = 0; j < 16; ++j) wsl[16 * q + j] = wdl[16 * q + j] = 0.0;
        return;
    }
    cplx a[16];
    panel_local(G, p, mk(tx[i], ty[i]), a);
    const int self = (onsurf && i / 16 == p) ? (int)(i % 16) : -1;
    double Ws[16], Wd[16];
    pair_weights(a, G.ph[p], mk(0.0, 0.0), self, mk(ts[2 * q], ts[2 * q + 1]), alpha, P, Ws, Wd);
    for (int j = 0; j < 16; ++j) {
        wsl[16 * q + j] = Ws[j];
        wdl[16 * q + j] = Wd[j];
    }
}

__global__ void near_weights_kernel(GeoView G, const double *__restrict__ tx, const double *__restrict__ ty,
                                    int onsurf, const int32_t *__restrict__ panel, const int32_t *__restrict__ tgt,
                                    const double *__restrict__ ts, int64_t nnz, double alpha, NearParams P,
                                    double *__restrict__ wsl, double *__restrict__ wdl)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    near_weights_body(q, G, tx, ty, onsurf, panel, tgt, ts, alpha, P, wsl, wdl);
}

/* gradient correction weights of the off-surface pairs: wg[b][q][j] */
__global__ void near_grad_weights_kernel(GeoView G, const double *__restrict__ tx, const double *__restrict__ ty,
                                         const int32_t *__restrict__ panel, const int32_t *__restrict__ tgt,
                                         const double *__restrict__ ts, int64_t nnz, double alpha, NearParams P,
                                         double *__restrict__ wg)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const int64_t p = panel[q], i = tgt[q];
    double W[4][16];
    if (p < 0 || p >= G.Np) {
        for (int b = 0; b < 4; ++b)
            for (int j = 0; j < 16; ++j) W[b][j] = 0.0;
    } else {
        cplx a[16];
        panel_local(G, p, mk(tx[i], ty[i]), a);
        pair_grad_weights(a, G.ph[p], mk(0.0, 0.0), mk(ts[2 * q], ts[2 * q + 1]), alpha, P, W);
    }
    for (int b = 0; b < 4; ++b)
        for (int j = 0; j < 16; ++j) wg[(b * nnz + q) * 16 + j] = W[b][j];
}

/* stresslet correction weights of all pairs: ws[b][q][j] */
__global__ void near_stokes_weights_kernel(GeoView G, const double *__restrict__ tx, const double *__restrict__ ty,
                                           int onsurf, const int32_t *__restrict__ panel,
                                           const int32_t *__restrict__ tgt, const double *__restrict__ ts,
                                           int64_t nnz, double alpha, NearParams P, double *__restrict__ wst)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const int64_t p = panel[q], i = tgt[q];
    double W[4][16];
    if (p < 0 || p >= G.Np) {
        for (int b = 0; b < 4; ++b)
            for (int j = 0; j < 16; ++j) W[b][j] = 0.0;
    } else {
        cplx a[16];
        panel_local(G, p, mk(tx[i], ty[i]), a);
        const int self = (onsurf && i / 16 == p) ? (int)(i % 16) : -1;
        pair_stokes_weights(a, G.ph[p], mk(0.0, 0.0), self, mk(ts[2 * q], ts[2 * q + 1]), alpha, P, W);
    }
    for (int b = 0; b < 4; ++b)
        for (int j = 0; j < 16; ++j) wst[(b * nnz + q) * 16 + j] = W[b][j];
}

/* stresslet gradient correction weights of the off-surface pairs: wg[b][q][j] */
__global__ void near_stokes_grad_weights_kernel(GeoView G, const double *__restrict__ tx,
                                                const double *__restrict__ ty, const int32_t *__restrict__ panel,
                                                const int32_t *__restrict__ tgt, const double *__restrict__ ts,
                                                int64_t nnz, double alpha, NearParams P, double *__restrict__ wg)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const int64_t p = panel[q], i = tgt[q];
    double W[8][16];
    if (p < 0 || p >= G.Np) {
        for (int b = 0; b < 8; ++b)
            for (int j = 0; j < 16; ++j) W[b][j] = 0.0;
    } else {
        cplx a[16];
        panel_local(G, p, mk(tx[i], ty[i]), a);
        pair_stokes_grad_weights(a, G.ph[p], mk(0.0, 0.0), mk(ts[2 * q], ts[2 * q + 1]), alpha, P, W);
    }
    for (int b = 0; b < 8; ++b)
        for (int j = 0; j < 16; ++j) wg[(b * nnz + q) * 16 + j] = W[b][j];
}

/* ------------------------------------------------------------------------ */
/* far field + corrections, FP64                                             */
/* ------------------------------------------------------------------------ */
constexpr int FT_THREADS = 256;
constexpr int FT_SRC = 256; /* sources per LDS tile = 16 panels */

struct FarArgs {
    const double *sx, *sy, *sw, *snx, *sny;
    const double *sigma, *mu;
    int64_t N;
    const double *tx, *ty;
    int64_t M;
    const int32_t *nptr, *npan;
    const double *wsl, *wdl;
    double alpha;
    double half_term; /* 0.5 for (1/2 I + D) on an on-surface plan, else 0 */
    double *us, *ud;
    int64_t Np;
    int32_t pps;      /* panels per source split (blockIdx.y) */
    double *part_s, *part_d; /* [nsplit][M] partial far sums when split */
    /* device-driven GMRES: when gs is set the density is column gs->j of the
       basis (mu + j*jstride) and the launch does nothing once gs->done */
    const GState *gs;
    int64_t jstride;
    const int32_t *perm; /* output index of internal target i (NULL: identity) */
    const double *pcx, *pcy, *prad; /* bounding circle of each panel */
    /* FP64 far field as a stream of (target block, panel) units: the launch's
       skP blocks take equal contiguous ranges of the skU = TB Np units and
       leave one partial sum per target block they touch, slot = block - first
       block of that target block ([layer][skS][M]); wcls[wave Np + p] - 1 is
       the fine piece every pair of the wave with panel p lies in (plan time) */
    int64_t skU;
    int32_t skP, skS;
    int32_t skStride; /* unit j of a target block is panel (j skStride) mod Np */
    double *skps, *skpd;
    const uint8_t *wcls = nullptr;
    const double *fq = nullptr; /* [2][KQ_NP] scales of the fine pieces at the plan's alpha (fine_scales) */
};


/* density of a far launch: fixed, or the current GMRES basis column;
   false when the launch is a no-op */
__device__ __forceinline__ bool far_density(const FarArgs &A, const double *&mu)
{
    mu = A.mu;
    if (A.gs) {
        if (A.gs->done) return false;
        mu += (int64_t)A.gs->j * A.jstride;
    }
    return true;
}

/* Near corrections, 1/(2 pi) scaling and identity term for target i. */
template <bool SLP, bool DLP>
__device__ __forceinline__ void far_epilogue(const FarArgs &A, const double *__restrict__ mu, int64_t i, double accs,
                                             double accd)
{
    double cs = 0.0, cd = 0.0;
    for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
        const int64_t p = A.npan[q];
        if (p < 0) continue;
        for (int jj = 0; jj < 16; ++jj) {
            if (SLP) cs = fma(A.wsl[16 * (int64_t)q + jj], A.sigma[16 * p + jj], cs);
            if (DLP) cd = fma(A.wdl[16 * (int64_t)q + jj], mu[16 * p + jj], cd);
        }
    }
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
    if (SLP) A.us[o] = fma(INV_2PI, accs, cs);
    if (DLP) {
        double v = fma(INV_2PI, accd, cd);
        /* identity term: only on-surface plans (targets are the nodes, M == N) */
        if (A.half_term != 0.0) v = fma(A.half_term, mu[i], v);
        A.ud[o] = v;
    }
}

/* Sum of the source-split partials, near corrections, 1/(2 pi) scaling and
   identity term.  A block takes FZ_TG consecutive targets with L lanes each
   (lane l is the l-th group of FZ_TG threads, so the partial loads of a lane
   are row segments of FZ_TG consecutive values; small blocks spread short
   lists over many CUs): lane
   l adds the partials l, l + L, ... and the correction terms of node l, l + L,
   ... of each near panel; the lane sums are then added in lane order.  L = 16
   for short target lists (many splits, few targets: the on-surface operator),
   L = 1 (one thread per target, 256 targets a block) otherwise. */
constexpr int FZ_TG = 16, FZ_L = 16, FZ_SHORT = 16384;

template <bool SLP, bool DLP, int L>
__global__ __launch_bounds__(L == 1 ? 256 : FZ_TG * L) void far_finalize(FarArgs A, int nsplit)
{
    constexpr int TG = L == 1 ? 256 : FZ_TG;
    __shared__ double red[4][L == 1 ? 1 : L][L == 1 ? 1 : TG]; /* far S, near S, far D, near D */
    const double *mu;
    if (!far_density(A, mu)) return; /* the same for every thread of the launch */
    const int g = threadIdx.x % TG, l = L == 1 ? 0 : threadIdx.x / TG; /* L = 1: loops unroll */
    const int64_t i = blockIdx.x * (int64_t)TG + g;
    double fs = 0.0, ns = 0.0, fd = 0.0, nd = 0.0;
    if (i < A.M) {
        for (int k = l; k < nsplit; k += L) {
            if (SLP) fs += A.part_s[k * A.M + i];
            if (DLP) fd += A.part_d[k * A.M + i];
        }
        for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
            const int64_t p = A.npan[q];
            if (p < 0) continue;
            for (int jj = l; jj < 16; jj += L) {
                if (SLP) ns = fma(A.wsl[16 * (int64_t)q + jj], A.sigma[16 * p + jj], ns);
                if (DLP) nd = fma(A.wdl[16 * (int64_t)q + jj], mu[16 * p + jj], nd);
            }
        }
    }
    if (L > 1) {
        red[0][l][g] = fs;
        red[1][l][g] = ns;
        red[2][l][g] = fd;
        red[3][l][g] = nd;
        __syncthreads();
        if (l != 0) return;
        for (int q = 1; q < L; ++q) {
            fs += red[0][q][g];
            ns += red[1][q][g];
            fd += red[2][q][g];
            nd += red[3][q][g];
        }
    }
    if (i >= A.M) return;
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
    if (SLP) A.us[o] = fma(INV_2PI, fs, ns);
    if (DLP) {
        double v = fma(INV_2PI, fd, nd);
        if (A.half_term != 0.0) v = fma(A.half_term, mu[i], v);
        A.ud[o] = v;
    }
}

/* Sum over the 64 lanes of a wave with DPP moves (no LDS traffic): adds of
   the value 1, 2, 4, 8 lanes lower within each row of 16 lanes, then the last
   lane of each row carried into the next row (row_bcast15) and lane 31 into
   the upper half (row_bcast31): lane 63 then holds the sum, a fixed tree, and
   readlane returns it to every lane.  Lanes with no source add zero. */
__device__ __forceinline__ double dpp_add(double v, int ctrl_sel)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int rlo, rhi;
    switch (ctrl_sel) {
    case 0: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, false);
            rhi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, false); break;
    case 1: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x112, 0xf, 0xf, false);
            rhi = __builtin_amdgcn_update_dpp(0, hi, 0x112, 0xf, 0xf, false); break;
    case 2: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x114, 0xf, 0xf, false);
            rhi = __builtin_amdgcn_update_dpp(0, hi, 0x114, 0xf, 0xf, false); break;
    case 3: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x118, 0xf, 0xf, false);
            rhi = __builtin_amdgcn_update_dpp(0, hi, 0x118, 0xf, 0xf, false); break;
    case 4: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xa, 0xf, false);
            rhi = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xa, 0xf, false); break;
    default: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xc, 0xf, false);
             rhi = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xc, 0xf, false); break;
    }
    return v + __hiloint2double(rhi, rlo);
}

__device__ __forceinline__ double wave_sum_dpp(double v)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) v = dpp_add(v, k);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

/* ---- on-surface double layer, each unordered far pair once ----
   K1(z)/r depends on the pair only through r, so one evaluation serves the
   term of source j at node i and of source i at node j.  Tiles pair a block of
   SYM_R = 256 row nodes (16 panels) with a chunk of SYM_C = 16 column nodes
   (one panel; small tiles keep enough blocks in flight); tile (I, J) exists
   when the chunk does not start before the block (column panels >= 16 I), and on the block's own chunks only row < column
   counts.  The row node takes the column terms (unless the column panel is
   listed near it) into p1[J][i]; each column node takes the row terms (unless
   the row's panel is listed near the column node), summed over lanes by a
   butterfly and over waves in order, into p2[I][j].  Every pair of distinct
   nodes is evaluated in exactly one tile. */
constexpr int SYM_R = 256, SYM_C = 16, SYM_RP = SYM_R / 16, SYM_CP = SYM_C / 16, SYM_NMAX = 8192;

/* sum over the 64 lanes of a wave by a fixed butterfly (every lane gets it) */
__device__ __forceinline__ double gsf_wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}


struct SymArgs {
    FarArgs A;
    const int2 *tiles;
    double *p1, *p2;
    const uint32_t *bits; /* [N][nw] near panels of each node */
    int nw;
    const uint8_t *cls;   /* [N/64 row waves][Np] fine piece + 1 of every pair of (wave, column panel); bit 7:
                             some pair of them is near on either side */
};
static_assert(SYM_RP == 16 && SYM_CP == 1, "the near masks below read 16 row panels and one column panel");

/* per node, its near panels as a bit set of nw words */
__global__ void near_bits_kernel(const int32_t *__restrict__ nptr, const int32_t *__restrict__ npan, int64_t M,
                                 int nw, uint32_t *__restrict__ bits)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    uint32_t *b = bits + i * nw;
    for (int k = 0; k < nw; ++k) b[k] = 0u;
    for (int32_t q = nptr[i]; q < nptr[i + 1]; ++q) {
        const int32_t p = npan[q];
        if (p >= 0) b[p >> 5] |= 1u << (p & 31);
    }
}

/* the column loop of sym_far_kernel for 16 columns, two at a time, with the
   fine piece PC (-1: z <= 2; KQ_NP: per-pair selection) of the wave and column
   panel.  MASK: the wave has near pairs (on either side) or is on the diagonal
   block, where only row < column counts.  The row terms accumulate in the
   returned sum; the column terms go to colv[s][t] for the block's reduction. */
template <int PC, bool MASK>
__device__ __forceinline__ double sym_columns(const FarArgs &A, const FarConst &fc, int ncol, int64_t i, int64_t j0,
                                              bool valid, bool diag, double x, double y, double dix, double diy,
                                              uint32_t rnear, int kp, const double *cx, const double *cy,
                                              const double *cdx, const double *cdy, const uint32_t *cmask,
                                              double (*colv)[SYM_R])
{
    constexpr int K = PC < 0 || PC >= KQ_NP ? 0 : PC;
    const FarTab T = far_table();
    double qa, qk;
    fine_q<K>(A.fq, qa, qk);
    const int t = threadIdx.x;
    double acc = 0.0;
#pragma unroll 1
    for (int s = 0; s < ncol; s += 2) {
        const int64_t ja = j0 + s, jb = ja + 1;
        const double ex0 = x - cx[s], ey0 = y - cy[s], ex1 = x - cx[s + 1], ey1 = y - cy[s + 1];
        double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
        bool r0 = valid, r1 = valid, c0 = valid, c1 = valid;
        if (MASK) {
            /* row and column terms wanted for the two columns (s, s + 1 share a panel) */
            const bool rfar = valid && !(rnear & 1u);
            r0 = rfar && (!diag || i < ja);
            r1 = rfar && (!diag || i < jb);
            c0 = valid && !((cmask[s] >> kp) & 1u) && (!diag || i < ja);
            c1 = valid && !((cmask[s + 1] >> kp) & 1u) && (!diag || i < jb);
            r20 = (r0 || c0) ? r20 : 1.0; /* unused pairs (the node itself among them) */
            r21 = (r1 || c1) ? r21 : 1.0;
        }
        K01 o0, o1;
        if constexpr (PC >= KQ_NP)
            k01_far2<false, true, true, true>(T, fc, r20, r21, o0, o1);
        else
            k01_far2_fixed<false, true, PC>(T, fc, qa, qk, r20, r21, o0, o1);
        const double f0 = fma(ex0, cdx[s], ey0 * cdy[s]), f1 = fma(ex1, cdx[s + 1], ey1 * cdy[s + 1]);
        const double g0 = -fma(ex0, dix, ey0 * diy), g1 = -fma(ex1, dix, ey1 * diy);
        if (MASK) {
            if (r0) acc = fma(o0.ak1r, f0, acc);
            if (r1) acc = fma(o1.ak1r, f1, acc);
            colv[s][t] = c0 ? o0.ak1r * g0 : 0.0;
            colv[s + 1][t] = c1 ? o1.ak1r * g1 : 0.0;
        } else {
            acc = fma(o1.ak1r, f1, fma(o0.ak1r, f0, acc));
            colv[s][t] = o0.ak1r * g0;
            colv[s + 1][t] = o1.ak1r * g1;
        }
    }
    return acc;
}

template <bool MASK>
__device__ __forceinline__ double sym_columns_pc(int pc, const FarArgs &A, const FarConst &fc, int ncol, int64_t i,
                                                 int64_t j0, bool valid, bool diag, double x, double y, double dix,
                                                 double diy, uint32_t rnear, int kp, const double *cx,
                                                 const double *cy, const double *cdx, const double *cdy,
                                                 const uint32_t *cmask, double (*colv)[SYM_R])
{
    switch (pc) {
#define MHLP_SYM_PC(PCV)                                                                                   \
    case PCV:                                                                                              \
        return sym_columns<PCV, MASK>(A, fc, ncol, i, j0, valid, diag, x, y, dix, diy, rnear, kp, cx, cy, cdx, \
                                      cdy, cmask, colv);
        MHLP_SYM_PC(-1)
        MHLP_SYM_PC(0)
        MHLP_SYM_PC(1)
        MHLP_SYM_PC(2)
        MHLP_SYM_PC(3)
        MHLP_SYM_PC(4)
        MHLP_SYM_PC(5)
        MHLP_SYM_PC(6)
        MHLP_SYM_PC(7)
        MHLP_SYM_PC(8)
        MHLP_SYM_PC(9)
        MHLP_SYM_PC(10)
        MHLP_SYM_PC(11)
        MHLP_SYM_PC(12)
        MHLP_SYM_PC(13)
        MHLP_SYM_PC(14)
#undef MHLP_SYM_PC
    default:
        return sym_columns<KQ_NP, MASK>(A, fc, ncol, i, j0, valid, diag, x, y, dix, diy, rnear, kp, cx, cy, cdx,
                                        cdy, cmask, colv);
    }
}

/* One tile: 256 row nodes (block I) against the 16 nodes of column panel J.
   The row sums go to p1[J][i]; the column terms of the tile's 256 rows are
   reduced through LDS (each thread adds 16 rows of one column, 16 lanes then
   combine by a fixed butterfly) into p2[I][j].  Each wave takes the fine piece
   of its (row wave, column panel) from the plan's class table and checks near
   masks only when that pair of wave and panel has near pairs on either side or
   lies on the diagonal block. */
__global__ __launch_bounds__(SYM_R) void sym_far_kernel(SymArgs S)
{
    const FarArgs &A = S.A;
    __shared__ double cx[SYM_C], cy[SYM_C], cdx[SYM_C], cdy[SYM_C];
    __shared__ uint32_t cmask[SYM_C];
    __shared__ double colv[SYM_C][SYM_R];
    const double *mu;
    if (!far_density(A, mu)) return; /* the same for the whole launch */
    const int2 tl = S.tiles[blockIdx.x];
    const int I = tl.x, J = tl.y, t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t N = A.N, i = (int64_t)I * SYM_R + t, j0 = (int64_t)J * SYM_C;
    const int pb = SYM_RP * I; /* first panel of the row block */
    if (t < SYM_C) {
        const int64_t j = j0 + t;
        double xj = 0.0, yj = 0.0, dx = 0.0, dy = 0.0;
        uint32_t msk = 0;
        if (j < N) {
            xj = A.sx[j];
            yj = A.sy[j];
            const double m = (A.alpha * A.sw[j]) * mu[j];
            dx = m * A.snx[j];
            dy = m * A.sny[j];
            msk = (S.bits[j * S.nw + (pb >> 5)] >> (pb & 31)) & 0xFFFFu; /* the block's 16 panels */
        }
        cx[t] = xj;
        cy[t] = yj;
        cdx[t] = dx;
        cdy[t] = dy;
        cmask[t] = msk;
    }
    const bool valid = i < N;
    double x = 0.0, y = 0.0, dix = 0.0, diy = 0.0;
    uint32_t rnear = 0; /* bit 0: column panel J listed near row i */
    int kp = 0;         /* row panel within the block */
    if (valid) {
        x = A.sx[i];
        y = A.sy[i];
        const double m = (A.alpha * A.sw[i]) * mu[i];
        dix = m * A.snx[i];
        diy = m * A.sny[i];
        kp = (int)(i / 16) - pb;
        rnear = (S.bits[i * S.nw + (J >> 5)] >> (J & 31)) & 1u;
    }
    const bool diag = SYM_CP * J < pb + SYM_RP; /* the chunk lies in the row block */
    __syncthreads();
    const FarConst fc = far_const(A.alpha);
    const int ncol = (int)min((int64_t)SYM_C, N - j0);
    const int cw = S.cls[((int64_t)I * (SYM_R / 64) + wv) * A.Np + J];
    const int pc = (cw & 0x7f) - 1;
    const double acc = (diag || (cw & 0x80))
                           ? sym_columns_pc<true>(pc, A, fc, ncol, i, j0, valid, diag, x, y, dix, diy, rnear, kp,
                                                  cx, cy, cdx, cdy, cmask, colv)
                           : sym_columns_pc<false>(pc, A, fc, ncol, i, j0, valid, diag, x, y, dix, diy, rnear, kp,
                                                   cx, cy, cdx, cdy, cmask, colv);
    __syncthreads();
    /* column c = t / 16: thread (c, g) adds rows g, g + 16, ..., g + 240, then the
       16 lanes of the column combine */
    {
        const int c = t >> 4, g = t & 15;
        double sc = 0.0;
        if (c < ncol)
            for (int r = g; r < SYM_R; r += 16) sc += colv[c][r];
        for (int off = 8; off > 0; off >>= 1) sc += __shfl_xor(sc, off);
        if (g == 0 && c < ncol) S.p2[(int64_t)I * N + j0 + c] = sc;
    }
    if (valid) S.p1[(int64_t)J * N + i] = acc;
}

/* Plan time, symmetric on-surface plans: for every (wave of 64 row nodes,
   column panel) the fine piece that holds z for every pair the tile evaluates
   (row i < column j, and not near on both sides; exact extreme distances; a
   two-neighbour piece when they straddle one boundary, KQ_NP + 1 otherwise),
   plus bit 7 when some such pair is near on either side (the row node lists
   the column panel, or the column node lists the row node's panel).  Pairs
   with j <= i are never evaluated by tile (row block of i, column panel of j),
   which exists only for column panels from 16 x the row block on. */
__global__ __launch_bounds__(256) void sym_class_kernel(const double *__restrict__ x, const double *__restrict__ y,
                                                        int64_t N, int64_t Np, double alpha,
                                                        const uint32_t *__restrict__ bits, int nw,
                                                        uint8_t *__restrict__ cls)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool valid = i < N;
    const int64_t iv = valid ? i : N - 1;
    const int64_t w = i >> 6, pi = iv / 16;
    const double xi = x[iv], yi = y[iv];
    for (int64_t p = 0; p < Np; ++p) {
        double r2lo = 1e300, r2hi = -1.0;
        const bool rn = ((bits[iv * nw + (p >> 5)] >> (p & 31)) & 1u) != 0;
        bool near = false;
        for (int jj = 0; jj < 16; ++jj) {
            const int64_t j = 16 * p + jj;
            if (!valid || j <= i) continue;
            const bool cn = ((bits[j * nw + (pi >> 5)] >> (pi & 31)) & 1u) != 0;
            near = near || rn || cn;
            if (rn && cn) continue; /* neither term is taken */
            const double ex = xi - x[j], ey = yi - y[j];
            const double r2 = fma(ex, ex, ey * ey);
            r2lo = fmin(r2lo, r2);
            r2hi = fmax(r2hi, r2);
        }
        int lo = KQ_NB + 1, hi = -1; /* lanes without pairs do not vote */
        if (r2hi >= 0.0) {
            const double zlo = alpha * sqrt(r2lo), zhi = alpha * sqrt(r2hi);
            lo = 0;
            hi = 0;
            for (int b = 0; b < KQ_NB; ++b) {
                lo += zlo > KQ_B[b] ? 1 : 0;
                hi += zhi > KQ_B[b] ? 1 : 0;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        int c = KQ_NP + 1;
        if (hi < 0)
            c = KQ_NP + 1;
        else if (lo == hi)
            c = lo; /* piece lo - 1 (0: z <= 2) */
        else if (lo >= 1 && hi == lo + 1 && lo <= KQ_NB - 1)
            c = KQ_NB + lo; /* pieces lo - 1 and lo */
        if (__ballot(near) != 0) c |= 0x80;
        if ((threadIdx.x & 63) == 0) cls[w * Np + p] = (uint8_t)c;
    }
}

/* node n: row sums of the chunks from its block on, column sums of the blocks
   up to its own, then the near corrections, 1/(2 pi) and the identity term;
   FZ_L lanes per node and FZ_TG nodes per block as in far_finalize.  Every
   thread of the block returns. */
__device__ __forceinline__ void sym_finalize_body(const SymArgs &S, const double *mu, int nchunk,
                                                  double (&red)[2][FZ_L][FZ_TG])
{
    const FarArgs &A = S.A;
    const int g = threadIdx.x % FZ_TG, l = threadIdx.x / FZ_TG;
    const int64_t n = blockIdx.x * (int64_t)FZ_TG + g;
    double fd = 0.0, nd = 0.0;
    if (n < A.N) {
        const int B = (int)(n / SYM_R);
#pragma unroll 4
        for (int c = SYM_RP * B / SYM_CP + l; c < nchunk; c += FZ_L) fd += S.p1[(int64_t)c * A.N + n];
        for (int b = l; b <= B; b += FZ_L) fd += S.p2[(int64_t)b * A.N + n];
        for (int32_t q = A.nptr[n]; q < A.nptr[n + 1]; ++q) {
            const int64_t p = A.npan[q];
            if (p < 0) continue;
            nd = fma(A.wdl[16 * (int64_t)q + l], mu[16 * p + l], nd);
        }
    }
    red[0][l][g] = fd;
    red[1][l][g] = nd;
    __syncthreads();
    if (l == 0 && n < A.N) {
        for (int q = 1; q < FZ_L; ++q) {
            fd += red[0][q][g];
            nd += red[1][q][g];
        }
        double v = fma(INV_2PI, fd, nd);
        if (A.half_term != 0.0) v = fma(A.half_term, mu[n], v);
        A.ud[n] = v;
    }
}

__global__ __launch_bounds__(FZ_TG *FZ_L) void sym_finalize(SymArgs S, int nchunk)
{
    __shared__ double red[2][FZ_L][FZ_TG];
    const double *mu;
    if (!far_density(S.A, mu)) return;
    sym_finalize_body(S, mu, nchunk, red);
}

/* the 16 sources of one LDS panel (offset l0) against the lane's target: PC the
   fine piece (-1: z <= 2; KQ_NP: per-pair selection over the three-piece fits) */
template <bool SLP, bool DLP, int PC>
__device__ __forceinline__ void far_panel_fp64(const FarArgs &A, const FarConst &fc, double x, double y,
                                               const double *lx, const double *ly, const double *lq,
                                               const double *ldx, const double *ldy, int l0, double &accs,
                                               double &accd)
{
    constexpr int K = PC < 0 || PC >= KQ_NP ? 0 : PC;
    /* the table pointer once per panel: the piece's coefficients stay in
       scalar registers for its 8 loop trips */
    const FarTab T = far_table();
    double qa, qk;
    fine_q<K>(A.fq, qa, qk);
#pragma unroll 1
    for (int s = 0; s < 16; s += 2) {
        const int a0 = l0 + s, a1 = a0 + 1;
        const double ex0 = x - lx[a0], ey0 = y - ly[a0];
        const double ex1 = x - lx[a1], ey1 = y - ly[a1];
        const double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
        K01 o0, o1;
        if constexpr (PC >= KQ_NP)
            k01_far2<SLP, DLP, true, true>(T, fc, r20, r21, o0, o1);
        else
            k01_far2_fixed<SLP, DLP, PC>(T, fc, qa, qk, r20, r21, o0, o1);
        if (SLP) accs = fma(o1.k0, lq[a1], fma(o0.k0, lq[a0], accs));
        if (DLP)
            accd = fma(o1.ak1r, fma(ex1, ldx[a1], ey1 * ldy[a1]), fma(o0.ak1r, fma(ex0, ldx[a0], ey0 * ldy[a0]), accd));
    }
}

/* waves per SIMD the FP64 far kernel is compiled for (96 registers per lane) */
constexpr int SK_WAVES = 4;

/* The stream position of hardware block b of a P-block launch.  The chip's
   dispatcher deals blocks to its 8 XCDs (each with its own L2) in turn, block b
   to XCD b mod 8; numbering the stream XCD by XCD gives each XCD one
   contiguous stretch of it, so the blocks that share a target block share an
   L2 and read its targets and class rows from there.  A bijection of
   [0, P) for every P. */
__device__ __forceinline__ int64_t xcd_major(int64_t b, int64_t P)
{
    const int64_t q = P >> 3, r = P & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

/* first unit of block b of the stream decomposition, and the block that holds unit u */
__host__ __device__ inline int64_t sk_start(int64_t U, int P, int64_t b) { return (U * b) / P; }
__host__ __device__ inline int64_t sk_block_of(int64_t U, int P, int64_t u)
{
    int64_t b = (u * P) / U;
    while (b > 0 && sk_start(U, P, b) > u) --b;
    while (b + 1 < P && sk_start(U, P, b + 1) <= u) ++b;
    return b;
}

/* The FP64 far field as a stream of units (target block of FT_THREADS targets,
   one panel): block b takes units sk_start(b) .. sk_start(b+1) - 1 in order,
   i.e. a run of units of one target block, then possibly the start of the
   next, and so on; every block has the same number of units.  Unit j of a
   target block is panel (j skStride) mod Np, a stride near 0.618 Np coprime to
   Np, so that each block's run mixes panels near and far from its targets and
   the blocks cost about the same.  For each target block it touches, the block
   sums its panels (a target skips the panels it lists as near) and writes the
   partial sums of its targets into slot (b - first block of the target block);
   far_sk_finalize adds the slots in order with the near corrections.  Sources
   are staged in LDS 16 panels at a time; each panel is evaluated with the fine
   piece the plan-time class table gives for (wave, panel) (low 7 bits: piece
   + 1, KQ_NP + 1 for the per-pair selection; bit 7: some target of the wave
   lists the panel, only then do the lanes look it up in their lists). */
template <bool SLP, bool DLP>
__global__ __launch_bounds__(FT_THREADS, SK_WAVES) void far_eval_fp64(FarArgs A)
{
    __shared__ double lx[FT_SRC], ly[FT_SRC], lq[FT_SRC], ldx[FT_SRC], ldy[FT_SRC];
    __shared__ int32_t lp[16];
    const double *mu;
    if (!far_density(A, mu)) return;
    const int64_t Np = A.Np;
    const int64_t blk = xcd_major(blockIdx.x, A.skP);
    int64_t u = sk_start(A.skU, A.skP, blk);
    const int64_t uend = sk_start(A.skU, A.skP, blk + 1);
    const FarConst fc = far_const(A.alpha);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    while (u < uend) {
        const int64_t tb = u / Np;
        const int64_t jb = u - tb * Np;
        const int64_t je = min(Np, uend - tb * Np);
        const int64_t i = tb * FT_THREADS + threadIdx.x;
        const bool valid = i < A.M;
        /* lanes past the last target repeat its position (results discarded) */
        const int64_t iv = valid ? i : A.M - 1;
        const double x = A.tx[iv], y = A.ty[iv];
        const int32_t k0 = A.nptr[iv], k1 = A.nptr[iv + 1];
        const uint8_t *cls = A.wcls + (tb * (FT_THREADS / 64) + wv) * Np;
        double accs = 0.0, accd = 0.0;
        for (int64_t jt = jb; jt < je; jt += 16) {
            const int npl = (je - jt) < 16 ? (int)(je - jt) : 16;
            __syncthreads();
            if (threadIdx.x < 16 * npl) {
                const int64_t p = ((jt + (threadIdx.x >> 4)) * A.skStride) % Np;
                const int64_t jn = 16 * p + (threadIdx.x & 15);
                const double wj = A.sw[jn];
                lx[threadIdx.x] = A.sx[jn];
                ly[threadIdx.x] = A.sy[jn];
                if (SLP) lq[threadIdx.x] = wj * A.sigma[jn];
                if (DLP) {
                    /* alpha goes with the dipole: the pair evaluates K1(z)/r */
                    const double m = (A.alpha * wj) * mu[jn];
                    ldx[threadIdx.x] = m * A.snx[jn];
                    ldy[threadIdx.x] = m * A.sny[jn];
                }
                if ((threadIdx.x & 15) == 0) lp[threadIdx.x >> 4] = (int32_t)p;
            }
            __syncthreads();
            for (int pl = 0; pl < npl; ++pl) {
                const int32_t p = lp[pl];
                const int cw = cls[p];
                if (cw & 0x80) { /* some target of the wave lists the panel */
                    bool listed = false;
                    for (int32_t q = k0; q < k1; ++q) listed = listed || A.npan[q] == p;
                    if (listed) continue;
                }
                const int pc = (cw & 0x7f) - 1;
                const int l0 = pl * 16;
                switch (pc) {
#define MHLP_FAR_PANEL(PCV)                                                                               \
    case PCV:                                                                                              \
        far_panel_fp64<SLP, DLP, PCV>(A, fc, x, y, lx, ly, lq, ldx, ldy, l0, accs, accd);                  \
        break;
                    MHLP_FAR_PANEL(-1)
                    MHLP_FAR_PANEL(0)
                    MHLP_FAR_PANEL(1)
                    MHLP_FAR_PANEL(2)
                    MHLP_FAR_PANEL(3)
                    MHLP_FAR_PANEL(4)
                    MHLP_FAR_PANEL(5)
                    MHLP_FAR_PANEL(6)
                    MHLP_FAR_PANEL(7)
                    MHLP_FAR_PANEL(8)
                    MHLP_FAR_PANEL(9)
                    MHLP_FAR_PANEL(10)
                    MHLP_FAR_PANEL(11)
                    MHLP_FAR_PANEL(12)
                    MHLP_FAR_PANEL(13)
                    MHLP_FAR_PANEL(14)
#undef MHLP_FAR_PANEL
                default:
                    far_panel_fp64<SLP, DLP, KQ_NP>(A, fc, x, y, lx, ly, lq, ldx, ldy, l0, accs, accd);
                }
            }
        }
        const int64_t slot = blk - sk_block_of(A.skU, A.skP, tb * Np);
        if (valid) {
            if (SLP) A.skps[slot * A.M + i] = accs;
            if (DLP) A.skpd[slot * A.M + i] = accd;
        }
        u = (tb + 1) * Np;
    }
}

/* Sum of the stream partials of each target (slots of its target block in
   order), near corrections, 1/(2 pi) and the identity term; lanes as in
   far_finalize (L per target). */
template <bool SLP, bool DLP, int L>
__global__ __launch_bounds__(L == 1 ? 256 : FZ_TG * L) void far_sk_finalize(FarArgs A)
{
    constexpr int TG = L == 1 ? 256 : FZ_TG;
    __shared__ double red[4][L == 1 ? 1 : L][L == 1 ? 1 : TG]; /* far S, near S, far D, near D */
    const double *mu;
    if (!far_density(A, mu)) return;
    const int g = threadIdx.x % TG, l = L == 1 ? 0 : threadIdx.x / TG;
    const int64_t i = blockIdx.x * (int64_t)TG + g;
    double fs = 0.0, ns = 0.0, fd = 0.0, nd = 0.0;
    if (i < A.M) {
        const int64_t tb = i / FT_THREADS;
        const int64_t b0 = sk_block_of(A.skU, A.skP, tb * A.Np);
        const int64_t nseg = sk_block_of(A.skU, A.skP, tb * A.Np + A.Np - 1) - b0 + 1;
        for (int64_t q = l; q < nseg; q += L) {
            if (SLP) fs += A.skps[q * A.M + i];
            if (DLP) fd += A.skpd[q * A.M + i];
        }
        for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
            const int64_t p = A.npan[q];
            if (p < 0) continue;
            for (int jj = l; jj < 16; jj += L) {
                if (SLP) ns = fma(A.wsl[16 * (int64_t)q + jj], A.sigma[16 * p + jj], ns);
                if (DLP) nd = fma(A.wdl[16 * (int64_t)q + jj], mu[16 * p + jj], nd);
            }
        }
    }
    if (L > 1) {
        red[0][l][g] = fs;
        red[1][l][g] = ns;
        red[2][l][g] = fd;
        red[3][l][g] = nd;
        __syncthreads();
        if (l != 0) return;
        for (int q = 1; q < L; ++q) {
            fs += red[0][q][g];
            ns += red[1][q][g];
            fd += red[2][q][g];
            nd += red[3][q][g];
        }
    }
    if (i >= A.M) return;
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
    if (SLP) A.us[o] = fma(INV_2PI, fs, ns);
    if (DLP) {
        double v = fma(INV_2PI, fd, nd);
        if (A.half_term != 0.0) v = fma(A.half_term, mu[i], v);
        A.ud[o] = v;
    }
}

/* Plan time: the fine piece of every (wave of 64 targets, panel) for the FP64
   far field (low 7 bits: piece + 1, 0 for z <= 2 everywhere, KQ_NP + 1 when
   the pairs need the per-pair selection; bit 7 set when some target of the
   wave lists the panel as near), from the exact extreme distances of the
   wave's targets to the panel's nodes; targets that list the panel do not vote
   (they skip it).  Lanes past the last target repeat it. */
__global__ __launch_bounds__(256) void far_class_kernel(const double *__restrict__ tx, const double *__restrict__ ty,
                                                        int64_t M, const double *__restrict__ sx,
                                                        const double *__restrict__ sy, int64_t Np, double alpha,
                                                        const int32_t *__restrict__ nptr,
                                                        const int32_t *__restrict__ npan, uint8_t *__restrict__ cls)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t iv = i < M ? i : M - 1;
    const int64_t w = i >> 6;
    const double x = tx[iv], y = ty[iv];
    int32_t k = nptr[iv];
    const int32_t kend = nptr[iv + 1];
    while (k < kend && npan[k] < 0) ++k;
    for (int64_t p = 0; p < Np; ++p) {
        double r2lo = 1e300, r2hi = 0.0;
        for (int j = 0; j < 16; ++j) {
            const double ex = x - sx[16 * p + j], ey = y - sy[16 * p + j];
            const double r2 = fma(ex, ex, ey * ey);
            r2lo = fmin(r2lo, r2);
            r2hi = fmax(r2hi, r2);
        }
        bool listed = false;
        if (k < kend && npan[k] == p) {
            listed = true;
            ++k;
        }
        const double zlo = alpha * sqrt(r2lo), zhi = alpha * sqrt(r2hi);
        int kl = 0, kh = 0;
        for (int b = 0; b < KQ_NB; ++b) {
            kl += zlo > KQ_B[b] ? 1 : 0;
            kh += zhi > KQ_B[b] ? 1 : 0;
        }
        /* the voting lanes' extreme piece indices */
        int lo = listed ? KQ_NB + 1 : kl, hi = listed ? -1 : kh;
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        int c = KQ_NP + 1;
        if (hi < 0)
            c = KQ_NP + 1; /* every target skips the panel */
        else if (lo == hi)
            c = lo; /* piece lo - 1 (0: z <= 2) */
        else if (lo >= 1 && hi == lo + 1 && lo <= KQ_NB - 1)
            c = KQ_NB + lo; /* pieces lo - 1 and lo */
        if (__ballot(listed) != 0) c |= 0x80;
        if ((threadIdx.x & 63) == 0) cls[w * Np + p] = (uint8_t)c;
    }
}

/* ------------------------------------------------------------------------ */
/* far field, mixed precision: FP32 kernel values and products, differences  */
/* x - y formed exactly in FP64 then rounded, FP32 partial sums over each     */
/* 16-node panel accumulated in FP64; corrections and identity term in FP64. */
/* ------------------------------------------------------------------------ */
/* the classes -1 .. KQ_NP - 1 of the plan's (wave, panel) table, for a switch */
#define MHLP_PC_CASES(X) X(-1) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
static_assert(KQ_NP == 15, "MHLP_PC_CASES lists the fine pieces");

/* the 16 sources of one LDS panel (offset l0) against the lane's target in
   FP32, in piece PC of the plan's class table (k01_fp32_pc) */
template <bool SLP, bool DLP, int PC>
__device__ __forceinline__ void mixed_panel(double x, double y, const double *lx, const double *ly, const float *lq,
                                            const float *ldx, const float *ldy, int l0, float alpha, float a2q,
                                            float a4, float &ps, float &pd)
{
#pragma unroll 4
    for (int s = 0; s < 16; ++s) {
        const int l = l0 + s;
        const float ex = (float)(x - lx[l]), ey = (float)(y - ly[l]);
        const float r2 = fmaf(ex, ex, ey * ey);
        const K01f o = k01_fp32_pc<SLP, DLP, PC>(r2, alpha, a2q, a4);
        if (SLP) ps = fmaf(o.k0, lq[l], ps);
        if (DLP) pd = fmaf(o.ak1r, fmaf(ex, ldx[l], ey * ldy[l]), pd);
    }
}

template <bool SLP, bool DLP, bool SPLIT>
__global__ __launch_bounds__(FT_THREADS) void far_eval_mixed(FarArgs A)
{
    __shared__ double lx[FT_SRC], ly[FT_SRC];
    __shared__ float lq[FT_SRC], ldx[FT_SRC], ldy[FT_SRC];
    const double *mu;
    if (!far_density(A, mu)) return;
    const int64_t i = blockIdx.x * (int64_t)FT_THREADS + threadIdx.x;
    const bool valid = i < A.M;
    const double x = valid ? A.tx[i] : 0.0, y = valid ? A.ty[i] : 0.0;
    const int64_t pb = SPLIT ? (int64_t)blockIdx.y * A.pps : 0;
    const int64_t pe = SPLIT ? min(A.Np, pb + A.pps) : A.Np;
    int32_t k = 0, kend = 0;
    if (valid) {
        k = A.nptr[i];
        kend = A.nptr[i + 1];
        while (k < kend && A.npan[k] >= 0 && A.npan[k] < pb) ++k;
    }
    int32_t nxt = (k < kend) ? A.npan[k] : INT_MAX;
    const float alpha = (float)A.alpha, a2q = 0.25f * alpha * alpha, a4 = 4.0f / alpha;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *cls = A.wcls ? A.wcls + ((int64_t)blockIdx.x * (FT_THREADS / 64) + wv) * A.Np : nullptr;
    double accs = 0.0, accd = 0.0;
    for (int64_t base = 16 * pb; base < 16 * pe; base += FT_SRC) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (j < 16 * pe) {
            const double wj = A.sw[j];
            lx[threadIdx.x] = A.sx[j];
            ly[threadIdx.x] = A.sy[j];
            if (SLP) lq[threadIdx.x] = (float)(wj * A.sigma[j]);
            if (DLP) {
                const double m = wj * mu[j];
                ldx[threadIdx.x] = (float)(m * A.snx[j]);
                ldy[threadIdx.x] = (float)(m * A.sny[j]);
            }
        }
        __syncthreads();
        const int32_t p0 = (int32_t)(base / 16);
        const int npl = (pe - p0) < 16 ? (int)(pe - p0) : 16;
        for (int pl = 0; pl < npl; ++pl) {
            if (p0 + pl == nxt) {
                ++k;
                nxt = (k < kend) ? A.npan[k] : INT_MAX;
                continue;
            }
            float ps = 0.0f, pd = 0.0f;
            const int pc = cls ? (cls[p0 + pl] & 0x7f) - 1 : KQ_NP;
            switch (pc) {
#define MHLP_MIXED_PANEL(PCV)                                                                              \
    case PCV:                                                                                              \
        mixed_panel<SLP, DLP, PCV>(x, y, lx, ly, lq, ldx, ldy, pl * 16, alpha, a2q, a4, ps, pd);           \
        break;
                MHLP_PC_CASES(MHLP_MIXED_PANEL)
#undef MHLP_MIXED_PANEL
            default:
                mixed_panel<SLP, DLP, KQ_NP>(x, y, lx, ly, lq, ldx, ldy, pl * 16, alpha, a2q, a4, ps, pd);
            }
            if (SLP) accs += (double)ps;
            if (DLP) accd += (double)pd;
        }
    }
    if (!valid) return;
    if (SPLIT) {
        if (SLP) A.part_s[blockIdx.y * A.M + i] = accs;
        if (DLP) A.part_d[blockIdx.y * A.M + i] = accd;
    } else {
        far_epilogue<SLP, DLP>(A, mu, i, accs, accd);
    }
}

/* ------------------------------------------------------------------------ */
/* volume sum over a tensor grid (all pairs) with the self-cell correction   */
/*   u_i = sum_{j != i} K0(alpha r_ij)/(2 pi) w_j f_j + (w_i/h^2) Wcell f_i    */
/* Sources are targets; the self pair (r == 0) is skipped in the sum.        */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* target gradients of the layer potentials, FP64 (off-surface plans)        */
/*   grad S:  -(1/2pi) sum_j alpha K1(alpha r)/r (x - y_j) w_j sigma_j        */
/*   grad D:  (1/2pi) sum_j [A n_j - ((x - y_j).n_j)(x - y_j)(alpha^2 K0 + 2A)/r^2] w_j mu_j, */
/*            A = alpha K1(alpha r)/r                                          */
/* with the listed near panels replaced by their gradient correction weights. */
/* ------------------------------------------------------------------------ */
struct GradArgs {
    const double *sx, *sy, *sw, *snx, *sny;
    const double *sigma, *mu;
    const double *tx, *ty;
    int64_t M, Np, nnz;
    const int32_t *nptr, *npan, *perm;
    const double *wg;  /* [4][nnz][16] */
    double alpha;
    int32_t pps;
    double *part;      /* [4][nsplit][M] when split */
    double *out[4];    /* d/dx1 S, d/dx2 S, d/dx1 D, d/dx2 D (caller order) */
    const uint8_t *wcls = nullptr; /* the plan's (wave, panel) fine-piece classes, if any */
    const double *fq = nullptr;    /* the fine pieces' scales at the plan's alpha */
};

template <bool GS, bool GD>
__device__ __forceinline__ void grad_epilogue(const GradArgs &A, int64_t i, const double *acc)
{
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
        const int64_t p = A.npan[q];
        if (p < 0) continue;
        for (int jj = 0; jj < 16; ++jj) {
            const int64_t o = 16 * (int64_t)q + jj;
            if (GS) {
                const double sg = A.sigma[16 * p + jj];
                c[0] = fma(A.wg[o], sg, c[0]);
                c[1] = fma(A.wg[A.nnz * 16 + o], sg, c[1]);
            }
            if (GD) {
                const double m = A.mu[16 * p + jj];
                c[2] = fma(A.wg[2 * A.nnz * 16 + o], m, c[2]);
                c[3] = fma(A.wg[3 * A.nnz * 16 + o], m, c[3]);
            }
        }
    }
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
    if (GS) {
        A.out[0][o] = fma(-INV_2PI, acc[0], c[0]);
        A.out[1][o] = fma(-INV_2PI, acc[1], c[1]);
    }
    if (GD) {
        A.out[2][o] = fma(INV_2PI, acc[2], c[2]);
        A.out[3][o] = fma(INV_2PI, acc[3], c[3]);
    }
}

template <bool GS, bool GD>
__global__ void grad_finalize(GradArgs A, int nsplit)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.M) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nsplit; ++k)
        for (int b = 0; b < 4; ++b)
            if ((b < 2 && GS) || (b >= 2 && GD)) acc[b] += A.part[((int64_t)b * nsplit + k) * A.M + i];
    grad_epilogue<GS, GD>(A, i, acc);
}

/* the 16 sources of one LDS panel (offset l0) against the lane's target for
   the gradients: PC the fine piece of the plan's class table (-1: z <= 2;
   KQ_NP: per-pair selection over the three-piece fits) */
template <bool GS, bool GD, int PC>
__device__ __forceinline__ void grad_panel_fp64(const GradArgs &A, const FarConst &fc, double x, double y,
                                                const double *lx, const double *ly, const double *lq,
                                                const double *ldx, const double *ldy, int l0, double &sx,
                                                double &sy, double &dx, double &dy)
{
    constexpr int K = PC < 0 || PC >= KQ_NP ? 0 : PC;
    const FarTab T = far_table();
    double qa, qk;
    fine_q<K>(A.fq, qa, qk);
#pragma unroll 1
    for (int s = 0; s < 16; s += 2) {
        const int l0s = l0 + s, l1 = l0s + 1;
        const double ex0 = x - lx[l0s], ey0 = y - ly[l0s];
        const double ex1 = x - lx[l1], ey1 = y - ly[l1];
        const double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
        K01 o0, o1; /* ak1r holds K1(z)/r; the staged densities carry alpha */
        if constexpr (PC >= KQ_NP)
            k01_far2<GD, true, true, true>(T, fc, r20, r21, o0, o1);
        else
            k01_far2_fixed<GD, true, PC>(T, fc, qa, qk, r20, r21, o0, o1);
        if (GS) {
            const double c0 = o0.ak1r * lq[l0s], c1 = o1.ak1r * lq[l1];
            sx = fma(c1, ex1, fma(c0, ex0, sx));
            sy = fma(c1, ey1, fma(c0, ey0, sy));
        }
        if (GD) {
            /* (alpha^2 K0 + 2 alpha K1/r) (x-y).d / r^2, alpha from the dipole */
            const double n0 = fma(ex0, ldx[l0s], ey0 * ldy[l0s]), n1 = fma(ex1, ldx[l1], ey1 * ldy[l1]);
            const double b0 = n0 * fma(A.alpha, o0.k0, 2.0 * o0.ak1r) * o0.ri2;
            const double b1 = n1 * fma(A.alpha, o1.k0, 2.0 * o1.ak1r) * o1.ri2;
            dx = fma(-b1, ex1, fma(o1.ak1r, ldx[l1], fma(-b0, ex0, fma(o0.ak1r, ldx[l0s], dx))));
            dy = fma(-b1, ey1, fma(o1.ak1r, ldy[l1], fma(-b0, ey0, fma(o0.ak1r, ldy[l0s], dy))));
        }
    }
}

/* Each panel takes the fine piece of the plan's (wave, panel) class table, the
   one the fused evaluation uses (targets in the same order, waves of 64);
   lanes past the last target repeat it, as the table assumes. */
template <bool GS, bool GD, bool SPLIT>
__global__ __launch_bounds__(FT_THREADS) void far_grad_fp64(GradArgs A)
{
    __shared__ double lx[FT_SRC], ly[FT_SRC], lq[FT_SRC], ldx[FT_SRC], ldy[FT_SRC];
    const int64_t i = blockIdx.x * (int64_t)FT_THREADS + threadIdx.x;
    const bool valid = i < A.M;
    const int64_t iv = valid ? i : A.M - 1;
    const double x = A.tx[iv], y = A.ty[iv];
    const int64_t pb = SPLIT ? (int64_t)blockIdx.y * A.pps : 0;
    const int64_t pe = SPLIT ? min(A.Np, pb + A.pps) : A.Np;
    int32_t k = A.nptr[iv];
    const int32_t kend = A.nptr[iv + 1];
    while (k < kend && A.npan[k] >= 0 && A.npan[k] < pb) ++k;
    int32_t nxt = (k < kend) ? A.npan[k] : INT_MAX;
    const FarConst fc = far_const(A.alpha);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *cls = A.wcls ? A.wcls + ((int64_t)blockIdx.x * (FT_THREADS / 64) + wv) * A.Np : nullptr;
    double sx = 0.0, sy = 0.0, dx = 0.0, dy = 0.0;
    for (int64_t base = 16 * pb; base < 16 * pe; base += FT_SRC) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (j < 16 * pe) {
            /* alpha goes with the charges and dipoles: the pair evaluates K1(z)/r */
            const double wj = A.alpha * A.sw[j];
            lx[threadIdx.x] = A.sx[j];
            ly[threadIdx.x] = A.sy[j];
            if (GS) lq[threadIdx.x] = wj * A.sigma[j];
            if (GD) {
                const double m = wj * A.mu[j];
                ldx[threadIdx.x] = m * A.snx[j];
                ldy[threadIdx.x] = m * A.sny[j];
            }
        }
        __syncthreads();
        const int32_t p0 = (int32_t)(base / 16);
        const int npl = (pe - p0) < 16 ? (int)(pe - p0) : 16;
        for (int pl = 0; pl < npl; ++pl) {
            if (p0 + pl == nxt) {
                ++k;
                nxt = (k < kend) ? A.npan[k] : INT_MAX;
                continue;
            }
            const int pc = cls ? (cls[p0 + pl] & 0x7f) - 1 : KQ_NP;
            const int l0 = pl * 16;
            switch (pc) {
#define MHLP_GRAD_PANEL(PCV)                                                                              \
    case PCV:                                                                                              \
        grad_panel_fp64<GS, GD, PCV>(A, fc, x, y, lx, ly, lq, ldx, ldy, l0, sx, sy, dx, dy);               \
        break;
                MHLP_GRAD_PANEL(-1)
                MHLP_GRAD_PANEL(0)
                MHLP_GRAD_PANEL(1)
                MHLP_GRAD_PANEL(2)
                MHLP_GRAD_PANEL(3)
                MHLP_GRAD_PANEL(4)
                MHLP_GRAD_PANEL(5)
                MHLP_GRAD_PANEL(6)
                MHLP_GRAD_PANEL(7)
                MHLP_GRAD_PANEL(8)
                MHLP_GRAD_PANEL(9)
                MHLP_GRAD_PANEL(10)
                MHLP_GRAD_PANEL(11)
                MHLP_GRAD_PANEL(12)
                MHLP_GRAD_PANEL(13)
                MHLP_GRAD_PANEL(14)
#undef MHLP_GRAD_PANEL
            default:
                grad_panel_fp64<GS, GD, KQ_NP>(A, fc, x, y, lx, ly, lq, ldx, ldy, l0, sx, sy, dx, dy);
            }
        }
    }
    if (!valid) return;
    const double acc[4] = {sx, sy, dx, dy};
    if (SPLIT) {
        const int ns = gridDim.y;
        for (int b = 0; b < 4; ++b)
            if ((b < 2 && GS) || (b >= 2 && GD)) A.part[((int64_t)b * ns + blockIdx.y) * A.M + i] = acc[b];
    } else {
        grad_epilogue<GS, GD>(A, i, acc);
    }
}

/* ------------------------------------------------------------------------ */
/* modified-Stokes double layer, FP64 (stokes plans)                         */
/*   u_i(x) = sum_j D_ij(x, y_j) w_j mu_j,                                     */
/*   D_ij = -[A1 (n_i r_j + r_i n_j + d_ij r.n) + A2 r_i r_j r.n + A3 r_i n_j], */
/*   r = x - y, A1 = alpha^2 T1, A2 = alpha^4 T2, A3 = alpha^2 T3            */
/* with the listed near panels replaced by their stresslet weights, and on    */
/* on-surface plans (BIE) the 1/2 mu and W mu = n sum_j w_j mu_j.n_j / |Gamma| */
/* terms.  Densities and outputs are [2][N] / [2][M] (component-major).       */
/* ------------------------------------------------------------------------ */
struct StkArgs {
    const double *sx, *sy, *sw, *snx, *sny;
    const double *mu; /* [2][N] (or the GMRES basis, column j at mu + j*jstride) */
    int64_t N;
    const double *tx, *ty;
    int64_t M, Np, nnz;
    const int32_t *nptr, *npan, *perm;
    const double *wst; /* [4][nnz][16] */
    double alpha;
    int32_t pps;
    double *part;      /* [2][nsplit][M] */
    double *u;         /* u1 = u[o], u2 = u[ustride + o] */
    int64_t ustride;
    int32_t bie;
    const double *flux; /* sum_j w_j mu_j.n_j / |Gamma| (bie) */
    const GState *gs;
    int64_t jstride;
    const uint8_t *wcls = nullptr; /* the plan's (wave, panel) fine-piece classes, if any */
    const double *fq = nullptr;    /* the fine pieces' scales at the plan's alpha */
};

__device__ __forceinline__ bool stk_density(const StkArgs &A, const double *&mu)
{
    mu = A.mu;
    if (A.gs) {
        if (A.gs->done) return false;
        mu += (int64_t)A.gs->j * A.jstride;
    }
    return true;
}

__device__ __forceinline__ void stk_epilogue(const StkArgs &A, const double *__restrict__ mu, int64_t i, double a1,
                                             double a2)
{
    for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
        const int64_t p = A.npan[q];
        if (p < 0) continue;
        for (int jj = 0; jj < 16; ++jj) {
            const int64_t o = 16 * (int64_t)q + jj;
            const double m1 = mu[16 * p + jj], m2 = mu[A.N + 16 * p + jj];
            a1 = fma(A.wst[o], m1, fma(A.wst[A.nnz * 16 + o], m2, a1));
            a2 = fma(A.wst[2 * A.nnz * 16 + o], m1, fma(A.wst[3 * A.nnz * 16 + o], m2, a2));
        }
    }
    if (A.bie) {
        const double f = A.flux[0];
        a1 = fma(0.5, mu[i], fma(A.snx[i], f, a1));
        a2 = fma(0.5, mu[A.N + i], fma(A.sny[i], f, a2));
    }
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
    A.u[o] = a1;
    A.u[A.ustride + o] = a2;
}

/* Split partials + the epilogue, laid out as far_finalize: L = FZ_L lanes per
   target (lane l: partials l, l + L, ..., node l of each near panel, lane sums
   added in lane order) for short target lists, one thread per target
   otherwise. */
template <int L>
__global__ __launch_bounds__(L == 1 ? 256 : FZ_TG * L) void stk_finalize(StkArgs A, int nsplit)
{
    if (L == 1) {
        const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
        const double *mu;
        if (i >= A.M || !stk_density(A, mu)) return;
        double a1 = 0.0, a2 = 0.0;
        for (int k = 0; k < nsplit; ++k) {
            a1 += A.part[(int64_t)k * A.M + i];
            a2 += A.part[((int64_t)nsplit + k) * A.M + i];
        }
        stk_epilogue(A, mu, i, a1, a2);
        return;
    }
    __shared__ double red[4][L][FZ_TG]; /* far 1, near 1, far 2, near 2 */
    const double *mu;
    if (!stk_density(A, mu)) return; /* the same for every thread of the launch */
    const int g = threadIdx.x % FZ_TG, l = threadIdx.x / FZ_TG;
    const int64_t i = blockIdx.x * (int64_t)FZ_TG + g;
    double f1 = 0.0, n1 = 0.0, f2 = 0.0, n2 = 0.0;
    if (i < A.M) {
        for (int k = l; k < nsplit; k += L) {
            f1 += A.part[(int64_t)k * A.M + i];
            f2 += A.part[((int64_t)nsplit + k) * A.M + i];
        }
        for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
            const int64_t p = A.npan[q];
            if (p < 0) continue;
            const int64_t o = 16 * (int64_t)q + l;
            const double m1 = mu[16 * p + l], m2 = mu[A.N + 16 * p + l];
            n1 = fma(A.wst[o], m1, fma(A.wst[A.nnz * 16 + o], m2, n1));
            n2 = fma(A.wst[2 * A.nnz * 16 + o], m1, fma(A.wst[3 * A.nnz * 16 + o], m2, n2));
        }
    }
    red[0][l][g] = f1;
    red[1][l][g] = n1;
    red[2][l][g] = f2;
    red[3][l][g] = n2;
    __syncthreads();
    if (l != 0 || i >= A.M) return;
    for (int q = 1; q < L; ++q) {
        f1 += red[0][q][g];
        n1 += red[1][q][g];
        f2 += red[2][q][g];
        n2 += red[3][q][g];
    }
    double a1 = f1 + n1, a2 = f2 + n2;
    if (A.bie) {
        const double f = A.flux[0];
        a1 = fma(0.5, mu[i], fma(A.snx[i], f, a1));
        a2 = fma(0.5, mu[A.N + i], fma(A.sny[i], f, a2));
    }
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
    A.u[o] = a1;
    A.u[A.ustride + o] = a2;
}

/* flux sum_j w_j mu_j.n_j / |Gamma| of the density into flux[0]; one block,
   fixed summation order */
__global__ __launch_bounds__(256) void stk_flux_kernel(StkArgs A, double inv_len, double *__restrict__ flux)
{
    __shared__ double red[256];
    const double *mu;
    if (!stk_density(A, mu)) return;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < A.N; j += 256) s = fma(A.sw[j], fma(mu[j], A.snx[j], mu[A.N + j] * A.sny[j]), s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) flux[0] = red[0] * inv_len;
}

/* the 16 sources of one LDS panel (offset l0) against the lane's target for
   the stresslet double layer, in piece PC of the class table */
template <int PC>
__device__ __forceinline__ void stk_panel_fp64(const double *fq, const FarConst &fc, double al2, double ial2, double x,
                                               double y, const double *lx, const double *ly, const double *lm1,
                                               const double *lm2, const double *lnx, const double *lny, int l0,
                                               double &a1, double &a2)
{
    constexpr int K = PC < 0 || PC >= KQ_NP ? 0 : PC;
    const FarTab T = far_table();
    double qa, qk;
    fine_q<K>(fq, qa, qk);
#pragma unroll 1
    for (int s = 0; s < 16; s += 2) {
        const int l0s = l0 + s;
        const double ex0 = x - lx[l0s], ey0 = y - ly[l0s];
        const double ex1 = x - lx[l0s + 1], ey1 = y - ly[l0s + 1];
        const double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
        double Ak2[2][3];
        stk_far2_pc<PC>(T, fc, qa, qk, al2, ial2, r20, r21, Ak2[0], Ak2[1]);
        const double ex[2] = {ex0, ex1}, ey[2] = {ey0, ey1};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int l = l0s + u;
            const double *Ak = Ak2[u];
            const double nx = lnx[l], ny = lny[l], m1 = lm1[l], m2 = lm2[l];
            const double rn = fma(ex[u], nx, ey[u] * ny);
            const double rm = fma(ex[u], m1, ey[u] * m2);
            const double nm = fma(nx, m1, ny * m2);
            const double c = fma(Ak[1] * rm, rn, Ak[2] * nm);
            a1 -= fma(Ak[0], fma(nx, rm, fma(ex[u], nm, m1 * rn)), c * ex[u]);
            a2 -= fma(Ak[0], fma(ny, rm, fma(ey[u], nm, m2 * rn)), c * ey[u]);
        }
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(FT_THREADS) void far_stokes_fp64(StkArgs A)
{
    __shared__ double lx[FT_SRC], ly[FT_SRC], lm1[FT_SRC], lm2[FT_SRC], lnx[FT_SRC], lny[FT_SRC];
    const double *mu;
    if (!stk_density(A, mu)) return;
    const int64_t i = blockIdx.x * (int64_t)FT_THREADS + threadIdx.x;
    const bool valid = i < A.M;
    const int64_t iv = valid ? i : A.M - 1; /* lanes past the last target repeat it */
    const double x = A.tx[iv], y = A.ty[iv];
    const int64_t pb = SPLIT ? (int64_t)blockIdx.y * A.pps : 0;
    const int64_t pe = SPLIT ? min(A.Np, pb + A.pps) : A.Np;
    int32_t k = A.nptr[iv];
    const int32_t kend = A.nptr[iv + 1];
    while (k < kend && A.npan[k] >= 0 && A.npan[k] < pb) ++k;
    int32_t nxt = (k < kend) ? A.npan[k] : INT_MAX;
    const FarConst fc = far_const(A.alpha);
    const double al2 = A.alpha * A.alpha, ial2 = fc.ia * fc.ia;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *cls = A.wcls ? A.wcls + ((int64_t)blockIdx.x * (FT_THREADS / 64) + wv) * A.Np : nullptr;
    double a1 = 0.0, a2 = 0.0;
    for (int64_t base = 16 * pb; base < 16 * pe; base += FT_SRC) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (j < 16 * pe) {
            const double wj = A.sw[j];
            lx[threadIdx.x] = A.sx[j];
            ly[threadIdx.x] = A.sy[j];
            lm1[threadIdx.x] = wj * mu[j];
            lm2[threadIdx.x] = wj * mu[A.N + j];
            lnx[threadIdx.x] = A.snx[j];
            lny[threadIdx.x] = A.sny[j];
        }
        __syncthreads();
        const int32_t p0 = (int32_t)(base / 16);
        const int npl = (pe - p0) < 16 ? (int)(pe - p0) : 16;
        for (int pl = 0; pl < npl; ++pl) {
            if (p0 + pl == nxt) {
                ++k;
                nxt = (k < kend) ? A.npan[k] : INT_MAX;
                continue;
            }
            const int pc = cls ? (cls[p0 + pl] & 0x7f) - 1 : KQ_NP;
            const int l0 = pl * 16;
            switch (pc) {
#define MHLP_STK_PANEL(PCV)                                                                                \
    case PCV:                                                                                              \
        stk_panel_fp64<PCV>(A.fq, fc, al2, ial2, x, y, lx, ly, lm1, lm2, lnx, lny, l0, a1, a2);           \
        break;
                MHLP_PC_CASES(MHLP_STK_PANEL)
#undef MHLP_STK_PANEL
            default:
                stk_panel_fp64<KQ_NP>(A.fq, fc, al2, ial2, x, y, lx, ly, lm1, lm2, lnx, lny, l0, a1, a2);
            }
        }
    }
    if (!valid) return;
    if (SPLIT) {
        const int ns = gridDim.y;
        A.part[(int64_t)blockIdx.y * A.M + i] = a1;
        A.part[((int64_t)ns + blockIdx.y) * A.M + i] = a2;
    } else {
        stk_epilogue(A, mu, i, a1, a2);
    }
}

/* ------------------------------------------------------------------------ */
/* target gradient of the modified-Stokes double layer, FP64 (off-surface    */
/* stokes plans):  d u_i/d x_l = sum_j d_l D_ij(x, y_j) w_j mu_j with        */
/*   d_l D_ij m_j = -[ r_l Pm_i + n_l (A1 m_i + A2 (r.m) r_i)                  */
/*                     + m_l (A1 n_i + A2 (r.n) r_i)                           */
/*                     + d_il ((A1 + A3)(n.m) + A2 (r.n)(r.m)) ],              */
/*   Pm_i = B1 (n_i (r.m) + m_i (r.n)) + r_i (B2 (r.n)(r.m) + (B1 + B3)(n.m)), */
/* B_k = A_k'(r)/r, and the listed near panels replaced by their weights.    */
/* Outputs g[c][M], c = 2i + l.                                               */
/* ------------------------------------------------------------------------ */
struct StkGArgs {
    const double *sx, *sy, *sw, *snx, *sny;
    const double *mu; /* [2][N] */
    int64_t N;
    const double *tx, *ty;
    int64_t M, Np, nnz;
    const int32_t *nptr, *npan, *perm;
    const double *wg; /* [8][nnz][16] */
    double alpha;
    int32_t pps;
    double *part;     /* [4][nsplit][M] */
    double *g;        /* [4][M] */
    const uint8_t *wcls = nullptr; /* the plan's (wave, panel) fine-piece classes, if any */
    const double *fq = nullptr;    /* the fine pieces' scales at the plan's alpha */
};

__device__ __forceinline__ void stkg_epilogue(const StkGArgs &A, int64_t i, const double *acc)
{
    double c[4] = {acc[0], acc[1], acc[2], acc[3]};
    const int64_t bs = A.nnz * 16;
    for (int32_t q = A.nptr[i]; q < A.nptr[i + 1]; ++q) {
        const int64_t p = A.npan[q];
        if (p < 0) continue;
        for (int jj = 0; jj < 16; ++jj) {
            const int64_t o = 16 * (int64_t)q + jj;
            const double m1 = A.mu[16 * p + jj], m2 = A.mu[A.N + 16 * p + jj];
#pragma unroll
            for (int b = 0; b < 4; ++b) c[b] = fma(A.wg[(2 * b) * bs + o], m1, fma(A.wg[(2 * b + 1) * bs + o], m2, c[b]));
        }
    }
    const int64_t o = A.perm ? (int64_t)A.perm[i] : i;
#pragma unroll
    for (int b = 0; b < 4; ++b) A.g[b * A.M + o] = c[b];
}

__global__ void stkg_finalize(StkGArgs A, int nsplit)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.M) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nsplit; ++k)
        for (int b = 0; b < 4; ++b) acc[b] += A.part[((int64_t)b * nsplit + k) * A.M + i];
    stkg_epilogue(A, i, acc);
}

/* ---- on-surface stresslet double layer, each unordered far pair once ----
   The far term of source j at node i is -F(e; n_j, m_j), e = x_i - x_j, m = w mu,
   F(e; n, m) = A1 (n (e.m) + e (n.m) + m (e.n)) + (A2 (e.m)(e.n) + A3 (n.m)) e
   with A1, A2, A3 = alpha^2 T1, alpha^4 T2, alpha^2 T3 of |e| (App. B), the
   contraction of far_stokes_fp64.  F is odd in e, so one evaluation of the A_k
   serves both terms of the pair: source j at node i and +F(e; n_i, m_i) for
   source i at node j.  Tiles, near bit set and order rules as sym_far_kernel;
   the column terms of a tile are summed over each row of 16 lanes by DPP
   moves, then the 16 row sums of a column in order through LDS. */
struct StkSymArgs {
    StkArgs A;
    const int2 *tiles;
    double *p1, *p2; /* [column panel][2][N], [row block][2][N] */
    const uint32_t *bits;
    int nw;
};

/* inclusive sums within each row of 16 lanes: lane 15 of a row holds its sum */
__device__ __forceinline__ double row16_sum_dpp(double v)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) v = dpp_add(v, k);
    return v;
}

__global__ __launch_bounds__(SYM_R) void stk_sym_kernel(StkSymArgs S)
{
    const StkArgs &A = S.A;
    __shared__ double cx[SYM_C], cy[SYM_C], cnx[SYM_C], cny[SYM_C], cm1[SYM_C], cm2[SYM_C], cnm[SYM_C];
    __shared__ uint32_t cmask[SYM_C];
    __shared__ double colv[2][SYM_C][SYM_R / 16];
    const double *mu;
    if (!stk_density(A, mu)) return; /* the same for the whole launch */
    const int2 tl = S.tiles[blockIdx.x];
    const int I = tl.x, J = tl.y, t = threadIdx.x;
    const int64_t N = A.N, i = (int64_t)I * SYM_R + t, j0 = (int64_t)J * SYM_C;
    const int pb = SYM_RP * I; /* first panel of the row block */
    if (t < SYM_C) {
        const int64_t j = j0 + t;
        double xj = 0.0, yj = 0.0, nxj = 0.0, nyj = 0.0, m1 = 0.0, m2 = 0.0;
        uint32_t msk = 0;
        if (j < N) {
            xj = A.sx[j];
            yj = A.sy[j];
            nxj = A.snx[j];
            nyj = A.sny[j];
            const double wj = A.sw[j];
            m1 = wj * mu[j];
            m2 = wj * mu[N + j];
            msk = (S.bits[j * S.nw + (pb >> 5)] >> (pb & 31)) & 0xFFFFu; /* the block's 16 panels */
        }
        cx[t] = xj;
        cy[t] = yj;
        cnx[t] = nxj;
        cny[t] = nyj;
        cm1[t] = m1;
        cm2[t] = m2;
        cnm[t] = fma(nxj, m1, nyj * m2);
        cmask[t] = msk;
    }
    const bool valid = i < N;
    double x = 0.0, y = 0.0, nxi = 0.0, nyi = 0.0, mi1 = 0.0, mi2 = 0.0;
    uint32_t rnear = 0; /* bit 0: column panel J listed near row i */
    int kp = 0;         /* row panel within the block */
    if (valid) {
        x = A.sx[i];
        y = A.sy[i];
        nxi = A.snx[i];
        nyi = A.sny[i];
        const double wi = A.sw[i];
        mi1 = wi * mu[i];
        mi2 = wi * mu[N + i];
        kp = (int)(i / 16) - pb;
        rnear = (S.bits[i * S.nw + (J >> 5)] >> (J & 31)) & 1u;
    }
    const double nmi = fma(nxi, mi1, nyi * mi2);
    const bool diag = SYM_CP * J < pb + SYM_RP; /* the chunk lies in the row block */
    const bool rfar = valid && !(rnear & 1u);
    __syncthreads();
    const FarConst fc = far_const(A.alpha);
    const double al2 = A.alpha * A.alpha, ial2 = fc.ia * fc.ia;
    const int ncol = (int)min((int64_t)SYM_C, N - j0);
    const int slot = t >> 4; /* row of 16 lanes: 4 per wave */
    double a1 = 0.0, a2 = 0.0;
#pragma unroll 1
    for (int s = 0; s < ncol; s += 2) {
        const FarTab T = far_table();
        double ex[2], ey[2], r2[2];
        bool rw[2], cl[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = s + u;
            const bool order = !diag || i < j0 + c; /* on the diagonal block only row < column */
            ex[u] = x - cx[c];
            ey[u] = y - cy[c];
            rw[u] = rfar && order;
            cl[u] = valid && order && !((cmask[c] >> kp) & 1u);
            const double d2 = fma(ex[u], ex[u], ey[u] * ey[u]);
            r2[u] = (rw[u] || cl[u]) ? d2 : 1.0; /* unused pairs (the node itself among them) */
        }
        double Ak[2][3];
        stk_far2(T, fc, al2, ial2, r2[0], r2[1], Ak[0], Ak[1]);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = s + u;
            const double *K = Ak[u];
            if (rw[u]) {
                const double rn = fma(ex[u], cnx[c], ey[u] * cny[c]), rm = fma(ex[u], cm1[c], ey[u] * cm2[c]);
                const double nm = cnm[c], cf = fma(K[1] * rm, rn, K[2] * nm);
                a1 -= fma(K[0], fma(cnx[c], rm, fma(ex[u], nm, cm1[c] * rn)), cf * ex[u]);
                a2 -= fma(K[0], fma(cny[c], rm, fma(ey[u], nm, cm2[c] * rn)), cf * ey[u]);
            }
            double v1 = 0.0, v2 = 0.0;
            if (cl[u]) {
                const double rn = fma(ex[u], nxi, ey[u] * nyi), rm = fma(ex[u], mi1, ey[u] * mi2);
                const double cf = fma(K[1] * rm, rn, K[2] * nmi);
                v1 = fma(K[0], fma(nxi, rm, fma(ex[u], nmi, mi1 * rn)), cf * ex[u]);
                v2 = fma(K[0], fma(nyi, rm, fma(ey[u], nmi, mi2 * rn)), cf * ey[u]);
            }
            v1 = row16_sum_dpp(v1);
            v2 = row16_sum_dpp(v2);
            if ((t & 15) == 15) {
                colv[0][c][slot] = v1;
                colv[1][c][slot] = v2;
            }
        }
    }
    __syncthreads();
    if (t < 2 * SYM_C) {
        const int comp = t / SYM_C, c = t % SYM_C;
        if (c < ncol) {
            double sc = 0.0;
            for (int r = 0; r < SYM_R / 16; ++r) sc += colv[comp][c][r];
            S.p2[((int64_t)I * 2 + comp) * N + j0 + c] = sc;
        }
    }
    if (valid) {
        S.p1[(int64_t)J * 2 * N + i] = a1;
        S.p1[((int64_t)J * 2 + 1) * N + i] = a2;
    }
}

/* node n: both components of the row sums of the chunks from its block on and
   of the column sums of the blocks up to its own, the near corrections, and
   on the BIE operator the flux term and mu/2; FZ_L lanes per node, FZ_TG
   nodes per block, lane sums added in lane order. */
__global__ __launch_bounds__(FZ_TG *FZ_L) void stk_sym_finalize(StkSymArgs S, int nchunk)
{
    const StkArgs &A = S.A;
    __shared__ double red[4][FZ_L][FZ_TG]; /* far 1, near 1, far 2, near 2 */
    const double *mu;
    if (!stk_density(A, mu)) return; /* the same for every thread of the launch */
    const int g = threadIdx.x % FZ_TG, l = threadIdx.x / FZ_TG;
    const int64_t N = A.N, n = blockIdx.x * (int64_t)FZ_TG + g;
    double f1 = 0.0, n1 = 0.0, f2 = 0.0, n2 = 0.0;
    if (n < N) {
        const int B = (int)(n / SYM_R);
        for (int c = SYM_RP * B / SYM_CP + l; c < nchunk; c += FZ_L) {
            f1 += S.p1[(int64_t)c * 2 * N + n];
            f2 += S.p1[((int64_t)c * 2 + 1) * N + n];
        }
        for (int b = l; b <= B; b += FZ_L) {
            f1 += S.p2[(int64_t)b * 2 * N + n];
            f2 += S.p2[((int64_t)b * 2 + 1) * N + n];
        }
        for (int32_t q = A.nptr[n]; q < A.nptr[n + 1]; ++q) {
            const int64_t p = A.npan[q];
            if (p < 0) continue;
            const int64_t o = 16 * (int64_t)q + l;
            const double m1 = mu[16 * p + l], m2 = mu[N + 16 * p + l];
            n1 = fma(A.wst[o], m1, fma(A.wst[A.nnz * 16 + o], m2, n1));
            n2 = fma(A.wst[2 * A.nnz * 16 + o], m1, fma(A.wst[3 * A.nnz * 16 + o], m2, n2));
        }
    }
    red[0][l][g] = f1;
    red[1][l][g] = n1;
    red[2][l][g] = f2;
    red[3][l][g] = n2;
    __syncthreads();
    if (l != 0 || n >= N) return;
    for (int q = 1; q < FZ_L; ++q) {
        f1 += red[0][q][g];
        n1 += red[1][q][g];
        f2 += red[2][q][g];
        n2 += red[3][q][g];
    }
    double a1 = f1 + n1, a2 = f2 + n2;
    if (A.bie) {
        const double f = A.flux[0];
        a1 = fma(0.5, mu[n], fma(A.snx[n], f, a1));
        a2 = fma(0.5, mu[N + n], fma(A.sny[n], f, a2));
    }
    const int64_t o = A.perm ? (int64_t)A.perm[n] : n;
    A.u[o] = a1;
    A.u[A.ustride + o] = a2;
}

/* the 16 sources of one LDS panel (offset l0) against the lane's target for
   the stresslet target gradient, in piece PC of the class table; g: the
   lane's four accumulators */
template <int PC>
__device__ __forceinline__ void stkg_panel_fp64(const double *fq, const FarConst &fc, double al2, double ial2, double x,
                                                double y, const double *lx, const double *ly, const double *lm1,
                                                const double *lm2, const double *lnx, const double *lny, int l0,
                                                double *g)
{
    constexpr int K = PC < 0 || PC >= KQ_NP ? 0 : PC;
    const FarTab T = far_table();
    double qa, qk;
    fine_q<K>(fq, qa, qk);
#pragma unroll 1
    for (int s = 0; s < 16; s += 2) {
        const int l0s = l0 + s;
        const double ex0 = x - lx[l0s], ey0 = y - ly[l0s];
        const double ex1 = x - lx[l0s + 1], ey1 = y - ly[l0s + 1];
        const double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
        double Ak[2][3], Bk[2][3];
        stk_far2_ab_pc<PC>(T, fc, qa, qk, al2, ial2, r20, r21, Ak[0], Bk[0], Ak[1], Bk[1]);
        const double ex[2] = {ex0, ex1}, ey[2] = {ey0, ey1};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int l = l0s + u;
            const double *a = Ak[u], *b = Bk[u];
            const double nx = lnx[l], ny = lny[l], m1 = lm1[l], m2 = lm2[l];
            const double rn = fma(ex[u], nx, ey[u] * ny);
            const double rm = fma(ex[u], m1, ey[u] * m2);
            const double nm = fma(nx, m1, ny * m2);
            const double sr = fma(b[1] * rn, rm, (b[0] + b[2]) * nm);
            const double p1 = fma(b[0], fma(nx, rm, m1 * rn), ex[u] * sr);
            const double p2 = fma(b[0], fma(ny, rm, m2 * rn), ey[u] * sr);
            const double a1 = fma(a[0], m1, a[1] * rm * ex[u]), a2 = fma(a[0], m2, a[1] * rm * ey[u]);
            const double c1 = fma(a[0], nx, a[1] * rn * ex[u]), c2 = fma(a[0], ny, a[1] * rn * ey[u]);
            const double d = fma(a[0] + a[2], nm, a[1] * rn * rm);
            g[0] -= fma(ex[u], p1, fma(nx, a1, fma(m1, c1, d)));
            g[1] -= fma(ey[u], p1, fma(ny, a1, m2 * c1));
            g[2] -= fma(ex[u], p2, fma(nx, a2, m1 * c2));
            g[3] -= fma(ey[u], p2, fma(ny, a2, fma(m2, c2, d)));
        }
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(FT_THREADS) void far_stokes_grad_fp64(StkGArgs A)
{
    __shared__ double lx[FT_SRC], ly[FT_SRC], lm1[FT_SRC], lm2[FT_SRC], lnx[FT_SRC], lny[FT_SRC];
    const int64_t i = blockIdx.x * (int64_t)FT_THREADS + threadIdx.x;
    const bool valid = i < A.M;
    const int64_t iv = valid ? i : A.M - 1; /* lanes past the last target repeat it */
    const double x = A.tx[iv], y = A.ty[iv];
    const int64_t pb = SPLIT ? (int64_t)blockIdx.y * A.pps : 0;
    const int64_t pe = SPLIT ? min(A.Np, pb + A.pps) : A.Np;
    int32_t k = A.nptr[iv];
    const int32_t kend = A.nptr[iv + 1];
    while (k < kend && A.npan[k] >= 0 && A.npan[k] < pb) ++k;
    int32_t nxt = (k < kend) ? A.npan[k] : INT_MAX;
    const FarConst fc = far_const(A.alpha);
    const double al2 = A.alpha * A.alpha, ial2 = fc.ia * fc.ia;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *cls = A.wcls ? A.wcls + ((int64_t)blockIdx.x * (FT_THREADS / 64) + wv) * A.Np : nullptr;
    double g11 = 0.0, g12 = 0.0, g21 = 0.0, g22 = 0.0;
    for (int64_t base = 16 * pb; base < 16 * pe; base += FT_SRC) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (j < 16 * pe) {
            const double wj = A.sw[j];
            lx[threadIdx.x] = A.sx[j];
            ly[threadIdx.x] = A.sy[j];
            lm1[threadIdx.x] = wj * A.mu[j];
            lm2[threadIdx.x] = wj * A.mu[A.N + j];
            lnx[threadIdx.x] = A.snx[j];
            lny[threadIdx.x] = A.sny[j];
        }
        __syncthreads();
        const int32_t p0 = (int32_t)(base / 16);
        const int npl = (pe - p0) < 16 ? (int)(pe - p0) : 16;
        for (int pl = 0; pl < npl; ++pl) {
            if (p0 + pl == nxt) {
                ++k;
                nxt = (k < kend) ? A.npan[k] : INT_MAX;
                continue;
            }
            const int pc = cls ? (cls[p0 + pl] & 0x7f) - 1 : KQ_NP;
            const int l0 = pl * 16;
            double gg[4] = {g11, g12, g21, g22};
            switch (pc) {
#define MHLP_STKG_PANEL(PCV)                                                                               \
    case PCV:                                                                                              \
        stkg_panel_fp64<PCV>(A.fq, fc, al2, ial2, x, y, lx, ly, lm1, lm2, lnx, lny, l0, gg);              \
        break;
                MHLP_PC_CASES(MHLP_STKG_PANEL)
#undef MHLP_STKG_PANEL
            default:
                stkg_panel_fp64<KQ_NP>(A.fq, fc, al2, ial2, x, y, lx, ly, lm1, lm2, lnx, lny, l0, gg);
            }
            g11 = gg[0];
            g12 = gg[1];
            g21 = gg[2];
            g22 = gg[3];
        }
    }
    if (!valid) return;
    const double acc[4] = {g11, g12, g21, g22};
    if (SPLIT) {
        const int ns = gridDim.y;
        for (int b = 0; b < 4; ++b) A.part[((int64_t)b * ns + blockIdx.y) * A.M + i] = acc[b];
    } else {
        stkg_epilogue(A, i, acc);
    }
}

struct VolArgs {
    const double *x, *y, *w, *f;
    int64_t n;
    double alpha;
    double selfc;   /* Wcell / h^2 */
    int64_t per_split;
    double *part;   /* [nsplit][n] */
    double *u;
    const double *selfc_dev; /* when set, Wcell / h^2 is read here instead of selfc */
};

template <bool MIXED, bool SPLIT>
__global__ __launch_bounds__(FT_THREADS) void volume_kernel(VolArgs A)
{
    __shared__ double lx[FT_SRC], ly[FT_SRC];
    __shared__ double lq[FT_SRC];
    const int64_t i = blockIdx.x * (int64_t)FT_THREADS + threadIdx.x;
    const bool valid = i < A.n;
    const double x = valid ? A.x[i] : 0.0, y = valid ? A.y[i] : 0.0;
    const int64_t jb = SPLIT ? (int64_t)blockIdx.y * A.per_split : 0;
    const int64_t je = SPLIT ? min(A.n, jb + A.per_split) : A.n;
    const FarConst fc = far_const(A.alpha);
    const float af = (float)A.alpha, a2qf = 0.25f * af * af, a4f = 4.0f / af;
    double acc = 0.0;
    for (int64_t base = jb; base < je; base += FT_SRC) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (j < je) {
            lx[threadIdx.x] = A.x[j];
            ly[threadIdx.x] = A.y[j];
            lq[threadIdx.x] = A.w[j] * A.f[j];
        } else {
            lx[threadIdx.x] = 0.0;
            ly[threadIdx.x] = 0.0;
            lq[threadIdx.x] = 0.0;
        }
        __syncthreads();
        const int cnt = (je - base) < FT_SRC ? (int)(je - base) : FT_SRC;
        if (MIXED) {
            float ps = 0.0f;
            for (int l = 0; l < cnt; ++l) {
                const float ex = (float)(x - lx[l]), ey = (float)(y - ly[l]);
                float r2 = fmaf(ex, ex, ey * ey);
                const bool self = r2 == 0.0f;
                r2 = self ? 1.0f : r2;
                const K01f o = k01_fp32<true, false>(r2, af, a2qf, a4f);
                ps = fmaf(self ? 0.0f : o.k0, (float)lq[l], ps);
                if ((l & 15) == 15) {
                    acc += (double)ps;
                    ps = 0.0f;
                }
            }
            acc += (double)ps;
        } else {
            /* pairs of sources; an odd count reads one zero-padded slot (lq = 0) */
#pragma unroll 1
            for (int l = 0; l < cnt; l += 2) {
                const FarTab T = far_table();
                const double ex0 = x - lx[l], ey0 = y - ly[l];
                const double ex1 = x - lx[l + 1], ey1 = y - ly[l + 1];
                double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
                const bool self0 = r20 == 0.0, self1 = r21 == 0.0;
                r20 = self0 ? 1.0 : r20;
                r21 = self1 ? 1.0 : r21;
                K01 o0, o1;
                k01_far2<true, false, false>(T, fc, r20, r21, o0, o1);
                acc = fma(self1 ? 0.0 : o1.k0, lq[l + 1], fma(self0 ? 0.0 : o0.k0, lq[l], acc));
            }
        }
    }
    if (!valid) return;
    if (SPLIT)
        A.part[blockIdx.y * A.n + i] = acc;
    else
        A.u[i] = fma(INV_2PI, acc, (A.selfc_dev ? A.selfc_dev[0] : A.selfc) * A.w[i] * A.f[i]);
}

__global__ void volume_finalize(VolArgs A, int nsplit)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    double s_ = 0.0;
    for (int k = 0; k < nsplit; ++k) s_ += A.part[k * A.n + i];
    A.u[i] = fma(INV_2PI, s_, (A.selfc_dev ? A.selfc_dev[0] : A.selfc) * A.w[i] * A.f[i]);
}

/* Integral of K0(alpha |x|)/(2 pi) over the h x h cell centred at the origin:
   (1/2pi) 8 int_0^{pi/4} (1 - a K1(a))/alpha^2 dtheta, a = alpha h/(2 cos theta)
   (from int_0^R K0(alpha s) s ds = (1 - alpha R K1(alpha R))/alpha^2);
   composite 32-point Gauss-Legendre on 8 pieces.  One thread.  out[0] = the
   integral; out_per_h2 (may be NULL) receives it divided by h^2. */
__global__ void self_cell_kernel(double alpha, double h, double *out, double *out_per_h2)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double L = 0.25 * PI;
    double acc = 0.0;
    for (int qp = 0; qp < 8; ++qp) {
        const double a0 = L * qp / 8.0, a1 = L * (qp + 1) / 8.0;
        const double mid = 0.5 * (a0 + a1), half = 0.5 * (a1 - a0);
        for (int k = 0; k < 32; ++k) {
            const double th = mid + half * GL32_T[k];
            const double R = 0.5 * h / cos(th);
            const K01 o = k01_fp64<false, true>(R * R, alpha, 0.25 * alpha * alpha, 4.0 / alpha);
            /* o.ak1r = alpha K1(alpha R)/R  =>  alpha R K1 = o.ak1r R^2 */
            acc += GL32_W[k] * half * (1.0 - o.ak1r * R * R) / (alpha * alpha);
        }
    }
    const double wc = 8.0 * acc * INV_2PI;
    if (out) out[0] = wc;
    if (out_per_h2) out_per_h2[0] = wc / (h * h);
}

/* ------------------------------------------------------------------------ */
/* GMRES BLAS-1                                                              */
/* ------------------------------------------------------------------------ */
/* out[c] = sum_i V[c*ld + i] * w[i], one block per column */
__global__ __launch_bounds__(256) void multi_dot_kernel(const double *__restrict__ V, int64_t ld, const double *__restrict__ w,
                                                        int64_t N, double *__restrict__ out)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    const double *v = V + c * ld;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += 256) s = fma(v[i], w[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}


/* out = s * in */
__global__ void scale_kernel(const double *__restrict__ in, double s, double *__restrict__ out, int64_t N)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) out[i] = s * in[i];
}

/* r = g - a */
__global__ void residual_kernel(const double *__restrict__ g, const double *__restrict__ a, double *__restrict__ r,
                                int64_t N)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) r[i] = g[i] - a[i];
}

/* ---- device-driven GMRES steps (every kernel does nothing once done) ---- */
/* Column k = j of the Hessenberg matrix (CGS2 coefficients h1 + h2,
   subdiagonal ||w|| = sqrt(hnsq)), the earlier Givens rotations applied to it,
   a new rotation that zeroes the subdiagonal, the rotated right-hand side g
   and the stopping decision.  H is (R+1) x R row-major.  Called by every
   thread of one block: the column and the rotations are staged in LDS (col:
   R + 2 values, rot: 2R) by all threads, the rotations run on thread 0, and
   the column is written back by all threads. */
__device__ void gs_finish_block(GState *__restrict__ gs, double *__restrict__ H, int R, double *__restrict__ cs,
                                double *__restrict__ sn, double *__restrict__ gv, const double *__restrict__ h1,
                                const double *__restrict__ h2, double hnsq, double *col, double *rot)
{
    const int k = gs->j;
    for (int c = threadIdx.x; c <= k; c += blockDim.x) {
        col[c] = h1[c] + h2[c];
        if (c < k) {
            rot[2 * c] = cs[c];
            rot[2 * c + 1] = sn[c];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double hn1 = sqrt(hnsq);
        col[k + 1] = hn1;
        for (int j = 0; j < k; ++j) {
            const double a = col[j], c = col[j + 1];
            col[j] = rot[2 * j] * a + rot[2 * j + 1] * c;
            col[j + 1] = -rot[2 * j + 1] * a + rot[2 * j] * c;
        }
        const double a = col[k], c = col[k + 1];
        const double den = hypot(a, c);
        const double ck = a / den, sk = c / den;
        cs[k] = ck;
        sn[k] = sk;
        col[k] = den;
        col[k + 1] = 0.0;
        gv[k + 1] = -sk * gv[k];
        gv[k] = ck * gv[k];
        gs->steps = k + 1;
        gs->resest = fabs(gv[k + 1]);
        gs->inv = hn1 > 0.0 ? 1.0 / hn1 : 0.0;
        if (gs->resest <= gs->thresh || hn1 == 0.0 || k + 1 >= gs->kmax) gs->done = 1;
    }
    __syncthreads();
    for (int c = threadIdx.x; c <= k + 1; c += blockDim.x) H[(int64_t)c * R + k] = col[c];
}

constexpr int GSF_T = 1024, GSF_W = GSF_T / 64, GSF_RMAX = 256;

/* The whole Gram-Schmidt part of an Arnoldi step in one block with the new
   vector held in registers (vectors up to GSR_NMAX long, any step): thread t
   owns elements t, t + GSF_T, ... (E of them).  The basis columns go through
   registers in chunks of C = 32 / E; while all columns fit in one chunk they
   are loaded once, together with the new vector, and serve both CGS passes.
   A pass forms the thread's partial dot products, sums them over the wave by
   a fixed butterfly and over the waves in wave order, then subtracts the
   projection in column order.  Then the norm, the Hessenberg column
   (gs_finish_block), and the next basis vector from the registers. */
constexpr int64_t GSR_NMAX = 8 * GSF_T;
/* basis columns the one-block form keeps in registers for vectors of length N;
   it serves the steps whose columns all fit, the slice form the later ones */
__host__ __device__ inline int gsr_cols(int64_t N) { return N <= GSF_T ? 32 : N <= 2 * GSF_T ? 16 : N <= 4 * GSF_T ? 8 : 4; }
/* steps take the one-block form while their basis columns exceed the register
   capacity by at most this many (read one at a time), the slice form after */
constexpr int GSR_EXTRA = 8;

/* v[c][k] = V_{c0+c}[t + k GSF_T] for the chunk's columns below ncol (0 elsewhere) */
template <int C, int E>
__device__ __forceinline__ void gsr_load(const double *__restrict__ V, int64_t ld, int64_t N, int c0, int ncol,
                                         double (&v)[C][E])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int64_t i = t + (int64_t)k * GSF_T;
            v[c][k] = (c0 + c < ncol && i < N) ? V[(int64_t)(c0 + c) * ld + i] : 0.0;
        }
}

/* the chunk's dot products with x: wave sums (wave_sum_dpp) into
   red[wave][c0 + c] */
template <int C, int E>
__device__ __forceinline__ void gsr_dots(const double (&v)[C][E], const double (&x)[E], int c0, int ncol,
                                         double (*red)[GSF_RMAX])
{
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    double p[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        p[c] = 0.0;
#pragma unroll
        for (int k = 0; k < E; ++k) p[c] = fma(v[c][k], x[k], p[c]);
        p[c] = wave_sum_dpp(p[c]);
    }
    if (ln == 0)
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c0 + c < ncol) red[wv][c0 + c] = p[c];
}

/* hp[c] = sum over the waves of red[.][c], in wave order (after a barrier) */
__device__ __forceinline__ void gsr_collect(double (*red)[GSF_RMAX], int ncol, double *hp)
{
    __syncthreads();
    for (int c = threadIdx.x; c < ncol; c += GSF_T) {
        double sacc = red[0][c];
        for (int q = 1; q < GSF_W; ++q) sacc += red[q][c];
        hp[c] = sacc;
    }
    __syncthreads();
}

template <int C, int E>
__device__ __forceinline__ void gsr_sub(const double (&v)[C][E], double (&x)[E], int c0, int ncol, const double *hp)
{
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (c0 + c >= ncol) break;
        const double h = hp[c0 + c];
#pragma unroll
        for (int k = 0; k < E; ++k) x[k] = fma(-h, v[c][k], x[k]);
    }
}

/* LDS of the one-block Gram-Schmidt */
struct GsrShared {
    double red[GSF_W][GSF_RMAX];
    double hs[2][GSF_RMAX];
    double nrm[GSF_W], hnl[1];
    double col[GSF_RMAX + 2], rot[2 * GSF_RMAX];
};

/* The one-block CGS2 step on w (length N), by every thread of a GSF_T block. */
template <int E>
__device__ __forceinline__ void gsr_body(GState *__restrict__ gs, double *__restrict__ V, int64_t ld,
                                         const double *__restrict__ w, int64_t N, double *__restrict__ H, int R,
                                         double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ gv,
                                         GsrShared &sh)
{
    constexpr int C = 32 / E;
    const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
    const int j = gs->j, ncol = j + 1;
    double x[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int64_t i = t + (int64_t)k * GSF_T;
        x[k] = i < N ? w[i] : 0.0;
    }
    if (ncol <= C) {
        double v[C][E];
        gsr_load<C, E>(V, ld, N, 0, ncol, v);
        for (int pass = 0; pass < 2; ++pass) {
            gsr_dots<C, E>(v, x, 0, ncol, sh.red);
            gsr_collect(sh.red, ncol, sh.hs[pass]);
            gsr_sub<C, E>(v, x, 0, ncol, sh.hs[pass]);
        }
    } else {
        /* the first C columns stay in registers for both passes; the others
           are read one at a time, twice per pass */
        double v[C][E];
        gsr_load<C, E>(V, ld, N, 0, ncol, v);
        for (int pass = 0; pass < 2; ++pass) {
            gsr_dots<C, E>(v, x, 0, ncol, sh.red);
            for (int c = C; c < ncol; ++c) {
                double u[1][E];
                gsr_load<1, E>(V, ld, N, c, ncol, u);
                gsr_dots<1, E>(u, x, c, ncol, sh.red);
            }
            gsr_collect(sh.red, ncol, sh.hs[pass]);
            gsr_sub<C, E>(v, x, 0, ncol, sh.hs[pass]);
            for (int c = C; c < ncol; ++c) {
                double u[1][E];
                gsr_load<1, E>(V, ld, N, c, ncol, u);
                gsr_sub<1, E>(u, x, c, ncol, sh.hs[pass]);
            }
        }
    }
    double sacc = 0.0;
#pragma unroll
    for (int k = 0; k < E; ++k) sacc = fma(x[k], x[k], sacc);
    sacc = wave_sum_dpp(sacc);
    if (ln == 0) sh.nrm[wv] = sacc;
    __syncthreads();
    if (t == 0) {
        double s2 = sh.nrm[0];
        for (int q = 1; q < GSF_W; ++q) s2 += sh.nrm[q];
        sh.hnl[0] = s2;
    }
    __syncthreads();
    gs_finish_block(gs, H, R, cs, sn, gv, sh.hs[0], sh.hs[1], sh.hnl[0], sh.col, sh.rot);
    if (gs->done) return; /* written by thread 0 before the block's last barrier */
    const double inv = gs->inv;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int64_t i = t + (int64_t)k * GSF_T;
        if (i < N) V[(int64_t)(j + 1) * ld + i] = inv * x[k];
    }
    __syncthreads(); /* every thread has read gs->j and gs->done */
    if (t == 0) gs->j = j + 1;
}

template <int E>
__global__ __launch_bounds__(GSF_T) void gs_reg_kernel(GState *__restrict__ gs, double *__restrict__ V, int64_t ld,
                                                       const double *__restrict__ w, int64_t N,
                                                       double *__restrict__ H, int R, double *__restrict__ cs,
                                                       double *__restrict__ sn, double *__restrict__ gv)
{
    __shared__ GsrShared sh;
    if (gs->done) return; /* the whole block */
    gsr_body<E>(gs, V, ld, w, N, H, R, cs, sn, gv, sh);
}

/* The Gram-Schmidt part of an Arnoldi step over many blocks (CGS2), for
   vectors too long for one block.  Block b owns the element slice
   [b L, (b+1) L); a pass leaves one partial dot product per (block, column)
   in P[b][c] (row stride pld), and the next kernel adds the partials in
   block order, so no result depends on timing.  Column c of a slice's dot
   products is summed by wave c % GSM_W. */
constexpr int GSM_T = 256, GSM_W = GSM_T / 64, GSM_NBMAX = 128, GSM_HMAX = 520;


/* slice length: a multiple of GSM_T giving at most GSM_NBMAX blocks */
static int64_t gsm_slice(int64_t N)
{
    const int64_t per = (N + (int64_t)GSM_T * GSM_NBMAX - 1) / ((int64_t)GSM_T * GSM_NBMAX);
    return GSM_T * std::max<int64_t>(1, per);
}

__device__ void gsm_partial_dots(const double *__restrict__ V, int64_t ld, const double *__restrict__ w, int64_t i0,
                                 int64_t n, int ncol, double *__restrict__ Prow)
{
    const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
    for (int c = wv; c < ncol; c += GSM_W) {
        const double *v = V + (int64_t)c * ld + i0;
        double sacc = 0.0;
        for (int64_t e = ln; e < n; e += 64) sacc = fma(v[e], w[i0 + e], sacc);
        sacc = gsf_wave_sum(sacc);
        if (ln == 0) Prow[c] = sacc;
    }
}

/* first pass: P[b][c] = V_c . w over slice b, c <= j */
__global__ __launch_bounds__(GSM_T) void gsm_dot_kernel(const GState *__restrict__ gs, const double *__restrict__ V,
                                                        int64_t ld, const double *__restrict__ w, int64_t N,
                                                        int64_t L, double *__restrict__ P, int pld)
{
    if (gs->done) return;
    const int64_t i0 = blockIdx.x * L;
    gsm_partial_dots(V, ld, w, i0, min(L, N - i0), gs->j + 1, P + (int64_t)blockIdx.x * pld);
}

/* h = sum_b Pin[b] (block 0 also stores it in hout); w -= sum_c h_c V_c on
   the slice; then either the partial dots of the new w (NORM = false, into
   Pout[b][c]) or its partial squared norm (NORM = true, into Pout[b]). */
template <bool NORM>
__global__ __launch_bounds__(GSM_T) void gsm_sub_kernel(const GState *__restrict__ gs, const double *__restrict__ V,
                                                        int64_t ld, double *__restrict__ w, int64_t N, int64_t L,
                                                        const double *__restrict__ Pin, int nb, int pld,
                                                        double *__restrict__ hout, double *__restrict__ Pout)
{
    __shared__ double hl[GSM_HMAX];
    __shared__ double red[GSM_W];
    if (gs->done) return;
    const int t = threadIdx.x;
    const int ncol = gs->j + 1;
    for (int c = t; c < ncol; c += GSM_T) {
        double h = Pin[c];
        for (int b = 1; b < nb; ++b) h += Pin[(int64_t)b * pld + c];
        hl[c] = h;
        if (blockIdx.x == 0) hout[c] = h;
    }
    __syncthreads();
    const int64_t i0 = blockIdx.x * L, n = min(L, N - i0);
    double sq = 0.0;
    for (int64_t e = t; e < n; e += GSM_T) {
        const int64_t i = i0 + e;
        double v = w[i];
        for (int c = 0; c < ncol; ++c) v = fma(-hl[c], V[(int64_t)c * ld + i], v);
        w[i] = v;
        sq = fma(v, v, sq);
    }
    if (NORM) {
        sq = gsf_wave_sum(sq);
        if ((t & 63) == 0) red[t >> 6] = sq;
        __syncthreads();
        if (t == 0) {
            double s2 = red[0];
            for (int q = 1; q < GSM_W; ++q) s2 += red[q];
            Pout[blockIdx.x] = s2;
        }
    } else {
        __syncthreads(); /* the slice of w, written above, is read across waves */
        gsm_partial_dots(V, ld, w, i0, n, ncol, Pout + (int64_t)blockIdx.x * pld);
    }
}

/* ||w||^2 from the slice partials (block order), the Hessenberg column, then
   V_{j+1} = w / ||w|| and the advance; one block */
__global__ __launch_bounds__(GSF_T) void gsm_finish_kernel(GState *__restrict__ gs, double *__restrict__ V,
                                                           int64_t ld, const double *__restrict__ w, int64_t N,
                                                           const double *__restrict__ Pn, int nb,
                                                           double *__restrict__ H, int R, double *__restrict__ cs,
                                                           double *__restrict__ sn, double *__restrict__ gv,
                                                           const double *__restrict__ h1,
                                                           const double *__restrict__ h2)
{
    __shared__ double col[GSM_HMAX + 2], rot[2 * GSM_HMAX];
    __shared__ double hn;
    if (gs->done) return;
    const int t = threadIdx.x;
    const int j = gs->j;
    if (t == 0) {
        double s2 = Pn[0];
        for (int b = 1; b < nb; ++b) s2 += Pn[b];
        hn = s2;
    }
    __syncthreads();
    gs_finish_block(gs, H, R, cs, sn, gv, h1, h2, hn, col, rot);
    if (gs->done) return; /* written by thread 0 before the block's last barrier */
    const double inv = gs->inv;
    for (int64_t i = t; i < N; i += GSF_T) V[(int64_t)(j + 1) * ld + i] = inv * w[i];
    __syncthreads(); /* every thread has read gs->j and gs->done */
    if (t == 0) gs->j = j + 1;
}

/* start of a cycle: state, g = beta e_1 */
__global__ void gs_init_kernel(GState *__restrict__ gs, double *__restrict__ gv, int R, int kmax, double beta,
                               double thresh, double *xout)
{
    for (int i = threadIdx.x; i <= R; i += blockDim.x) gv[i] = i == 0 ? beta : 0.0;
    if (threadIdx.x == 0) {
        gs->j = 0;
        gs->kmax = kmax;
        gs->done = 0;
        gs->steps = 0;
        gs->thresh = thresh;
        gs->inv = 0.0;
        gs->resest = beta;
        gs->xout = xout;
    }
}

/* start of the first cycle of a zero-guess solve whose ||b|| stays on the
   device: beta = ||b|| from its square bn2[0], V_0 = b / beta (zero when b
   is), g = beta e_1, the stopping threshold half_tol * beta, and ||b|| kept in
   the state for the host's first read (a zero b ends the cycle at once) */
__global__ void gs_init_dev_kernel(GState *__restrict__ gs, double *__restrict__ gv, int R, int kmax,
                                   double half_tol, const double *__restrict__ bn2, const double *__restrict__ b,
                                   double *__restrict__ V0, int64_t N, double *xout)
{
    const double beta = sqrt(bn2[0]);
    const double sc = beta > 0.0 ? 1.0 / beta : 0.0;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) V0[i] = sc * b[i];
    if (blockIdx.x != 0) return;
    for (int k = threadIdx.x; k <= R; k += blockDim.x) gv[k] = k == 0 ? beta : 0.0;
    if (threadIdx.x == 0) {
        gs->j = 0;
        gs->kmax = kmax;
        gs->done = beta > 0.0 ? 0 : 1;
        gs->steps = 0;
        gs->thresh = half_tol * beta;
        gs->inv = 0.0;
        gs->resest = beta;
        gs->bnorm = beta;
        gs->xout = xout;
    }
}

/* ---- end of a cycle, enqueued after its last chunk of steps; every kernel
   does nothing unless the cycle has ended (gs->done) ---- */
/* y = R_k^{-1} g_k for the k = steps leading columns (upper triangular back
   substitution), one wave: the row sums are split over the 64 lanes.  Also
   arms the tail state for the operator application that follows: density
   x (column 0, stride 0), active only when the cycle has ended. */
__global__ __launch_bounds__(64) void gs_solve_kernel(const GState *__restrict__ gs, GState *__restrict__ tail,
                                                      const double *__restrict__ H, int R,
                                                      const double *__restrict__ gv, double *__restrict__ y)
{
    if (!gs->done) {
        if (threadIdx.x == 0) tail->done = 1;
        return;
    }
    const int k = gs->steps;
    for (int i = k - 1; i >= 0; --i) {
        double s = 0.0;
        for (int m = i + 1 + (int)threadIdx.x; m < k; m += 64) s = fma(H[(int64_t)i * R + m], y[m], s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (threadIdx.x == 0) y[i] = (gv[i] - s) / H[(int64_t)i * R + i];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tail->j = 0;
        tail->done = 0;
    }
}

/* x += sum_{c < steps} y[c] V_c */
__global__ void gs_addcols_kernel(const GState *__restrict__ gs, const double *__restrict__ V, int64_t ld,
                                  const double *__restrict__ y, double *__restrict__ x, int64_t N)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N || !gs->done) return;
    const int k = gs->steps;
    double v = x[i];
    for (int c = 0; c < k; ++c) v = fma(y[c], V[c * ld + i], v);
    x[i] = v;
}

/* r = b - a and gs->rn2 = ||r||^2 (the true residual of the cycle's new
   iterate x, a = A x), and x copied to gs->xout when set; one block; the sum
   runs in a fixed order (each thread's strided elements, wave sums, waves in
   order) */
__global__ __launch_bounds__(GSF_T) void tail_residual_kernel(const GState *__restrict__ tail,
                                                              const double *__restrict__ b,
                                                              const double *__restrict__ a,
                                                              const double *__restrict__ x, double *__restrict__ r,
                                                              int64_t N, GState *__restrict__ gs)
{
    __shared__ double red[GSF_W];
    if (tail->done) return;
    const int t = threadIdx.x;
    double *xout = gs->xout;
    double s = 0.0;
    for (int64_t i = t; i < N; i += GSF_T) {
        const double v = b[i] - a[i];
        r[i] = v;
        s = fma(v, v, s);
        if (xout) xout[i] = x[i];
    }
    s = wave_sum_dpp(s);
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        double q = red[0];
        for (int k = 1; k < GSF_W; ++k) q += red[k];
        gs->rn2 = q;
    }
}

/* Start of a zero-guess FP64 solve in one block (vectors up to
   GS_START_NMAX): beta = ||bsrc||, b = bsrc (the solve's own copy), x = 0,
   V_0 = b / beta (zero when b is), g = beta e_1, the stopping threshold
   half_tol * beta, and beta kept in the state for the host's first read (a
   zero b ends the cycle at once).  The sum runs in a fixed order. */
constexpr int64_t GS_START_NMAX = 64 * GSF_T;
__global__ __launch_bounds__(GSF_T) void gs_start_kernel(GState *__restrict__ gs, double *__restrict__ gv, int R,
                                                         int kmax, double half_tol, const double *__restrict__ bsrc,
                                                         double *__restrict__ b, double *__restrict__ x,
                                                         double *__restrict__ V0, int64_t N, double *xout)
{
    __shared__ double red[GSF_W];
    __shared__ double bsh;
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < N; i += GSF_T) {
        const double v = bsrc[i];
        b[i] = v;
        x[i] = 0.0;
        s = fma(v, v, s);
    }
    s = wave_sum_dpp(s);
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        double q = red[0];
        for (int k = 1; k < GSF_W; ++k) q += red[k];
        bsh = sqrt(q);
    }
    __syncthreads();
    const double beta = bsh;
    const double sc = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int64_t i = t; i < N; i += GSF_T) V0[i] = sc * bsrc[i];
    for (int k = t; k <= R; k += GSF_T) gv[k] = k == 0 ? beta : 0.0;
    if (t == 0) {
        gs->j = 0;
        gs->kmax = kmax;
        gs->done = beta > 0.0 ? 0 : 1;
        gs->steps = 0;
        gs->thresh = half_tol * beta;
        gs->inv = 0.0;
        gs->resest = beta;
        gs->bnorm = beta;
        gs->rn2 = 0.0;
        gs->xout = xout;
    }
}

__global__ void fill_i32_kernel(int32_t *__restrict__ x, int32_t v, int64_t N)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) x[i] = v;
}

__global__ void fill_kernel(double *__restrict__ x, double v, int64_t N)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) x[i] = v;
}

#include "fmm.h"
#include "fourier.h"

/* ------------------------------------------------------------------------ */
/* host helpers                                                              */
/* ------------------------------------------------------------------------ */
static inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class T>
static mhlp_status dalloc(T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) return MHLP_OK;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) return fail(MHLP_NO_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    return MHLP_OK;
}

#define TRY(x)                          \
    do {                                \
        mhlp_status s_ = (x);           \
        if (s_ != MHLP_OK) return s_;   \
    } while (0)

/* ------------------------------------------------------------------------ */
/* FMM tree (host side): root square, stable counting sort of sources and    */
/* targets into leaf boxes, per-level occupancy, leaf work items, and the    */
/* translation tables (computed on the device)                               */
/* ------------------------------------------------------------------------ */
namespace mhlp {
struct FmmTree {
    FmmDev d{};
    std::vector<void *> bufs;
    int32_t order = 0, level = 0;
    ~FmmTree()
    {
        for (void *b : bufs)
            if (b) (void)hipFree(b);
    }
    template <class T>
    mhlp_status alloc(T **p, int64_t n)
    {
        mhlp_status s = dalloc(p, n < 1 ? 1 : n);
        if (s == MHLP_OK) bufs.push_back((void *)*p);
        return s;
    }
};
} // namespace mhlp
using mhlp::FmmTree;

static int fmm_coord(double v, double v0, double side, int nb)
{
    const double f = std::floor((v - v0) / side);
    return f < 0.0 ? 0 : (f >= (double)nb ? nb - 1 : (int)f);
}

struct FmmGeom {
    double x0, y0, S;
};

/* root square of the sources and targets (same definition as the oracle's) */
static FmmGeom fmm_root(const std::vector<double> &sx, const std::vector<double> &sy, const std::vector<double> &tx,
                        const std::vector<double> &ty)
{
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    auto upd = [&](const std::vector<double> &a, const std::vector<double> &b) {
        for (size_t k = 0; k < a.size(); ++k) {
            xmin = std::min(xmin, a[k]);
            xmax = std::max(xmax, a[k]);
            ymin = std::min(ymin, b[k]);
            ymax = std::max(ymax, b[k]);
        }
    };
    upd(sx, sy);
    upd(tx, ty);
    const double cx = 0.5 * (xmin + xmax), cy = 0.5 * (ymin + ymax);
    const double ext = std::max(xmax - xmin, ymax - ymin);
    const double S = ext > 0.0 ? ext * (1.0 + 0x1p-20) : 1.0;
    const double hS = 0.5 * S;
    return FmmGeom{cx - hS, cy - hS, S};
}

/* every node of every near panel of a target lies in the target's 3x3 leaf
   neighbourhood (then skipping near panels in the direct part skips them everywhere) */
static bool fmm_contains_near(const FmmGeom &G, int L, const std::vector<double> &sx, const std::vector<double> &sy,
                              const std::vector<double> &tx, const std::vector<double> &ty,
                              const std::vector<int32_t> &nptr, const std::vector<int32_t> &npan)
{
    const int nb = 1 << L;
    const double side = G.S / (double)nb;
    const int64_t M = (int64_t)tx.size(), Np = (int64_t)sx.size() / 16;
    for (int64_t i = 0; i < M; ++i) {
        const int ix = fmm_coord(tx[i], G.x0, side, nb), iy = fmm_coord(ty[i], G.y0, side, nb);
        for (int32_t q = nptr[i]; q < nptr[i + 1]; ++q) {
            const int64_t pn = npan[q];
            if (pn < 0 || pn >= Np) continue;
            for (int j = 0; j < 16; ++j) {
                const int jx = fmm_coord(sx[16 * pn + j], G.x0, side, nb);
                const int jy = fmm_coord(sy[16 * pn + j], G.y0, side, nb);
                if (std::abs(jx - ix) > 1 || std::abs(jy - iy) > 1) return false;
            }
        }
    }
    return true;
}

/* Build the tree.  Sources: host copies sx, sy and device arrays dsx.. (gathered
   into leaf order; dnx/dny NULL for the volume); targets tx, ty (host), or the
   sources themselves when same_points. */
static mhlp_status fmm_build(FmmTree *F, const FmmGeom &G, int L, int p, double alpha,
                             const std::vector<double> &sx, const std::vector<double> &sy,
                             const std::vector<double> &tx, const std::vector<double> &ty, bool same_points,
                             const double *dsx, const double *dsy, const double *dsw, const double *dnx,
                             const double *dny, hipStream_t st)
{
    FmmDev &T = F->d;
    const int nb = 1 << L;
    const int64_t nleaf = (int64_t)nb * nb, N = (int64_t)sx.size(), M = same_points ? N : (int64_t)tx.size();
    T.L = L;
    T.p = p;
    T.alpha = alpha;
    T.x0 = G.x0;
    T.y0 = G.y0;
    T.S = G.S;
    for (int l = 0; l <= L; ++l) {
        T.side[l] = G.S / (double)(1 << l);
        T.sig[l] = std::min(1.0, alpha * T.side[l]);
    }
    T.lstart = L + 1;
    for (int l = 2; l <= L; ++l)
        if (alpha * 0.586 * T.side[l] <= 40.0) {
            T.lstart = l;
            break;
        }
    /* stable counting sorts into the leaves */
    auto sort_pts = [&](const std::vector<double> &ax, const std::vector<double> &ay, int64_t n,
                        std::vector<int32_t> &start, std::vector<int32_t> &idx) {
        std::vector<int32_t> leaf(n);
        start.assign(nleaf + 1, 0);
        for (int64_t k = 0; k < n; ++k) {
            const int ix = fmm_coord(ax[k], G.x0, T.side[L], nb), iy = fmm_coord(ay[k], G.y0, T.side[L], nb);
            leaf[k] = iy * nb + ix;
            ++start[leaf[k] + 1];
        }
        for (int64_t b = 0; b < nleaf; ++b) start[b + 1] += start[b];
        std::vector<int32_t> pos(start.begin(), start.end() - 1);
        idx.resize(n);
        for (int64_t k = 0; k < n; ++k) idx[pos[leaf[k]]++] = (int32_t)k;
    };
    std::vector<int32_t> sstart, sidx, tstart, tidx;
    sort_pts(sx, sy, N, sstart, sidx);
    if (same_points) {
        tstart = sstart;
        tidx = sidx;
    } else {
        sort_pts(tx, ty, M, tstart, tidx);
    }
    /* occupancy per level */
    const int64_t nall = mhlp::lev4(L + 1);
    std::vector<int32_t> socc(nall, 0), tocc(nall, 0);
    for (int64_t b = 0; b < nleaf; ++b) {
        socc[mhlp::lev4(L) + b] = sstart[b + 1] - sstart[b];
        tocc[mhlp::lev4(L) + b] = tstart[b + 1] - tstart[b];
    }
    for (int l = L - 1; l >= 0; --l) {
        const int n1 = 1 << l;
        for (int iy = 0; iy < 2 * n1; ++iy)
            for (int ix = 0; ix < 2 * n1; ++ix) {
                const int64_t c = mhlp::lev4(l + 1) + iy * 2 * n1 + ix, pb = mhlp::lev4(l) + (iy >> 1) * n1 + (ix >> 1);
                socc[pb] += socc[c];
                tocc[pb] += tocc[c];
            }
    }
    /* leaf work items */
    std::vector<int32_t> wbox, wt0;
    for (int64_t b = 0; b < nleaf; ++b)
        for (int32_t t0 = tstart[b]; t0 < tstart[b + 1]; t0 += mhlp::FMM_TILE) {
            wbox.push_back((int32_t)b);
            wt0.push_back(t0);
        }
    T.nwork = (int)wbox.size();
    /* expansions and tables */
    int64_t eo = 0, to = 0;
    const int64_t rl = 3 * p + 1;
    std::vector<mhlp::FmmRow> rows;
    for (int l = 0; l <= L; ++l) {
        T.eoff[l] = T.t2l[l] = T.tmm[l] = T.tll[l] = 0;
        if (l < T.lstart) continue;
        T.eoff[l] = eo;
        eo += 2 * ((int64_t)1 << (2 * l)) * (p + 1);
        T.t2l[l] = to;
        for (int ox = -3; ox <= 3; ++ox)
            for (int oy = -3; oy <= 3; ++oy) {
                if (std::abs(ox) <= 1 && std::abs(oy) <= 1) continue;
                rows.push_back(mhlp::FmmRow{-ox * T.side[l], -oy * T.side[l], T.sig[l],
                                            to + ((ox + 3) * 7 + (oy + 3)) * rl, 0});
            }
        to += 49 * rl;
        if (l < L) {
            const double hc = 0.5 * T.side[l + 1];
            T.tmm[l] = to;
            for (int ch = 0; ch < 4; ++ch)
                rows.push_back(mhlp::FmmRow{(ch & 1) ? hc : -hc, (ch >> 1) ? hc : -hc, T.sig[l], to + ch * rl, 1});
            to += 4 * rl;
            T.tll[l] = to;
            for (int ch = 0; ch < 4; ++ch)
                rows.push_back(mhlp::FmmRow{(ch & 1) ? hc : -hc, (ch >> 1) ? hc : -hc, T.sig[l + 1], to + ch * rl, 1});
            to += 4 * rl;
        }
    }
    int32_t *d_sstart, *d_tstart, *d_sidx, *d_tidx, *d_socc, *d_tocc, *d_wbox, *d_wt0, *d_lpan = nullptr;
    double *d_lx, *d_ly, *d_lw, *d_lnx = nullptr, *d_lny = nullptr;
    cplx *d_mexp, *d_lexp, *d_tab;
    TRY(F->alloc(&d_sstart, nleaf + 1));
    TRY(F->alloc(&d_tstart, nleaf + 1));
    TRY(F->alloc(&d_sidx, N));
    TRY(F->alloc(&d_tidx, M));
    TRY(F->alloc(&d_socc, nall));
    TRY(F->alloc(&d_tocc, nall));
    TRY(F->alloc(&d_wbox, T.nwork));
    TRY(F->alloc(&d_wt0, T.nwork));
    TRY(F->alloc(&d_lx, N));
    TRY(F->alloc(&d_ly, N));
    TRY(F->alloc(&d_lw, N));
    if (dnx) {
        TRY(F->alloc(&d_lnx, N));
        TRY(F->alloc(&d_lny, N));
        TRY(F->alloc(&d_lpan, N));
    }
    TRY(F->alloc(&d_mexp, eo));
    TRY(F->alloc(&d_lexp, mhlp::FMM_CH * eo));
    TRY(F->alloc(&d_tab, to));
    mhlp::FmmRow *d_rows = nullptr;
    double *d_scr = nullptr;
    const int nrows = (int)rows.size();
    if (nrows > 0) {
        TRY(dalloc(&d_rows, nrows));
        mhlp_status s2 = dalloc(&d_scr, (int64_t)nrows * (2 * p + 1));
        if (s2 != MHLP_OK) {
            (void)hipFree(d_rows);
            return s2;
        }
    }
    auto up = [&](void *d, const void *h, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t e = up(d_sstart, sstart.data(), sstart.size() * 4);
    if (e == hipSuccess) e = up(d_tstart, tstart.data(), tstart.size() * 4);
    if (e == hipSuccess) e = up(d_sidx, sidx.data(), sidx.size() * 4);
    if (e == hipSuccess) e = up(d_tidx, tidx.data(), tidx.size() * 4);
    if (e == hipSuccess) e = up(d_socc, socc.data(), socc.size() * 4);
    if (e == hipSuccess) e = up(d_tocc, tocc.data(), tocc.size() * 4);
    if (e == hipSuccess) e = up(d_wbox, wbox.data(), wbox.size() * 4);
    if (e == hipSuccess) e = up(d_wt0, wt0.data(), wt0.size() * 4);
    if (e == hipSuccess && nrows > 0) e = up(d_rows, rows.data(), rows.size() * sizeof(mhlp::FmmRow));
    if (e == hipSuccess) {
        mhlp::fmm_gather_kernel<<<nblocks(N, 256), 256, 0, st>>>(d_sidx, N, dsx, dsy, dsw, dnx, dny, d_lx, d_ly, d_lw,
                                                                 d_lnx, d_lny, d_lpan);
        if (nrows > 0)
            mhlp::fmm_tables_kernel<<<nblocks(nrows, 64), 64, 0, st>>>(d_rows, nrows, p, alpha, d_tab, d_scr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (d_rows) (void)hipFree(d_rows);
    if (d_scr) (void)hipFree(d_scr);
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("fmm build: ") + hipGetErrorString(e));
    T.sstart = d_sstart;
    T.tstart = d_tstart;
    T.sidx = d_sidx;
    T.tidx = d_tidx;
    T.socc = d_socc;
    T.tocc = d_tocc;
    T.wbox = d_wbox;
    T.wt0 = d_wt0;
    T.lx = d_lx;
    T.ly = d_ly;
    T.lw = d_lw;
    T.lnx = d_lnx;
    T.lny = d_lny;
    T.lpan = d_lpan;
    T.mexp = d_mexp;
    T.lexp = d_lexp;
    T.lch = eo;
    for (int l = 0; l <= mhlp::FMM_LMAX; ++l) T.nch[l] = ((int64_t)1 << (2 * l)) < mhlp::FMM_CH_BOXES ? mhlp::FMM_CH : 1;
    T.tab = d_tab;
    F->order = p;
    F->level = L;
    return MHLP_OK;
}

/* upward and downward passes; the leaf kernel is launched by the caller */
template <bool SLP, bool DLP>
static void fmm_passes(const FmmTree *F, const double *sigma, const double *mu, hipStream_t st)
{
    const FmmDev &T = F->d;
    if (T.lstart > T.L) return;
    mhlp::fmm_p2m_kernel<SLP, DLP><<<(unsigned)(1u << (2 * T.L)), 64, 0, st>>>(T, sigma, mu);
    for (int l = T.L - 1; l >= T.lstart; --l)
        mhlp::fmm_m2m_kernel<SLP, DLP><<<(unsigned)(1u << (2 * l)), 256, 0, st>>>(T, l);
    for (int l = T.lstart; l <= T.L; ++l)
        mhlp::fmm_down_kernel<SLP, DLP><<<dim3(1u << (2 * l), (unsigned)T.nch[l]), 64 * mhlp::FMM_DW, 0, st>>>(T, l);
}

template <bool SLP, bool DLP>
static void fmm_far_t(const FmmTree *F, const FarArgs &A, hipStream_t st)
{
    fmm_passes<SLP, DLP>(F, A.sigma, A.mu, st);
    if (F->d.nwork > 0)
        mhlp::fmm_leaf_kernel<SLP, DLP, 0><<<(unsigned)F->d.nwork, 64 * mhlp::FMM_LW, 0, st>>>(F->d, A, mhlp::FmmVol{});
}

static GeoView view(const mhlp_geometry *g)
{
    GeoView G;
    G.x = g->soa;
    G.y = g->soa + g->N;
    G.pa = g->pa;
    G.ph = g->ph;
    G.pcx = g->pcx;
    G.pcy = g->pcy;
    G.prad = g->prad;
    G.N = g->N;
    G.Np = g->Np;
    return G;
}

/* ------------------------------------------------------------------------ */
/* geometry API                                                              */
/* ------------------------------------------------------------------------ */
extern "C" mhlp_status mhlp_geometry_create(int32_t n_curves, const int32_t *curve_panel_offsets,
                                            int32_t nodes_per_panel, const double *node_soa,
                                            const double *panel_ends, void *stream, mhlp_geometry **out)
{
    if (!out) return fail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!node_soa) return fail(MHLP_INVALID_ARG, "node_soa is NULL");
    if (!curve_panel_offsets) return fail(MHLP_INVALID_ARG, "curve_panel_offsets is NULL");
    if (n_curves < 1) return fail(MHLP_INVALID_ARG, "n_curves must be >= 1");
    if (nodes_per_panel != 16) return fail(MHLP_UNSUPPORTED, "nodes_per_panel must be 16");
    if (curve_panel_offsets[0] != 0) return fail(MHLP_INVALID_ARG, "curve_panel_offsets[0] must be 0");
    for (int32_t c = 0; c < n_curves; ++c)
        if (curve_panel_offsets[c + 1] <= curve_panel_offsets[c])
            return fail(MHLP_INVALID_ARG, "curve_panel_offsets must increase (every curve has a panel)");
    const int64_t n_panels = curve_panel_offsets[n_curves];
    if (n_panels > (INT_MAX / 16)) return fail(MHLP_INVALID_ARG, "n_panels out of range");
    hipStream_t st = (hipStream_t)stream;
    mhlp_geometry *g = new mhlp_geometry();
    HIPCHECK(hipGetDevice(&g->device));
    g->Np = n_panels;
    g->N = 16 * n_panels;
    g->curve_off.assign(curve_panel_offsets, curve_panel_offsets + n_curves + 1);
    const int64_t N = g->N, Np = g->Np;
    mhlp_status s;
    if ((s = dalloc(&g->soa, 6 * N)) || (s = dalloc(&g->w, N)) || (s = dalloc(&g->nx, N)) || (s = dalloc(&g->ny, N)) ||
        (s = dalloc(&g->kappa, N)) || (s = dalloc(&g->pa, 32 * Np)) || (s = dalloc(&g->ph, Np)) ||
        (s = dalloc(&g->pcx, Np)) || (s = dalloc(&g->pcy, Np)) || (s = dalloc(&g->prad, Np))) {
        mhlp_geometry_destroy(g);
        return s;
    }
    hipError_t e = hipMemcpyAsync(g->soa, node_soa, sizeof(double) * 6 * N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        geom_prep_kernel<<<nblocks(Np, 64), 64, 0, st>>>(g->soa, N, Np, g->w, g->nx, g->ny, g->kappa, g->pa, g->ph,
                                                          g->pcx, g->pcy, g->prad);
        e = hipGetLastError();
    }
    std::vector<int32_t> flags;
    int32_t *dnext = nullptr;
    if (e == hipSuccess && panel_ends) {
        std::vector<int32_t> next((size_t)Np);
        for (int32_t c = 0; c < n_curves; ++c)
            for (int32_t p = curve_panel_offsets[c]; p < curve_panel_offsets[c + 1]; ++p)
                next[p] = (p + 1 < curve_panel_offsets[c + 1]) ? p + 1 : curve_panel_offsets[c];
        flags.resize((size_t)Np);
        /* one buffer: next panels, then the flags */
        if ((s = dalloc(&dnext, 2 * Np))) {
            mhlp_geometry_destroy(g);
            return s;
        }
        e = hipMemcpyAsync(dnext, next.data(), sizeof(int32_t) * Np, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            panel_ends_kernel<<<nblocks(Np, 64), 64, 0, st>>>(g->pa, g->soa, g->soa + N, g->ph, panel_ends, dnext, Np,
                                                              PANEL_ENDS_TOL, dnext + Np);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(flags.data(), dnext + Np, sizeof(int32_t) * Np, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dnext) (void)hipFree(dnext);
    if (e != hipSuccess) {
        mhlp_geometry_destroy(g);
        return fail(MHLP_HIP_ERROR, std::string("geometry_create: ") + hipGetErrorString(e));
    }
    for (int64_t p = 0; p < (int64_t)flags.size(); ++p)
        if (flags[p]) {
            mhlp_geometry_destroy(g);
            return fail(MHLP_INVALID_ARG,
                        std::string("panel_ends: panel ") + std::to_string(p) +
                            ((flags[p] & 1) ? " does not end where its node polynomial ends"
                                            : " does not end where the next panel of its curve starts"));
        }
    *out = g;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_geometry_info(const mhlp_geometry *g, int64_t *n_nodes, int64_t *n_panels,
                                          int32_t *n_curves, int32_t *curve_panel_offsets, int32_t cap)
{
    if (!g) return fail(MHLP_INVALID_ARG, "geometry is NULL");
    const int32_t nc = (int32_t)g->curve_off.size() - 1;
    if (n_nodes) *n_nodes = g->N;
    if (n_panels) *n_panels = g->Np;
    if (n_curves) *n_curves = nc;
    if (curve_panel_offsets)
        for (int32_t c = 0; c <= nc && c < cap; ++c) curve_panel_offsets[c] = g->curve_off[c];
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_geometry_destroy(mhlp_geometry *g)
{
    if (!g) return MHLP_OK;
    double *ptrs[] = {g->soa, g->w, g->nx, g->ny, g->kappa, g->pa, g->ph, g->pcx, g->pcy, g->prad};
    for (double *p : ptrs)
        if (p) (void)hipFree(p);
    delete g;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_geometry_arrays(const mhlp_geometry *g, const double **w, const double **nx,
                                            const double **ny, const double **kappa)
{
    if (!g) return fail(MHLP_INVALID_ARG, "geometry is NULL");
    if (w) *w = g->w;
    if (nx) *nx = g->nx;
    if (ny) *ny = g->ny;
    if (kappa) *kappa = g->kappa;
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* plan API                                                                  */
/* ------------------------------------------------------------------------ */
/* Source splits of the far field: ns requested splits of the panel range
   (1 = none); the partial-sum buffer grows as needed. */
static mhlp_status plan_set_split(mhlp_plan *P, int ns)
{
    const int64_t Np = P->g->Np;
    if (ns < 1) ns = 1;
    if (ns > Np) ns = (int)Np;
    const int32_t pps = (int32_t)((Np + ns - 1) / ns);
    const int nsplit = (int)((Np + pps - 1) / pps);
    const int64_t need = nsplit > 1 ? (P->onsurf ? 2 : 4) * (int64_t)nsplit * P->M : 0;
    if (need > P->part_cap) {
        if (P->part) {
            HIPCHECK(hipDeviceSynchronize()); /* queued launches may still use it */
            (void)hipFree(P->part);
            P->part = nullptr;
            P->part_cap = 0;
        }
        TRY(dalloc(&P->part, need));
        P->part_cap = need;
    }
    P->pps = pps;
    P->nsplit = nsplit;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_plan_destroy(mhlp_plan *P)
{
    if (!P) return MHLP_OK;
    if (!P->onsurf) {
        if (P->tx) (void)hipFree(P->tx);
        if (P->ty) (void)hipFree(P->ty);
    }
    for (auto &gp : P->graphs)
        if (gp.second.exec) (void)hipGraphExecDestroy(gp.second.exec);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    void *ptrs[] = {P->near_ptr, P->near_panel, P->near_tgt, P->near_ts, P->wslp,  P->wdlp,    P->ws,
                    P->hdev,     P->part,       P->gdev,     P->perm,    P->wgrad, P->wstk,    P->stk_flux,
                    P->wstkg,    P->sym_tiles,  P->sym_p1,   P->sym_p2,  P->sym_bits, P->wcls, P->skpart,
                    P->sym_cls,  P->fqd};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete P->fmm;
    if (P->hhost) (void)hipHostFree(P->hhost);
    if (P->gstate_host) (void)hipHostFree(P->gstate_host);
    delete P;
    return MHLP_OK;
}

/* Blocks of far_eval_fp64<SLP, DLP> the chip holds at once (per CU times CUs). */
template <bool SLP, bool DLP>
static mhlp_status far_resident_blocks(int *out)
{
    int dev = 0, cus = 0, nb = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, far_eval_fp64<SLP, DLP>, FT_THREADS, 0));
    *out = (nb > 0 ? nb : 1) * (cus > 0 ? cus : 1);
    return MHLP_OK;
}

/* The (wave of 64 targets, panel) class table of the far-field tiles and the
   fine pieces' scales at the plan's alpha (built on the stream after the near
   lists, which it reads); the fused evaluation, the gradients and the
   stresslet kernels read it. */
static mhlp_status far_class_setup(mhlp_plan *P, hipStream_t st)
{
    const int64_t M = P->M, Np = P->g->Np;
    const int64_t TB = (M + FT_THREADS - 1) / FT_THREADS;
    TRY(dalloc(&P->wcls, TB * (FT_THREADS / 64) * Np));
    double fq[2 * KQ_NP];
    fine_scales(P->alpha, fq);
    TRY(dalloc(&P->fqd, 2 * KQ_NP));
    HIPCHECK(hipMemcpyAsync(P->fqd, fq, sizeof(fq), hipMemcpyHostToDevice, st)); /* fq lives until the sync below */
    far_class_kernel<<<(unsigned)TB, FT_THREADS, 0, st>>>(P->tx, P->ty, M, P->g->soa, P->g->soa + P->g->N, Np,
                                                          P->alpha, P->near_ptr, P->near_panel, P->wcls);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st)); /* later calls may come on other streams */
    return MHLP_OK;
}

/* The FP64 far field's launch shape: one block per resident slot of the chip
   for each layer variant (at most one per unit), the partial slots a target
   block can need, their buffer, and the (wave, panel) class table (built on the
   stream after the near lists, which it reads). */
/* blocks of the stream launch per block the chip holds at once: later waves
   of blocks let the hardware dispatcher even out what the equal unit counts
   leave uneven (measured on config 2 at alpha = 5: 1.49 / 1.39 / 1.35 / 1.36 ms
   for 1, 2, 4, 8) */
constexpr int SK_OVERSUB = 4;
static mhlp_status far_stream_setup(mhlp_plan *P, hipStream_t st)
{
    const int64_t M = P->M, Np = P->g->Np;
    const int64_t TB = (M + FT_THREADS - 1) / FT_THREADS, U = TB * Np;
    int res[3] = {0, 0, 0};
    TRY((far_resident_blocks<true, true>(&res[0])));
    TRY((far_resident_blocks<true, false>(&res[1])));
    TRY((far_resident_blocks<false, true>(&res[2])));
    int32_t smax = 1;
    for (int v = 0; v < 3; ++v) {
        const int Pv = (int)std::min<int64_t>((int64_t)SK_OVERSUB * res[v], U);
        P->sk_P[v] = Pv;
        for (int64_t tb = 0; tb < TB; ++tb) {
            const int64_t n = sk_block_of(U, Pv, tb * Np + Np - 1) - sk_block_of(U, Pv, tb * Np) + 1;
            smax = (int32_t)std::max<int64_t>(smax, n);
        }
    }
    P->sk_S = smax;
    {
        int64_t st_ = std::llround(0.6180339887498949 * (double)Np);
        if (st_ < 1) st_ = 1;
        while (std::gcd(st_, Np) != 1) ++st_;
        P->sk_stride = (int32_t)(st_ % Np == 0 ? 1 : st_ % Np);
    }
    TRY(dalloc(&P->skpart, 2 * (int64_t)smax * M));
    return far_class_setup(P, st);
}

static mhlp_status plan_create_impl(const mhlp_geometry *g, double alpha, const double *tx, const double *ty,
                                    int64_t m, const mhlp_params *prm, void *stream, mhlp_plan **out, bool stokes)
{
    if (!out) return fail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!g) return fail(MHLP_INVALID_ARG, "geometry is NULL");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(MHLP_INVALID_ARG, "alpha must be finite and > 0");
    if (m < 0 || m > INT_MAX - 1) return fail(MHLP_INVALID_ARG, "number of targets out of range");
    if (m > 0 && (!tx || !ty)) return fail(MHLP_INVALID_ARG, "target arrays are NULL");
    hipStream_t st = (hipStream_t)stream;
    mhlp_plan *P = new mhlp_plan();
    P->g = g;
    P->alpha = alpha;
    P->stokes = stokes;
    P->np.rho_direct = 3.5;
    P->np.rho_split = std::sqrt(3.5);
    P->np.ah_max = 4.5;
    P->np.far_exp = 40.0;
    if (prm) {
        if (prm->near_factor > 0) P->near_factor = prm->near_factor;
        if (prm->rho_direct > 0) P->np.rho_direct = prm->rho_direct;
        if (prm->rho_split > 0) P->np.rho_split = prm->rho_split;
        if (prm->ah_max > 0) P->np.ah_max = prm->ah_max;
        if (prm->far_exp > 0) P->np.far_exp = prm->far_exp;
    }
    mhlp_status s;
    if (m == 0) {
        P->onsurf = true;
        P->M = g->N;
        P->tx = g->soa;
        P->ty = g->soa + g->N;
    } else {
        P->M = m;
        if ((s = dalloc(&P->tx, m)) || (s = dalloc(&P->ty, m)) || (s = dalloc(&P->perm, m))) {
            mhlp_plan_destroy(P);
            return s;
        }
        /* Targets are kept in Morton (Z-curve) order of their coordinates, so the
           64 lanes of a wave hold nearby targets: they share near panels and
           fall on the same side of the z = 2 switch of the kernel values more
           often.  Results are written back through perm. */
        std::vector<double> hx((size_t)m), hy((size_t)m);
        hipError_t e = hipMemcpyAsync(hx.data(), tx, sizeof(double) * m, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hy.data(), ty, sizeof(double) * m, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            mhlp_plan_destroy(P);
            return fail(MHLP_HIP_ERROR, std::string("plan_create copy: ") + hipGetErrorString(e));
        }
        double x0 = hx[0], x1 = hx[0], y0 = hy[0], y1 = hy[0];
        for (int64_t i = 0; i < m; ++i) {
            if (!std::isfinite(hx[i]) || !std::isfinite(hy[i])) {
                mhlp_plan_destroy(P);
                return fail(MHLP_INVALID_ARG, "target coordinates must be finite");
            }
            x0 = std::min(x0, hx[i]), x1 = std::max(x1, hx[i]);
            y0 = std::min(y0, hy[i]), y1 = std::max(y1, hy[i]);
        }
        const double span = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
        auto spread = [](uint32_t v) { /* 16 bits -> even bit positions */
            uint64_t b = v & 0xFFFFu;
            b = (b | (b << 8)) & 0x00FF00FFull;
            b = (b | (b << 4)) & 0x0F0F0F0Full;
            b = (b | (b << 2)) & 0x33333333ull;
            b = (b | (b << 1)) & 0x55555555ull;
            return b;
        };
        std::vector<std::pair<uint64_t, int32_t>> key((size_t)m);
        for (int64_t i = 0; i < m; ++i) {
            const uint32_t qx = (uint32_t)std::min(65535.0, std::floor((hx[i] - x0) / span * 65536.0));
            const uint32_t qy = (uint32_t)std::min(65535.0, std::floor((hy[i] - y0) / span * 65536.0));
            key[i] = {spread(qx) | (spread(qy) << 1), (int32_t)i};
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<uint64_t, int32_t> &a, const std::pair<uint64_t, int32_t> &b) {
                             return a.first < b.first;
                         });
        std::vector<double> px((size_t)m), py((size_t)m);
        std::vector<int32_t> pm((size_t)m);
        for (int64_t i = 0; i < m; ++i) {
            pm[i] = key[i].second;
            px[i] = hx[pm[i]];
            py[i] = hy[pm[i]];
        }
        e = hipMemcpyAsync(P->tx, px.data(), sizeof(double) * m, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(P->ty, py.data(), sizeof(double) * m, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(P->perm, pm.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            mhlp_plan_destroy(P);
            return fail(MHLP_HIP_ERROR, std::string("plan_create copy: ") + hipGetErrorString(e));
        }
    }
    const int64_t M = P->M;
    {
        /* source splits so that about 8192 blocks of 256 targets run (the
           chip holds about 1024 at a time; several rounds keep the tail
           short); at least 2 panels per split.  mhlp_plan_autotune refines. */
        const int64_t tblocks = (M + FT_THREADS - 1) / FT_THREADS;
        int64_t ns = (8192 + tblocks - 1) / tblocks;
        if (ns > g->Np / 2) ns = g->Np / 2;
        if (ns < 1) ns = 1;
        if ((s = plan_set_split(P, (int)ns))) {
            mhlp_plan_destroy(P);
            return s;
        }
    }
    if (P->onsurf && g->N <= SYM_NMAX && g->N % 16 == 0) {
        /* tiles of the symmetric on-surface double layer, scalar or stresslet
           (row block I, column chunk J from the block's first panel on); the
           stresslet keeps two components per partial sum and no piece table */
        const int64_t ncomp = P->stokes ? 2 : 1;
        const int64_t nrb = (g->N + SYM_R - 1) / SYM_R, ncc = (g->N + SYM_C - 1) / SYM_C;
        std::vector<int2> tiles;
        for (int64_t I = 0; I < nrb; ++I)
            for (int64_t J = SYM_RP * I / SYM_CP; J < ncc; ++J) tiles.push_back(make_int2((int)I, (int)J));
        P->sym_ntiles = (int32_t)tiles.size();
        P->sym_nw = (int32_t)((g->Np + 31) / 32);
        if ((s = dalloc(&P->sym_tiles, (int64_t)tiles.size())) || (s = dalloc(&P->sym_p1, ncomp * ncc * g->N)) ||
            (s = dalloc(&P->sym_p2, ncomp * nrb * g->N)) ||
            (s = dalloc(&P->sym_bits, (int64_t)P->sym_nw * g->N)) ||
            (!P->stokes && (s = dalloc(&P->sym_cls, nrb * (SYM_R / 64) * g->Np)))) {
            mhlp_plan_destroy(P);
            return s;
        }
        hipError_t e = hipMemcpyAsync(P->sym_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice,
                                      st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  /* tiles is freed at the end of this block */
        if (e != hipSuccess) {
            mhlp_plan_destroy(P);
            return fail(MHLP_HIP_ERROR, std::string("plan_create tile copy: ") + hipGetErrorString(e));
        }
    }
    int32_t *cnt = nullptr;
    if ((s = dalloc(&cnt, M + 1)) || (s = dalloc(&P->near_ptr, M + 1))) {
        if (cnt) (void)hipFree(cnt);
        mhlp_plan_destroy(P);
        return s;
    }
    GeoView G = view(g);
    /* cnt[M] doubles as the fill-mismatch flag */
    near_list_kernel<<<nblocks(M, 128), 128, 0, st>>>(0, G, P->tx, P->ty, M, P->onsurf ? 1 : 0, P->near_factor,
                                                       P->np.rho_direct, cnt, nullptr, nullptr, nullptr, nullptr,
                                                       nullptr);
    scan_kernel<<<1, 1024, 0, st>>>(cnt, M, P->near_ptr);
    int32_t nnz = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&nnz, P->near_ptr + M, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(cnt);
        mhlp_plan_destroy(P);
        return fail(MHLP_HIP_ERROR, std::string("plan_create near count: ") + hipGetErrorString(e));
    }
    P->nnz = nnz;
    if (nnz > 0) {
        if ((s = dalloc(&P->near_panel, nnz)) || (s = dalloc(&P->near_tgt, nnz)) || (s = dalloc(&P->near_ts, 2 * (int64_t)nnz)) ||
            (!stokes && ((s = dalloc(&P->wslp, 16 * (int64_t)nnz)) || (s = dalloc(&P->wdlp, 16 * (int64_t)nnz)))) ||
            (stokes && (s = dalloc(&P->wstk, 64 * (int64_t)nnz)))) {
            mhlp_plan_destroy(P);
            return s;
        }
        fill_i32_kernel<<<1, 1, 0, st>>>(cnt + M, 0, 1);
        near_list_kernel<<<nblocks(M, 128), 128, 0, st>>>(1, G, P->tx, P->ty, M, P->onsurf ? 1 : 0, P->near_factor,
                                                           P->np.rho_direct, nullptr, P->near_ptr, P->near_panel,
                                                           P->near_tgt, P->near_ts, cnt + M);
        /* validate the list on the host before any kernel indexes with it */
        {
            std::vector<int32_t> hp((size_t)nnz);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = hipMemcpyAsync(hp.data(), P->near_panel, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                (void)hipFree(cnt);
                mhlp_plan_destroy(P);
                return fail(MHLP_HIP_ERROR, std::string("plan_create near list: ") + hipGetErrorString(e));
            }
            for (int32_t v : hp)
                if (v < -1 || v >= g->Np) {
                    (void)hipFree(cnt);
                    mhlp_plan_destroy(P);
                    return fail(MHLP_HIP_ERROR, "plan_create: near list holds an invalid panel index");
                }
        }
        if (stokes)
            near_stokes_weights_kernel<<<nblocks(nnz, 64), 64, 0, st>>>(G, P->tx, P->ty, P->onsurf ? 1 : 0,
                                                                         P->near_panel, P->near_tgt, P->near_ts, nnz,
                                                                         alpha, P->np, P->wstk);
        else
            near_weights_kernel<<<nblocks(nnz, 64), 64, 0, st>>>(G, P->tx, P->ty, P->onsurf ? 1 : 0, P->near_panel,
                                                                  P->near_tgt, P->near_ts, nnz, alpha, P->np, P->wslp,
                                                                  P->wdlp);
        e = hipGetLastError();
        int32_t mism = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&mism, cnt + M, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(cnt);
            mhlp_plan_destroy(P);
            return fail(MHLP_HIP_ERROR, std::string("plan_create near weights: ") + hipGetErrorString(e));
        }
        P->fill_mismatch = mism;
    }
    (void)hipFree(cnt);
    if ((s = stokes ? far_class_setup(P, st) : far_stream_setup(P, st))) {
        mhlp_plan_destroy(P);
        return s;
    }
    if (P->sym_bits) {
        near_bits_kernel<<<nblocks(M, 256), 256, 0, st>>>(P->near_ptr, P->near_panel, M, P->sym_nw, P->sym_bits);
        if (P->sym_cls)
            sym_class_kernel<<<nblocks(M, SYM_R), SYM_R, 0, st>>>(P->g->soa, P->g->soa + P->g->N, M, P->g->Np,
                                                                   P->alpha, P->sym_bits, P->sym_nw, P->sym_cls);
        hipError_t eb = hipGetLastError();
        if (eb == hipSuccess) eb = hipStreamSynchronize(st); /* later calls may come on other streams */
        if (eb != hipSuccess) {
            mhlp_plan_destroy(P);
            return fail(MHLP_HIP_ERROR, std::string("plan_create near bits: ") + hipGetErrorString(eb));
        }
    }
    if (stokes) {
        /* W term: device scalar for the flux, host 1/|Gamma| */
        if ((s = dalloc(&P->stk_flux, 8))) {
            mhlp_plan_destroy(P);
            return s;
        }
        std::vector<double> hw((size_t)g->N);
        hipError_t e2 = hipMemcpyAsync(hw.data(), g->w, sizeof(double) * g->N, hipMemcpyDeviceToHost, st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        if (e2 != hipSuccess) {
            mhlp_plan_destroy(P);
            return fail(MHLP_HIP_ERROR, std::string("stokes plan: ") + hipGetErrorString(e2));
        }
        double len = 0.0;
        for (double v : hw) len += v;
        P->inv_len = 1.0 / len;
    }
    *out = P;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_plan_create(const mhlp_geometry *g, double alpha, const double *tx, const double *ty,
                                        int64_t m, const mhlp_params *prm, void *stream, mhlp_plan **out)
{
    return plan_create_impl(g, alpha, tx, ty, m, prm, stream, out, false);
}

extern "C" mhlp_status mhlp_stokes_plan_create(const mhlp_geometry *g, double alpha, const double *tx,
                                               const double *ty, int64_t m, const mhlp_params *prm, void *stream,
                                               mhlp_plan **out)
{
    return plan_create_impl(g, alpha, tx, ty, m, prm, stream, out, true);
}

extern "C" mhlp_status mhlp_plan_info(const mhlp_plan *P, int64_t *n_targets, int64_t *n_sources,
                                      int64_t *n_near_pairs, double *alpha)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (n_targets) *n_targets = P->M;
    if (n_sources) *n_sources = P->g->N;
    if (n_near_pairs) *n_near_pairs = P->nnz;
    if (alpha) *alpha = P->alpha;
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* evaluation                                                                */
/* ------------------------------------------------------------------------ */
template <bool SLP, bool DLP>
static void launch_far_t(FarArgs A, const mhlp_plan *P, int nsplit, int32_t precision, hipStream_t st)
{
    const unsigned nb = nblocks(A.M, FT_THREADS);
    if (precision == MHLP_FP64) {
        A.skP = P->sk_P[SLP && DLP ? 0 : SLP ? 1 : 2];
        far_eval_fp64<SLP, DLP><<<(unsigned)A.skP, FT_THREADS, 0, st>>>(A);
        if (A.M <= FZ_SHORT)
            far_sk_finalize<SLP, DLP, FZ_L><<<nblocks(A.M, FZ_TG), FZ_TG * FZ_L, 0, st>>>(A);
        else
            far_sk_finalize<SLP, DLP, 1><<<nblocks(A.M, 256), 256, 0, st>>>(A);
        return;
    }
    if (nsplit <= 1) {
        far_eval_mixed<SLP, DLP, false><<<nb, FT_THREADS, 0, st>>>(A);
        return;
    }
    dim3 grid(nb, nsplit);
    far_eval_mixed<SLP, DLP, true><<<grid, FT_THREADS, 0, st>>>(A);
    if (A.M <= FZ_SHORT)
        far_finalize<SLP, DLP, FZ_L><<<nblocks(A.M, FZ_TG), FZ_TG * FZ_L, 0, st>>>(A, nsplit);
    else
        far_finalize<SLP, DLP, 1><<<nblocks(A.M, 256), 256, 0, st>>>(A, nsplit);
}

/* The far-field launch arguments of plan P for the given densities and outputs. */
static FarArgs far_args(const mhlp_plan *P, const double *sigma, const double *mu, double *us, double *ud,
                        double half_term, const GState *gs, int64_t jstride)
{
    const mhlp_geometry *g = P->g;
    FarArgs A;
    A.sx = g->soa;
    A.sy = g->soa + g->N;
    A.sw = g->w;
    A.snx = g->nx;
    A.sny = g->ny;
    A.sigma = sigma;
    A.mu = mu;
    A.N = g->N;
    A.tx = P->tx;
    A.ty = P->ty;
    A.M = P->M;
    A.nptr = P->near_ptr;
    A.npan = P->near_panel;
    A.wsl = P->wslp;
    A.wdl = P->wdlp;
    A.alpha = P->alpha;
    A.half_term = half_term;
    A.us = us;
    A.ud = ud;
    A.Np = g->Np;
    A.pps = P->pps;
    A.part_s = P->part;
    A.part_d = P->part + (int64_t)P->nsplit * P->M;
    A.gs = gs;
    A.jstride = jstride;
    A.perm = P->perm;
    A.pcx = g->pcx;
    A.pcy = g->pcy;
    A.prad = g->prad;
    A.skU = (int64_t)((P->M + FT_THREADS - 1) / FT_THREADS) * g->Np;
    A.skP = P->sk_P[0];
    A.skS = P->sk_S;
    A.skStride = P->sk_stride;
    A.skps = P->skpart;
    A.skpd = P->skpart + (int64_t)P->sk_S * P->M;
    A.wcls = P->wcls;
    A.fq = P->fqd;
    return A;
}

/* The symmetric on-surface operator's launches (FP64, scalar plan with
   symmetric tiles) */
static SymArgs sym_args(const mhlp_plan *P, const FarArgs &A)
{
    return SymArgs{A, P->sym_tiles, P->sym_p1, P->sym_p2, P->sym_bits, P->sym_nw, P->sym_cls};
}

static mhlp_status launch_far(const mhlp_plan *P, const double *sigma, const double *mu, double *us, double *ud,
                              double half_term, int32_t precision, hipStream_t st, const GState *gs = nullptr,
                              int64_t jstride = 0)
{
    if (precision != MHLP_FP64 && precision != MHLP_MIXED) return fail(MHLP_INVALID_ARG, "unknown precision");
    if (P->stokes) return fail(MHLP_INVALID_ARG, "a stokes plan evaluates with the mhlp_stokes_* calls");
    const mhlp_geometry *g = P->g;
    if (half_term != 0.0 && (!P->onsurf || P->M != g->N))
        return fail(MHLP_INVALID_ARG, "identity term needs an on-surface plan");
    const FarArgs A = far_args(P, sigma, mu, us, ud, half_term, gs, jstride);
    if (P->sym_tiles && !sigma && mu && precision == MHLP_FP64) {
        const SymArgs S = sym_args(P, A);
        sym_far_kernel<<<(unsigned)P->sym_ntiles, SYM_R, 0, st>>>(S);
        sym_finalize<<<nblocks(A.M, FZ_TG), FZ_TG * FZ_L, 0, st>>>(S, (int)((g->N + SYM_C - 1) / SYM_C));
        HIPCHECK(hipGetLastError());
        return MHLP_OK;
    }
    if (P->fmm && precision == MHLP_FP64 && !gs) {
        if (sigma && mu)
            fmm_far_t<true, true>(P->fmm, A, st);
        else if (sigma)
            fmm_far_t<true, false>(P->fmm, A, st);
        else
            fmm_far_t<false, true>(P->fmm, A, st);
        HIPCHECK(hipGetLastError());
        return MHLP_OK;
    }
    if (sigma && mu)
        launch_far_t<true, true>(A, P, P->nsplit, precision, st);
    else if (sigma)
        launch_far_t<true, false>(A, P, P->nsplit, precision, st);
    else
        launch_far_t<false, true>(A, P, P->nsplit, precision, st);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_eval_layer(const mhlp_plan *P, const double *sigma, const double *mu, double *u_slp,
                                       double *u_dlp, int32_t precision, void *stream)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    const bool ds = sigma && u_slp, dd = mu && u_dlp;
    if (!ds && !dd) return fail(MHLP_INVALID_ARG, "no density/output pair given");
    if ((sigma && !u_slp) || (u_slp && !sigma) || (mu && !u_dlp) || (u_dlp && !mu))
        return fail(MHLP_INVALID_ARG, "density and output must be given together");
    return launch_far(P, sigma, mu, u_slp, u_dlp, 0.0, precision, (hipStream_t)stream);
}

/* ------------------------------------------------------------------------ */
/* far-field launch shape: source splits, and their autotuner               */
/* ------------------------------------------------------------------------ */
extern "C" mhlp_status mhlp_plan_set_split(mhlp_plan *P, int32_t nsplit)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (nsplit < 1) return fail(MHLP_INVALID_ARG, "nsplit must be >= 1");
    return plan_set_split(P, nsplit);
}

extern "C" mhlp_status mhlp_plan_get_split(const mhlp_plan *P, int32_t *nsplit)
{
    if (!P || !nsplit) return fail(MHLP_INVALID_ARG, "NULL argument");
    *nsplit = P->nsplit;
    return MHLP_OK;
}

static mhlp_status launch_stokes(const mhlp_plan *P, const double *mu, double *u, int64_t ustride, bool bie,
                                 hipStream_t st, const GState *gs = nullptr, int64_t jstride = 0);

extern "C" mhlp_status mhlp_plan_autotune(mhlp_plan *P, int32_t layers, int32_t precision, int32_t reps,
                                          void *stream, int32_t *best_nsplit, double *best_ms, int32_t *cand,
                                          double *cand_ms, int32_t cap, int32_t *n_cand)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (layers < 1 || layers > 7) return fail(MHLP_INVALID_ARG, "layers must be 1 to 7");
    if ((layers >= 6) != P->stokes) return fail(MHLP_INVALID_ARG, "layers 6 and 7 (and only they) tune a stokes plan");
    if (layers >= 6 && precision != MHLP_FP64) return fail(MHLP_INVALID_ARG, "the stresslet is FP64 only");
    if (layers == 7 && P->onsurf) return fail(MHLP_INVALID_ARG, "layers 7 (stresslet gradient) needs an off-surface plan");
    if (layers == 4 && !P->onsurf) return fail(MHLP_INVALID_ARG, "layers 4 (BIE operator) needs an on-surface plan");
    if (layers == 5 && P->onsurf) return fail(MHLP_INVALID_ARG, "layers 5 (gradients) needs an off-surface plan");
    if (layers == 5 && precision != MHLP_FP64) return fail(MHLP_INVALID_ARG, "gradients are FP64 only");
    if (precision != MHLP_FP64 && precision != MHLP_MIXED) return fail(MHLP_INVALID_ARG, "unknown precision");
    if (reps < 1 || reps > 1000) return fail(MHLP_INVALID_ARG, "reps must be in [1, 1000]");
    if (cap < 0 || (cap > 0 && (!cand || !cand_ms))) return fail(MHLP_INVALID_ARG, "candidate arrays");
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->g->N, M = P->M, Np = P->g->Np;
    /* The FP64 single and double layers run as a stream of (target block, panel)
       units and the FP64 operator of a symmetric on-surface plan on its own
       tiles: neither uses the split.  For them the split serves the MIXED
       launch of the same layers (potentials, and the inner operator of mixed
       GMRES refinement), which is what gets timed. */
    if (precision == MHLP_FP64 && (layers <= 3 || (layers == 4 && P->sym_tiles))) precision = MHLP_MIXED;
    std::vector<int> cs;
    for (int64_t ns = 1; ns <= Np && ns <= 256; ns *= 2) cs.push_back((int)ns);
    if (std::find(cs.begin(), cs.end(), P->nsplit) == cs.end()) cs.push_back(P->nsplit);
    double *dens = nullptr, *out = nullptr;
    TRY(dalloc(&dens, 2 * N));
    mhlp_status s = dalloc(&out, 4 * M);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s == MHLP_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        s = fail(MHLP_HIP_ERROR, "hipEventCreate");
    int best = P->nsplit;
    double bms = 1e300;
    int nc = 0;
    std::vector<std::pair<int, double>> tim;
    if (s == MHLP_OK) fill_kernel<<<nblocks(2 * N, 256), 256, 0, st>>>(dens, 1.0, 2 * N);
    for (size_t c = 0; c < cs.size() && s == MHLP_OK; ++c) {
        if ((s = plan_set_split(P, cs[c]))) break;
        auto run = [&]() -> mhlp_status {
            if (layers == 5) return mhlp_eval_grad(P, dens, dens, out, out + M, out + 2 * M, out + 3 * M, st);
            if (layers == 6) return launch_stokes(P, dens, out, M, P->onsurf, st);
            if (layers == 7) return mhlp_stokes_eval_grad(P, dens, out, st);
            const double *sg = (layers & 1) ? dens : nullptr, *mu = (layers & 2 || layers == 4) ? dens : nullptr;
            return launch_far(P, sg, mu, sg ? out : nullptr, mu ? out + M : nullptr, layers == 4 ? 0.5 : 0.0,
                              precision, st);
        };
        if ((s = run())) break;
        if (hipEventRecord(e0, st) != hipSuccess) {
            s = fail(MHLP_HIP_ERROR, "hipEventRecord");
            break;
        }
        for (int r = 0; r < reps && s == MHLP_OK; ++r) s = run();
        if (s) break;
        float ms = 0.f;
        hipError_t e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            s = fail(MHLP_HIP_ERROR, std::string("autotune timing: ") + hipGetErrorString(e));
            break;
        }
        const double per = (double)ms / reps;
        tim.emplace_back(P->nsplit, per);
        if (nc < cap) {
            cand[nc] = P->nsplit;
            cand_ms[nc] = per;
        }
        ++nc;
        if (per < bms) bms = per;
    }
    /* fewest splits within 1% of the fastest (fewer partial sums, and a choice
       that is stable under timing noise) */
    if (s == MHLP_OK && !tim.empty()) {
        best = INT_MAX;
        for (const auto &t : tim)
            if (t.second <= 1.01 * bms && t.first < best) best = t.first;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(dens);
    if (out) (void)hipFree(out);
    if (s) return s;
    TRY(plan_set_split(P, best));
    if (best_nsplit) *best_nsplit = best;
    if (best_ms)
        for (const auto &t : tim)
            if (t.first == best) *best_ms = t.second;
    if (n_cand) *n_cand = std::min(nc, cap);
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_eval_slp(const mhlp_plan *P, const double *sigma, double *u, int32_t precision,
                                     void *stream)
{
    if (!sigma || !u) return fail(MHLP_INVALID_ARG, "sigma or u is NULL");
    return mhlp_eval_layer(P, sigma, nullptr, u, nullptr, precision, stream);
}

extern "C" mhlp_status mhlp_eval_dlp(const mhlp_plan *P, const double *mu, double *u, int32_t precision, void *stream)
{
    if (!mu || !u) return fail(MHLP_INVALID_ARG, "mu or u is NULL");
    return mhlp_eval_layer(P, nullptr, mu, nullptr, u, precision, stream);
}

extern "C" mhlp_status mhlp_apply_bie_operator(const mhlp_plan *P, const double *mu, double *out, int32_t precision,
                                               void *stream)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (!P->onsurf) return fail(MHLP_INVALID_ARG, "apply_bie_operator needs an on-surface plan (m == 0)");
    if (!mu || !out) return fail(MHLP_INVALID_ARG, "mu or out is NULL");
    if (mu == out) return fail(MHLP_INVALID_ARG, "mu and out must not alias");
    return launch_far(P, nullptr, mu, nullptr, out, 0.5, precision, (hipStream_t)stream);
}

/* ------------------------------------------------------------------------ */
/* target gradients                                                          */
/* ------------------------------------------------------------------------ */
static mhlp_status ensure_grad_weights(mhlp_plan *P, hipStream_t st)
{
    if (P->wgrad || P->nnz == 0) return MHLP_OK;
    TRY(dalloc(&P->wgrad, 64 * P->nnz));
    near_grad_weights_kernel<<<nblocks(P->nnz, 64), 64, 0, st>>>(view(P->g), P->tx, P->ty, P->near_panel,
                                                                  P->near_tgt, P->near_ts, P->nnz, P->alpha, P->np,
                                                                  P->wgrad);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(P->wgrad);
        P->wgrad = nullptr;
        return fail(MHLP_HIP_ERROR, std::string("gradient weights: ") + hipGetErrorString(e));
    }
    return MHLP_OK;
}

template <bool GS, bool GD>
static void launch_grad_t(const GradArgs &A, int nsplit, hipStream_t st)
{
    const unsigned nb = nblocks(A.M, FT_THREADS);
    if (nsplit <= 1) {
        far_grad_fp64<GS, GD, false><<<nb, FT_THREADS, 0, st>>>(A);
        return;
    }
    far_grad_fp64<GS, GD, true><<<dim3(nb, nsplit), FT_THREADS, 0, st>>>(A);
    grad_finalize<GS, GD><<<nblocks(A.M, 256), 256, 0, st>>>(A, nsplit);
}

extern "C" mhlp_status mhlp_eval_grad(const mhlp_plan *Pc, const double *sigma, const double *mu, double *gs_x,
                                      double *gs_y, double *gd_x, double *gd_y, void *stream)
{
    if (!Pc) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (Pc->onsurf) return fail(MHLP_UNSUPPORTED, "eval_grad needs an off-surface plan (targets off the curve)");
    if (Pc->stokes) return fail(MHLP_INVALID_ARG, "eval_grad needs a scalar plan");
    const bool gs = sigma != nullptr, gd = mu != nullptr;
    if (!gs && !gd) return fail(MHLP_INVALID_ARG, "no density given");
    if (gs != (gs_x != nullptr) || gs != (gs_y != nullptr) || gd != (gd_x != nullptr) || gd != (gd_y != nullptr))
        return fail(MHLP_INVALID_ARG, "each density needs both of its gradient outputs (and only then)");
    mhlp_plan *P = const_cast<mhlp_plan *>(Pc); /* gradient weights are built on first use */
    hipStream_t st = (hipStream_t)stream;
    TRY(ensure_grad_weights(P, st));
    const mhlp_geometry *g = P->g;
    GradArgs A;
    A.sx = g->soa;
    A.sy = g->soa + g->N;
    A.sw = g->w;
    A.snx = g->nx;
    A.sny = g->ny;
    A.sigma = sigma;
    A.mu = mu;
    A.tx = P->tx;
    A.ty = P->ty;
    A.M = P->M;
    A.Np = g->Np;
    A.nnz = P->nnz;
    A.nptr = P->near_ptr;
    A.npan = P->near_panel;
    A.perm = P->perm;
    A.wg = P->wgrad;
    A.alpha = P->alpha;
    A.pps = P->pps;
    A.part = P->part;
    A.wcls = P->wcls;
    A.fq = P->fqd;
    A.out[0] = gs_x;
    A.out[1] = gs_y;
    A.out[2] = gd_x;
    A.out[3] = gd_y;
    if (gs && gd)
        launch_grad_t<true, true>(A, P->nsplit, st);
    else if (gs)
        launch_grad_t<true, false>(A, P->nsplit, st);
    else
        launch_grad_t<false, true>(A, P->nsplit, st);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* modified-Stokes double layer: entry points                                */
/* ------------------------------------------------------------------------ */
static mhlp_status launch_stokes(const mhlp_plan *P, const double *mu, double *u, int64_t ustride, bool bie,
                                 hipStream_t st, const GState *gs, int64_t jstride)
{
    const mhlp_geometry *g = P->g;
    StkArgs A;
    A.sx = g->soa;
    A.sy = g->soa + g->N;
    A.sw = g->w;
    A.snx = g->nx;
    A.sny = g->ny;
    A.mu = mu;
    A.N = g->N;
    A.tx = P->tx;
    A.ty = P->ty;
    A.M = P->M;
    A.Np = g->Np;
    A.nnz = P->nnz;
    A.nptr = P->near_ptr;
    A.npan = P->near_panel;
    A.perm = P->perm;
    A.wst = P->wstk;
    A.alpha = P->alpha;
    A.pps = P->pps;
    A.part = P->part;
    A.u = u;
    A.ustride = ustride;
    A.bie = bie ? 1 : 0;
    A.flux = P->stk_flux;
    A.gs = gs;
    A.jstride = jstride;
    A.wcls = P->wcls;
    A.fq = P->fqd;
    if (bie) stk_flux_kernel<<<1, 256, 0, st>>>(A, P->inv_len, P->stk_flux);
    if (P->sym_tiles) { /* on-surface: each unordered far pair once */
        const StkSymArgs S{A, P->sym_tiles, P->sym_p1, P->sym_p2, P->sym_bits, P->sym_nw};
        stk_sym_kernel<<<(unsigned)P->sym_ntiles, SYM_R, 0, st>>>(S);
        stk_sym_finalize<<<nblocks(g->N, FZ_TG), FZ_TG * FZ_L, 0, st>>>(S, (int)((g->N + SYM_C - 1) / SYM_C));
        HIPCHECK(hipGetLastError());
        return MHLP_OK;
    }
    const unsigned nb = nblocks(A.M, FT_THREADS);
    if (P->nsplit <= 1) {
        far_stokes_fp64<false><<<nb, FT_THREADS, 0, st>>>(A);
    } else {
        far_stokes_fp64<true><<<dim3(nb, P->nsplit), FT_THREADS, 0, st>>>(A);
        if (A.M <= FZ_SHORT)
            stk_finalize<FZ_L><<<nblocks(A.M, FZ_TG), FZ_TG * FZ_L, 0, st>>>(A, P->nsplit);
        else
            stk_finalize<1><<<nblocks(A.M, 256), 256, 0, st>>>(A, P->nsplit);
    }
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_stokes_eval(const mhlp_plan *P, const double *mu, double *u, void *stream)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (!P->stokes) return fail(MHLP_INVALID_ARG, "stokes_eval needs a plan from mhlp_stokes_plan_create");
    if (!mu || !u) return fail(MHLP_INVALID_ARG, "mu or u is NULL");
    if (mu == u) return fail(MHLP_INVALID_ARG, "mu and u must not alias");
    return launch_stokes(P, mu, u, P->M, false, (hipStream_t)stream);
}

extern "C" mhlp_status mhlp_stokes_apply_bie(const mhlp_plan *P, const double *mu, double *out, void *stream)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (!P->stokes || !P->onsurf)
        return fail(MHLP_INVALID_ARG, "stokes_apply_bie needs an on-surface plan from mhlp_stokes_plan_create");
    if (!mu || !out) return fail(MHLP_INVALID_ARG, "mu or out is NULL");
    if (mu == out) return fail(MHLP_INVALID_ARG, "mu and out must not alias");
    return launch_stokes(P, mu, out, P->M, true, (hipStream_t)stream);
}

static mhlp_status ensure_stokes_grad_weights(mhlp_plan *P, hipStream_t st)
{
    if (P->wstkg || P->nnz == 0) return MHLP_OK;
    TRY(dalloc(&P->wstkg, 128 * P->nnz));
    near_stokes_grad_weights_kernel<<<nblocks(P->nnz, 64), 64, 0, st>>>(view(P->g), P->tx, P->ty, P->near_panel,
                                                                         P->near_tgt, P->near_ts, P->nnz, P->alpha,
                                                                         P->np, P->wstkg);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(P->wstkg);
        P->wstkg = nullptr;
        return fail(MHLP_HIP_ERROR, std::string("stresslet gradient weights: ") + hipGetErrorString(e));
    }
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_stokes_eval_grad(const mhlp_plan *Pc, const double *mu, double *g, void *stream)
{
    if (!Pc) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (!Pc->stokes) return fail(MHLP_INVALID_ARG, "stokes_eval_grad needs a plan from mhlp_stokes_plan_create");
    if (Pc->onsurf) return fail(MHLP_UNSUPPORTED, "stokes_eval_grad needs an off-surface plan (targets off the curve)");
    if (!mu || !g) return fail(MHLP_INVALID_ARG, "mu or g is NULL");
    if (mu == g) return fail(MHLP_INVALID_ARG, "mu and g must not alias");
    mhlp_plan *P = const_cast<mhlp_plan *>(Pc); /* gradient weights are built on first use */
    hipStream_t st = (hipStream_t)stream;
    TRY(ensure_stokes_grad_weights(P, st));
    const mhlp_geometry *geo = P->g;
    StkGArgs A;
    A.sx = geo->soa;
    A.sy = geo->soa + geo->N;
    A.sw = geo->w;
    A.snx = geo->nx;
    A.sny = geo->ny;
    A.mu = mu;
    A.N = geo->N;
    A.tx = P->tx;
    A.ty = P->ty;
    A.M = P->M;
    A.Np = geo->Np;
    A.nnz = P->nnz;
    A.nptr = P->near_ptr;
    A.npan = P->near_panel;
    A.perm = P->perm;
    A.wg = P->wstkg;
    A.alpha = P->alpha;
    A.pps = P->pps;
    A.part = P->part;
    A.g = g;
    A.wcls = P->wcls;
    A.fq = P->fqd;
    const unsigned nb = nblocks(A.M, FT_THREADS);
    if (P->nsplit <= 1) {
        far_stokes_grad_fp64<false><<<nb, FT_THREADS, 0, st>>>(A);
    } else {
        far_stokes_grad_fp64<true><<<dim3(nb, P->nsplit), FT_THREADS, 0, st>>>(A);
        stkg_finalize<<<nblocks(A.M, 256), 256, 0, st>>>(A, P->nsplit);
    }
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* GMRES                                                                     */
/* ------------------------------------------------------------------------ */
/* length of the unknown vector and the on-surface operator of the plan:
   (1/2 I + D) mu for the scalar kernel (N), (1/2 I + D + W) mu for the
   stresslet (2N, component-major) */
static int64_t vlen(const mhlp_plan *P) { return P->stokes ? 2 * P->g->N : P->g->N; }

static mhlp_status apply_op(mhlp_plan *P, const double *x, double *out, int32_t prec, hipStream_t st,
                            const GState *gs = nullptr, int64_t jstride = 0)
{
    if (P->stokes) return launch_stokes(P, x, out, P->g->N, true, st, gs, jstride);
    return launch_far(P, nullptr, x, nullptr, out, 0.5, prec, st, gs, jstride);
}

static mhlp_status ensure_ws(mhlp_plan *P, int64_t cols)
{
    if (P->ws && P->ws_cols >= cols) return MHLP_OK;
    if (P->ws) (void)hipFree(P->ws);
    P->ws = nullptr;
    TRY(dalloc(&P->ws, (cols + 6) * vlen(P)));
    P->ws_cols = cols;
    if (!P->hdev) TRY(dalloc(&P->hdev, 4 * 1024));
    if (!P->hhost) HIPCHECK(hipHostMalloc((void **)&P->hhost, sizeof(double) * 4 * 1024, hipHostMallocDefault));
    return MHLP_OK;
}

/* ||v||_2 (synchronising) */
static mhlp_status dnorm(mhlp_plan *P, const double *v, int64_t N, hipStream_t st, double *out)
{
    multi_dot_kernel<<<1, 256, 0, st>>>(v, N, v, N, P->hdev);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(P->hhost, P->hdev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    *out = std::sqrt(P->hhost[0]);
    return MHLP_OK;
}

/* Device data of the device-driven GMRES for restart length R. */
struct GmresDev {
    GState *gs;
    GState *tail; /* density selector of the end-of-cycle operator: j = 0, done unless gs->done */
    double *H, *cs, *sn, *gv, *y, *h1, *h2, *hn;
    double *p1, *p2, *pn; /* multi-block Gram-Schmidt partials: [nb][R+1], [nb][R+1], [nb] */
};

static GmresDev gdev_view(const mhlp_plan *P)
{
    const int R = P->gdev_R;
    double *d = reinterpret_cast<double *>(P->gdev + 128);
    GmresDev v;
    v.gs = reinterpret_cast<GState *>(P->gdev);
    v.tail = reinterpret_cast<GState *>(P->gdev + 64);
    v.H = d;
    d += (int64_t)(R + 1) * R;
    v.cs = d;
    d += R;
    v.sn = d;
    d += R;
    v.gv = d;
    d += R + 1;
    v.y = d;
    d += R;
    v.h1 = d;
    d += R + 1;
    v.h2 = d;
    d += R + 1;
    v.hn = d;
    d += 1;
    const int64_t nb = (vlen(P) + gsm_slice(vlen(P)) - 1) / gsm_slice(vlen(P));
    v.p1 = d;
    d += nb * (R + 1);
    v.p2 = d;
    d += nb * (R + 1);
    v.pn = d;
    return v;
}

static mhlp_status ensure_gdev(mhlp_plan *P, int R)
{
    if (P->gdev && P->gdev_R >= R) return MHLP_OK;
    if (P->gdev) {
        HIPCHECK(hipDeviceSynchronize());
        (void)hipFree(P->gdev);
        P->gdev = nullptr;
    }
    const int64_t nb = (vlen(P) + gsm_slice(vlen(P)) - 1) / gsm_slice(vlen(P));
    const int64_t nd = (int64_t)(R + 1) * R + 3 * R + 3 * (R + 1) + 1 + nb * (2 * (R + 1) + 1);
    char *g = nullptr;
    TRY(dalloc(&g, 128 + 8 * nd));
    P->gdev = g;
    P->gdev_R = R;
    if (!P->gstate_host) HIPCHECK(hipHostMalloc((void **)&P->gstate_host, sizeof(GState), hipHostMallocDefault));
    return MHLP_OK;
}

/* Arnoldi steps of the first captured chunk of a GMRES cycle (later chunks
   follow the observed convergence rate); measured on the config-2 solves, 4
   saves a replay at alpha = 50 and 500 against 2 and costs nothing at 5 */
constexpr int GMRES_FIRST_CHUNK = 4;

/* Waits for the stream by polling it: the chunk reads of GMRES are a few tens
   of microseconds apart, shorter than a blocking wait takes to wake. */
static hipError_t spin_sync(hipStream_t st)
{
    hipError_t e;
    while ((e = hipStreamQuery(st)) == hipErrorNotReady) {
    }
    return e;
}

/* One Arnoldi step of the device-driven GMRES, enqueued on st (one_block: the
   Gram-Schmidt part in one block, else over element slices). */
static mhlp_status enqueue_step(mhlp_plan *P, int32_t prec, bool one_block, hipStream_t st)
{
    const int64_t N = vlen(P);
    const int R = P->gdev_R;
    double *V = P->ws, *w = P->ws + (int64_t)(R + 1) * N;
    const GmresDev d = gdev_view(P);
    TRY(apply_op(P, V, w, prec, st, d.gs, N));
    if (one_block) {
        if (N <= GSF_T)
            gs_reg_kernel<1><<<1, GSF_T, 0, st>>>(d.gs, V, N, w, N, d.H, R, d.cs, d.sn, d.gv);
        else if (N <= 2 * GSF_T)
            gs_reg_kernel<2><<<1, GSF_T, 0, st>>>(d.gs, V, N, w, N, d.H, R, d.cs, d.sn, d.gv);
        else if (N <= 4 * GSF_T)
            gs_reg_kernel<4><<<1, GSF_T, 0, st>>>(d.gs, V, N, w, N, d.H, R, d.cs, d.sn, d.gv);
        else
            gs_reg_kernel<8><<<1, GSF_T, 0, st>>>(d.gs, V, N, w, N, d.H, R, d.cs, d.sn, d.gv);
        HIPCHECK(hipGetLastError());
        return MHLP_OK;
    }
    /* classical Gram-Schmidt, twice, over element slices */
    const int64_t L = gsm_slice(N);
    const int nb = (int)((N + L - 1) / L);
    gsm_dot_kernel<<<nb, GSM_T, 0, st>>>(d.gs, V, N, w, N, L, d.p1, R + 1);
    gsm_sub_kernel<false><<<nb, GSM_T, 0, st>>>(d.gs, V, N, w, N, L, d.p1, nb, R + 1, d.h1, d.p2);
    gsm_sub_kernel<true><<<nb, GSM_T, 0, st>>>(d.gs, V, N, w, N, L, d.p2, nb, R + 1, d.h2, d.pn);
    gsm_finish_kernel<<<1, GSF_T, 0, st>>>(d.gs, V, N, w, N, d.pn, nb, d.H, R, d.cs, d.sn, d.gv, d.h1, d.h2);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* End of a cycle (each kernel a no-op unless the state says done): y from
   the rotated Hessenberg system, x += V y, and the true residual r = b - A x
   with the FP64 operator (whatever the precision of the cycle's Arnoldi
   steps) and its squared norm in the state, so that the host reads the
   outcome of the cycle with the state itself.  x and b are the solve's own
   vectors. */
static mhlp_status enqueue_tail(mhlp_plan *P, const double *b, double *x, hipStream_t st)
{
    const int64_t N = vlen(P);
    const int R = P->gdev_R;
    double *V = P->ws, *w = P->ws + (int64_t)(R + 1) * N, *r = w + N;
    const GmresDev d = gdev_view(P);
    gs_solve_kernel<<<1, 64, 0, st>>>(d.gs, d.tail, d.H, R, d.gv, d.y);
    gs_addcols_kernel<<<nblocks(N, 256), 256, 0, st>>>(d.gs, V, N, d.y, x, N);
    HIPCHECK(hipGetLastError());
    TRY(apply_op(P, x, w, MHLP_FP64, st, d.tail, 0));
    tail_residual_kernel<<<1, GSF_T, 0, st>>>(d.tail, b, w, x, r, N, d.gs);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* longest chunk of Arnoldi steps captured in one graph */
constexpr int GMRES_MAX_CHUNK = 16;

/* Executable graph of S consecutive Arnoldi steps (0 <= S <= GMRES_MAX_CHUNK),
   the first m of them with the one-block Gram-Schmidt, followed by the end of
   the cycle when `tail` is set; captured once per plan state (workspace,
   split, restart, the solve's x and b) on a private stream. */
static mhlp_status step_graph(mhlp_plan *P, int32_t prec, int m, int S, bool tail, const double *b, double *x,
                              hipGraphExec_t *out)
{
    const int key = (((prec == MHLP_MIXED ? 1 : 0) * (GMRES_MAX_CHUNK + 1) + S) * (GMRES_MAX_CHUNK + 1) + m) * 2 +
                    (tail ? 1 : 0);
    mhlp_plan::StepGraph &G = P->graphs[key];
    if (G.exec && G.ws == P->ws && G.part == P->part && G.gdev == P->gdev && G.R == P->gdev_R &&
        G.nsplit == P->nsplit && G.x == x && G.b == b) {
        *out = G.exec;
        return MHLP_OK;
    }
    if (G.exec) {
        (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
    }
    if (!P->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    HIPCHECK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    mhlp_status s = MHLP_OK;
    for (int k = 0; k < S && s == MHLP_OK; ++k) s = enqueue_step(P, prec, k < m, P->cap_stream);
    if (tail && s == MHLP_OK) s = enqueue_tail(P, b, x, P->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
    if (s != MHLP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("GMRES step capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        G.exec = nullptr;
        return fail(MHLP_HIP_ERROR, std::string("GMRES step graph: ") + hipGetErrorString(e));
    }
    G.ws = P->ws;
    G.part = P->part;
    G.gdev = P->gdev;
    G.R = P->gdev_R;
    G.nsplit = P->nsplit;
    G.x = x;
    G.b = b;
    *out = G.exec;
    return MHLP_OK;
}

/* One restarted-GMRES solve of A x = b to relative tolerance `tol` (relative
   to bnorm), FP64 Arnoldi with CGS2 on the operator in `prec`, each cycle
   ended by the true residual with the FP64 operator.  A cycle stops once its
   residual estimate is below 0.5 tol bnorm or, when larger, cycle_rel times
   the residual it started from: with the mixed-precision operator (cycle_rel
   = 0.5e-6, the FP32 far field resolving the operator to ~1e-7) this is
   iterative refinement, each cycle an inner solve of A d = r corrected by the
   FP64 residual.  x and b belong to
   the plan's workspace (captured graphs refer to them); x is updated in
   place.  The Arnoldi steps, the Givens rotations, the stopping test and the
   end of each cycle (x += V y, the true residual, and a copy of x into xout
   when given) run on the device; the
   host replays captured chunks of steps and reads the state once per chunk.
   The first chunk of a solve is as long as the first cycle of the previous
   solve on this plan (GMRES_FIRST_CHUNK the first time), later chunks follow
   the observed convergence rate; a chunk expected to end the cycle carries
   its end, and steps after the stopping point do nothing.  With first_dev
   the solve starts from x = 0 with ||b|| formed on the device from bsrc,
   which is copied into b. */
static mhlp_status gmres_core(mhlp_plan *P, double *b, double bnorm, double *x, double tol, int restart,
                              int max_iter, int32_t prec, hipStream_t st, int *iters, int *cycles, double *relres,
                              const double *r_first, double beta_first, bool first_dev_in = false,
                              const double *bsrc = nullptr, double *xout = nullptr, double cycle_rel = 0.0)
{
    const double half_tol = std::max(0.5 * tol, cycle_rel); /* first cycle of a device-normed solve */
    const int64_t N = vlen(P);
    TRY(ensure_gdev(P, restart));
    const int R = P->gdev_R;
    double *V = P->ws;
    double *w = P->ws + (int64_t)(R + 1) * N;
    double *r = w + N;
    const GmresDev d = gdev_view(P);
    const unsigned nbN = nblocks(N, 256);
    const int pi = prec == MHLP_MIXED ? 1 : 0;
    int it = 0;
    *cycles = 0;
    double beta_tail = 0.0;
    for (;;) {
        /* residual at the start of the cycle: handed over by the caller for
           the first cycle (b itself for a zero initial guess), left in r by
           the previous cycle's end otherwise */
        double beta;
        const double *rr;
        const bool first_dev = first_dev_in && *cycles == 0;
        if (first_dev) {
            beta = 0.0; /* known after the first read of the state */
            rr = nullptr;
        } else if (*cycles == 0 && r_first) {
            beta = beta_first;
            rr = r_first;
        } else if (*cycles == 0) {
            TRY(apply_op(P, x, w, MHLP_FP64, st));
            residual_kernel<<<nbN, 256, 0, st>>>(b, w, r, N);
            TRY(dnorm(P, r, N, st, &beta));
            rr = r;
        } else {
            beta = beta_tail;
            rr = r;
        }
        if (!first_dev) {
            *relres = beta / bnorm;
            if (*relres <= tol || it >= max_iter) break;
        }
        ++*cycles;
        const int kmax = std::min(restart, max_iter - it);
        if (first_dev) {
            if (N <= GS_START_NMAX) {
                gs_start_kernel<<<1, GSF_T, 0, st>>>(d.gs, d.gv, R, kmax, half_tol, bsrc, b, x, V, N, xout);
            } else {
                HIPCHECK(hipMemcpyAsync(b, bsrc, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
                fill_kernel<<<nbN, 256, 0, st>>>(x, 0.0, N);
                multi_dot_kernel<<<1, 256, 0, st>>>(b, N, b, N, P->hdev); /* ||b||^2 */
                gs_init_dev_kernel<<<nbN, 256, 0, st>>>(d.gs, d.gv, R, kmax, half_tol, P->hdev, b, V, N, xout);
            }
        } else {
            scale_kernel<<<nbN, 256, 0, st>>>(rr, 1.0 / beta, V, N);
            gs_init_kernel<<<1, 256, 0, st>>>(d.gs, d.gv, R, kmax, beta,
                                              std::max(0.5 * tol * bnorm, cycle_rel * beta), xout);
        }
        HIPCHECK(hipGetLastError());
        int done_steps = 0;
        /* the first cycle starts with the previous solve's count and its end
           appended; otherwise GMRES_FIRST_CHUNK steps */
        const bool hist = *cycles == 1 && P->gm_first_steps[pi] > 0;
        int chunk = hist ? P->gm_first_steps[pi] : GMRES_FIRST_CHUNK;
        bool expect_end = hist;
        double last_est = beta, thresh = std::max(0.5 * tol * bnorm, cycle_rel * beta);
        GState gsh;
        for (;;) {
            const int S = std::max(1, std::min({chunk, GMRES_MAX_CHUNK, kmax - done_steps}));
            const bool tail = expect_end || S == kmax - done_steps;
            /* Gram-Schmidt in one block for the steps whose basis columns fit
               its registers, or exceed them by at most GSR_EXTRA (step j has
               j + 1), over slices after them */
            const int m = (N <= GSR_NMAX && R <= GSF_RMAX)
                              ? std::max(0, std::min(S, gsr_cols(N) + GSR_EXTRA - done_steps))
                              : 0;
            hipGraphExec_t ex;
            TRY(step_graph(P, prec, m, S, tail, b, x, &ex));
            HIPCHECK(hipGraphLaunch(ex, st));
            HIPCHECK(hipMemcpyAsync(P->gstate_host, d.gs, sizeof(GState), hipMemcpyDeviceToHost, st));
            HIPCHECK(spin_sync(st));
            gsh = *P->gstate_host;
            if (first_dev && done_steps == 0) {
                bnorm = gsh.bnorm;
                if (bnorm == 0.0) { /* b = 0: x = 0 (set by the start kernel) */
                    *relres = 0.0;
                    *iters = 0;
                    *cycles = 0;
                    return MHLP_OK;
                }
                last_est = bnorm;
                thresh = half_tol * bnorm;
            }
            if (gsh.done) {
                if (!tail) { /* the cycle ended before its end was enqueued */
                    TRY(step_graph(P, prec, 0, 0, true, b, x, &ex));
                    HIPCHECK(hipGraphLaunch(ex, st));
                    HIPCHECK(hipMemcpyAsync(P->gstate_host, d.gs, sizeof(GState), hipMemcpyDeviceToHost, st));
                    HIPCHECK(spin_sync(st));
                    gsh = *P->gstate_host;
                }
                break;
            }
            /* steps still needed at the rate observed over this chunk */
            const int ran = gsh.steps - done_steps;
            done_steps = gsh.steps;
            expect_end = false;
            int need = GMRES_MAX_CHUNK;
            if (ran > 0 && gsh.resest > 0.0 && gsh.resest < last_est) {
                const double rate = std::pow(gsh.resest / last_est, 1.0 / ran);
                const double est = std::ceil(std::log(thresh / gsh.resest) / std::log(rate));
                if (est <= GMRES_MAX_CHUNK) {
                    need = std::max(1, (int)est);
                    expect_end = true;
                }
            }
            last_est = gsh.resest;
            chunk = need;
        }
        it += gsh.steps;
        if (*cycles == 1) P->gm_first_steps[pi] = std::max(1, gsh.steps);
        beta_tail = std::sqrt(gsh.rn2);
    }
    *iters = it;
    return MHLP_OK;
}

static mhlp_status gmres_solve_impl(const mhlp_plan *Pc, const double *g, double *mu, const mhlp_gmres_opts *opts,
                                    mhlp_gmres_info *info, void *stream)
{
    if (!Pc) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (!Pc->onsurf) return fail(MHLP_INVALID_ARG, "gmres_solve needs an on-surface plan (m == 0)");
    if (!g || !mu || !opts || !info) return fail(MHLP_INVALID_ARG, "NULL argument");
    if (g == mu) return fail(MHLP_INVALID_ARG, "g and mu must not alias");
    if (!(opts->tol > 0.0) || opts->max_iter < 1 || opts->restart < 1 || opts->restart > 512)
        return fail(MHLP_INVALID_ARG, "bad GMRES options");
    if (opts->precision != MHLP_FP64 && opts->precision != MHLP_MIXED)
        return fail(MHLP_INVALID_ARG, "unknown precision");
    if (Pc->stokes && opts->precision != MHLP_FP64)
        return fail(MHLP_INVALID_ARG, "the stresslet operator is FP64 only");
    mhlp_plan *P = const_cast<mhlp_plan *>(Pc);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = vlen(P);
    std::memset(info, 0, sizeof(*info));
    /* workspace columns: basis V_0..V_R, w, r (cycle residual), two spare
       vectors, and the solve's own x and b; R >= restart is the largest
       restart seen */
    TRY(ensure_gdev(P, opts->restart));
    const int R = P->gdev_R;
    TRY(ensure_ws(P, R + 1));
    const bool mixed = opts->precision == MHLP_MIXED;
    double *xw = P->ws + (int64_t)(R + 5) * N, *bw = P->ws + (int64_t)(R + 6) * N;
    /* a solve from zero forms ||g|| on the device and reads it with the first
       read of the GMRES state (one host round trip fewer); the others need it
       now */
    const bool bnorm_dev = !opts->use_x0 && opts->tol < 1.0;
    double bnorm = 0.0;
    if (!bnorm_dev) TRY(dnorm(P, g, N, st, &bnorm));
    info->used_x0 = opts->use_x0 ? 1 : 0;
    if (!bnorm_dev && bnorm == 0.0) {
        fill_kernel<<<nblocks(N, 256), 256, 0, st>>>(mu, 0.0, N);
        HIPCHECK(hipStreamSynchronize(st));
        info->converged = 1;
        return MHLP_OK;
    }
    /* residual of the initial guess (FP64 operator), kept in the residual slot
       of the first GMRES cycle (basis V_0..V_R, then w, r) so the cycle does
       not recompute it */
    double *r0 = P->ws + (int64_t)(R + 2) * N;
    double r0n = 0.0;
    if (opts->use_x0) {
        double *w = P->ws + (int64_t)(R + 1) * N;
        TRY(apply_op(P, mu, w, MHLP_FP64, st));
        residual_kernel<<<nblocks(N, 256), 256, 0, st>>>(g, w, r0, N);
        TRY(dnorm(P, r0, N, st, &r0n));
        info->x0_residual = r0n / bnorm;
        if (!(info->x0_residual < 1.0)) {
            fill_kernel<<<nblocks(N, 256), 256, 0, st>>>(xw, 0.0, N);
            info->used_x0 = 0;
        } else {
            HIPCHECK(hipMemcpyAsync(xw, mu, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        }
    } else {
        if (!bnorm_dev) fill_kernel<<<nblocks(N, 256), 256, 0, st>>>(xw, 0.0, N);
        info->x0_residual = 1.0;
    }
    int iters = 0, cycles = 0;
    double rel = 1.0;
    /* the solve runs on its own copies of g and mu (xw, bw), which the captured
       graphs refer to; the start kernel of a device-normed solve makes them,
       else they are copied here.  Mixed precision: Arnoldi steps on the FP32
       far field, each cycle an inner solve to 1e-6 of the residual it started
       from, its end the FP64 true residual (iterative refinement). */
    if (!bnorm_dev) HIPCHECK(hipMemcpyAsync(bw, g, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    TRY(gmres_core(P, bw, bnorm, xw, opts->tol, opts->restart, opts->max_iter, mixed ? MHLP_MIXED : MHLP_FP64, st,
                   &iters, &cycles, &rel, info->used_x0 ? r0 : bw, info->used_x0 ? r0n : bnorm, bnorm_dev, g, mu,
                   mixed ? 0.5e-6 : 0.0));
    /* every cycle's end copies x into mu; without a cycle x is the start */
    if (cycles == 0) HIPCHECK(hipMemcpyAsync(mu, xw, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    info->iters = iters;
    info->restarts = cycles;
    info->rel_residual = rel;
    info->converged = rel <= opts->tol ? 1 : 0;
    return info->converged ? MHLP_OK : MHLP_NOT_CONVERGED;
}

extern "C" mhlp_status mhlp_gmres_solve(const mhlp_plan *P, const double *g, double *mu, const mhlp_gmres_opts *opts,
                                        mhlp_gmres_info *info, void *stream)
{
    if (P && P->stokes) return fail(MHLP_INVALID_ARG, "stokes plans solve with mhlp_stokes_gmres_solve");
    return gmres_solve_impl(P, g, mu, opts, info, stream);
}

extern "C" mhlp_status mhlp_stokes_gmres_solve(const mhlp_plan *P, const double *g, double *mu,
                                               const mhlp_gmres_opts *opts, mhlp_gmres_info *info, void *stream)
{
    if (P && !P->stokes) return fail(MHLP_INVALID_ARG, "stokes_gmres_solve needs a plan from mhlp_stokes_plan_create");
    return gmres_solve_impl(P, g, mu, opts, info, stream);
}

/* ------------------------------------------------------------------------ */
/* volume API                                                                */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* FMM far field: plans and the volume sum                                   */
/* ------------------------------------------------------------------------ */
template <class T>
static mhlp_status to_host(std::vector<T> &h, const T *d, int64_t n, hipStream_t st)
{
    h.resize(n);
    if (n == 0) return MHLP_OK;
    hipError_t e = hipMemcpyAsync(h.data(), d, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("copy to host: ") + hipGetErrorString(e));
    return MHLP_OK;
}

static int fmm_auto_level(int64_t npts, int64_t per_leaf)
{
    int L = 0;
    while (L < 8 && ((int64_t)1 << (2 * L)) * per_leaf < npts) ++L;
    return L;
}

extern "C" mhlp_status mhlp_plan_set_fmm(mhlp_plan *P, int32_t order, int32_t leaf_level, void *stream)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (order == 0) {
        delete P->fmm;
        P->fmm = nullptr;
        return MHLP_OK;
    }
    if (P->stokes) return fail(MHLP_INVALID_ARG, "the FMM serves scalar plans");
    if (P->onsurf) return fail(MHLP_UNSUPPORTED, "the FMM serves off-surface plans");
    if (order < 4 || order > mhlp::FMM_PMAX) return fail(MHLP_INVALID_ARG, "order must be 0 or in [4, 60]");
    if (leaf_level < -1 || leaf_level > mhlp::FMM_LMAX) return fail(MHLP_INVALID_ARG, "leaf_level must be -1 or in [0, 10]");
    hipStream_t st = (hipStream_t)stream;
    const mhlp_geometry *g = P->g;
    std::vector<double> sx, sy, tx, ty;
    std::vector<int32_t> nptr, npan;
    TRY(to_host(sx, g->soa, g->N, st));
    TRY(to_host(sy, g->soa + g->N, g->N, st));
    TRY(to_host(tx, P->tx, P->M, st));
    TRY(to_host(ty, P->ty, P->M, st));
    TRY(to_host(nptr, P->near_ptr, P->M + 1, st));
    TRY(to_host(npan, P->near_panel, P->nnz, st));
    const FmmGeom G = fmm_root(sx, sy, tx, ty);
    int L = leaf_level;
    if (L < 0) {
        L = fmm_auto_level(P->M + g->N, 32);
        while (L > 0 && !fmm_contains_near(G, L, sx, sy, tx, ty, nptr, npan)) --L;
    } else if (!fmm_contains_near(G, L, sx, sy, tx, ty, nptr, npan)) {
        return fail(MHLP_INVALID_ARG, "leaf_level too fine: a near panel reaches beyond a target's 3x3 leaf neighbourhood");
    }
    FmmTree *F = new FmmTree();
    mhlp_status s = fmm_build(F, G, L, order, P->alpha, sx, sy, tx, ty, false, g->soa, g->soa + g->N, g->w, g->nx,
                              g->ny, st);
    if (s != MHLP_OK) {
        delete F;
        return s;
    }
    delete P->fmm;
    P->fmm = F;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_plan_get_fmm(const mhlp_plan *P, int32_t *order, int32_t *leaf_level)
{
    if (!P) return fail(MHLP_INVALID_ARG, "plan is NULL");
    if (order) *order = P->fmm ? P->fmm->order : 0;
    if (leaf_level) *leaf_level = P->fmm ? P->fmm->level : -1;
    return MHLP_OK;
}

struct mhlp_volume_fmm {
    FmmTree tree;
    int64_t n = 0;
    double alpha = 0.0, h = 0.0, selfc = 0.0, wcell = 0.0;
};

static mhlp_status self_cell_value(double alpha, double h, hipStream_t st, double *wc)
{
    double *dev = nullptr;
    TRY(dalloc(&dev, 1));
    self_cell_kernel<<<1, 64, 0, st>>>(alpha, h, dev, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(wc, dev, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("volume self cell: ") + hipGetErrorString(e));
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_volume_fmm_create(const double *x, const double *y, const double *w, int64_t n,
                                              double alpha, double h, int32_t order, int32_t leaf_level, void *stream,
                                              mhlp_volume_fmm **out)
{
    if (!out) return fail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!x || !y || !w) return fail(MHLP_INVALID_ARG, "NULL argument");
    if (n < 1 || n > INT_MAX - 1) return fail(MHLP_INVALID_ARG, "n out of range");
    if (!(alpha > 0.0) || !std::isfinite(alpha) || !(h > 0.0)) return fail(MHLP_INVALID_ARG, "alpha and h must be > 0");
    if (order < 4 || order > mhlp::FMM_PMAX) return fail(MHLP_INVALID_ARG, "order must be in [4, 60]");
    if (leaf_level < -1 || leaf_level > mhlp::FMM_LMAX) return fail(MHLP_INVALID_ARG, "leaf_level must be -1 or in [0, 10]");
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> hx, hy;
    TRY(to_host(hx, x, n, st));
    TRY(to_host(hy, y, n, st));
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(hx[k]) || !std::isfinite(hy[k])) return fail(MHLP_INVALID_ARG, "coordinates must be finite");
    const std::vector<double> none;
    const FmmGeom G = fmm_root(hx, hy, none, none);
    const int L = leaf_level < 0 ? fmm_auto_level(n, 64) : leaf_level;
    mhlp_volume_fmm *V = new mhlp_volume_fmm();
    V->n = n;
    V->alpha = alpha;
    V->h = h;
    mhlp_status s = self_cell_value(alpha, h, st, &V->wcell);
    if (s == MHLP_OK) s = fmm_build(&V->tree, G, L, order, alpha, hx, hy, none, none, true, x, y, w, nullptr, nullptr, st);
    if (s != MHLP_OK) {
        delete V;
        return s;
    }
    V->selfc = V->wcell / (h * h);
    *out = V;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_volume_fmm_eval(const mhlp_volume_fmm *V, const double *f, double *u, void *stream)
{
    if (!V) return fail(MHLP_INVALID_ARG, "volume FMM is NULL");
    if (!f || !u) return fail(MHLP_INVALID_ARG, "f or u is NULL");
    if (f == u) return fail(MHLP_INVALID_ARG, "f and u must not alias");
    hipStream_t st = (hipStream_t)stream;
    const FmmTree *F = &V->tree;
    fmm_passes<true, false>(F, f, nullptr, st);
    FarArgs A{};
    mhlp::FmmVol vol{f, V->selfc, u};
    if (F->d.nwork > 0)
        mhlp::fmm_leaf_kernel<true, false, 1><<<(unsigned)F->d.nwork, 64 * mhlp::FMM_LW, 0, st>>>(F->d, A, vol);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_volume_fmm_info(const mhlp_volume_fmm *V, int32_t *order, int32_t *leaf_level,
                                            double *self_cell)
{
    if (!V) return fail(MHLP_INVALID_ARG, "volume FMM is NULL");
    if (order) *order = V->tree.order;
    if (leaf_level) *leaf_level = V->tree.level;
    if (self_cell) *self_cell = V->wcell;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_volume_fmm_destroy(mhlp_volume_fmm *V)
{
    delete V;
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* particular solution on a periodic box                                     */
/* ------------------------------------------------------------------------ */
struct mhlp_box {
    int M = 0;
    double x0 = 0.0, y0 = 0.0, Lb = 0.0, alpha = 0.0;
    cplx *tw = nullptr;   /* M/2 twiddles */
    cplx *spec = nullptr; /* [2][M^2] forcing spectra */
    cplx *uh = nullptr;   /* [6][M^2] u^_1, u^_2 and the four gradient spectra */
    double *part = nullptr;
    int64_t part_cap = 0;
    double *sdc = nullptr; /* SISDC workspace */
    int64_t sdc_cap = 0;
    int point_method = 1;  /* 0: direct type-2 sums, 1: non-uniform FFT */
    cplx *twf = nullptr;   /* NUFFT: twiddles of the fine size 2M */
    double *corr = nullptr; /* NUFFT: hf / psi^(k_j), coarse FFT order */
    cplx *fine = nullptr;  /* NUFFT: [2][(2M)^2] */
    ~mhlp_box()
    {
        for (void *q : {(void *)tw, (void *)spec, (void *)uh, (void *)part, (void *)sdc, (void *)twf, (void *)corr,
                        (void *)fine})
            if (q) (void)hipFree(q);
    }
};

/* NUFFT tables of the box: fine twiddles and the deconvolution factors
   hf/psi^(k) with psi^(k) = (W hf/2) int_{-1}^{1} phi(z) cos(k W hf z/2) dz by
   composite 32-point Gauss-Legendre quadrature on 16 panels */
static mhlp_status box_nufft_setup(mhlp_box *B, hipStream_t st)
{
    if (B->fine) return MHLP_OK;
    const int M = B->M, Mf = 2 * M;
    const double hf = B->Lb / Mf, half = 0.5 * mhlp::NU_W * hf;
    std::vector<cplx> twf(Mf / 2);
    for (int j = 0; j < Mf / 2; ++j) {
        const double a = 2.0 * PI * (double)j / (double)Mf;
        twf[j] = mk(std::cos(a), -std::sin(a));
    }
    std::vector<double> corr(M);
    for (int j = 0; j < M; ++j) {
        const double k = 2.0 * PI / B->Lb * (j < M / 2 ? j : j - M);
        double s = 0.0;
        for (int pnl = 0; pnl < 16; ++pnl) {
            const double a = -1.0 + pnl * 0.125, b = a + 0.125;
            for (int q = 0; q < 32; ++q) {
                const double z = 0.5 * (a + b) + 0.5 * (b - a) * GL32_T[q];
                const double qz = 1.0 - z * z;
                const double ph = qz > 0.0 ? std::exp(mhlp::NU_BETA * (std::sqrt(qz) - 1.0)) : 0.0;
                s += 0.5 * (b - a) * GL32_W[q] * ph * std::cos(k * half * z);
            }
        }
        corr[j] = hf / (half * s);
    }
    cplx *d_twf = nullptr, *d_fine = nullptr;
    double *d_corr = nullptr;
    mhlp_status s = dalloc(&d_twf, Mf / 2);
    if (s == MHLP_OK) s = dalloc(&d_corr, M);
    if (s == MHLP_OK) s = dalloc(&d_fine, 2 * (int64_t)Mf * Mf);
    hipError_t e = hipSuccess;
    if (s == MHLP_OK) {
        e = hipMemcpyAsync(d_twf, twf.data(), sizeof(cplx) * twf.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_corr, corr.data(), sizeof(double) * M, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = fail(MHLP_HIP_ERROR, std::string("box NUFFT tables: ") + hipGetErrorString(e));
    }
    if (s != MHLP_OK) { /* nothing half-built stays behind */
        for (void *q : {(void *)d_twf, (void *)d_corr, (void *)d_fine})
            if (q) (void)hipFree(q);
        return s;
    }
    B->twf = d_twf;
    B->corr = d_corr;
    B->fine = d_fine;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_box_set_point_method(mhlp_box *B, int32_t method)
{
    if (!B) return fail(MHLP_INVALID_ARG, "box is NULL");
    if (method != 0 && method != 1) return fail(MHLP_INVALID_ARG, "method must be 0 (direct) or 1 (NUFFT)");
    if (method == 1 && B->M > 1024) return fail(MHLP_INVALID_ARG, "the NUFFT serves boxes with M <= 1024");
    B->point_method = method;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_box_create(int32_t M, double x0, double y0, double Lb, double alpha, void *stream,
                                       mhlp_box **out)
{
    if (!out) return fail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (M < 16 || M > 2048 || (M & (M - 1))) return fail(MHLP_INVALID_ARG, "M must be a power of two in [16, 2048]");
    if (!std::isfinite(x0) || !std::isfinite(y0) || !(Lb > 0.0) || !std::isfinite(Lb))
        return fail(MHLP_INVALID_ARG, "box corner must be finite and Lb > 0");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(MHLP_INVALID_ARG, "alpha must be finite and > 0");
    mhlp_box *B = new mhlp_box();
    B->M = M;
    B->x0 = x0;
    B->y0 = y0;
    B->Lb = Lb;
    B->alpha = alpha;
    B->point_method = M <= 1024 ? 1 : 0;
    const int64_t MM = (int64_t)M * M;
    mhlp_status s;
    if ((s = dalloc(&B->tw, M / 2)) || (s = dalloc(&B->spec, 2 * MM)) || (s = dalloc(&B->uh, 6 * MM))) {
        delete B;
        return s;
    }
    std::vector<cplx> tw(M / 2);
    for (int j = 0; j < M / 2; ++j) {
        const double a = 2.0 * PI * (double)j / (double)M;
        tw[j] = mk(std::cos(a), -std::sin(a));
    }
    hipError_t e = hipMemcpyAsync(B->tw, tw.data(), sizeof(cplx) * tw.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        delete B;
        return fail(MHLP_HIP_ERROR, std::string("box_create: ") + hipGetErrorString(e));
    }
    *out = B;
    return MHLP_OK;
}

static void fft2_fields(const mhlp_box *B, cplx *data, int nf, double sign, hipStream_t st)
{
    const int M = B->M;
    const int64_t MM = (int64_t)M * M;
    const size_t sh = sizeof(cplx) * 2 * (size_t)M;
    mhlp::fft_lines_kernel<<<dim3(M, nf), M / 2, sh, st>>>(data, M, 1, M, MM, B->tw, sign); /* rows (x) */
    mhlp::fft_lines_kernel<<<dim3(M, nf), M / 2, sh, st>>>(data, M, M, 1, MM, B->tw, sign); /* columns (y) */
}

extern "C" mhlp_status mhlp_box_particular(mhlp_box *B, const double *F, double *u, double *grad, int64_t n,
                                           const double *px, const double *py, double *up, void *stream)
{
    if (!B) return fail(MHLP_INVALID_ARG, "box is NULL");
    if (!F) return fail(MHLP_INVALID_ARG, "F is NULL");
    if (n < 0 || n > INT_MAX) return fail(MHLP_INVALID_ARG, "n out of range");
    if (n > 0 && (!px || !py || !up)) return fail(MHLP_INVALID_ARG, "points need px, py and up");
    if (!u && !grad && n == 0) return fail(MHLP_INVALID_ARG, "no output requested");
    hipStream_t st = (hipStream_t)stream;
    const int M = B->M;
    const int64_t MM = (int64_t)M * M;
    mhlp::fft_load_real_kernel<<<nblocks(2 * MM, 256), 256, 0, st>>>(F, 2 * MM, B->spec);
    fft2_fields(B, B->spec, 2, -1.0, st);
    mhlp::stokes_multiplier_kernel<<<nblocks(MM, 256), 256, 0, st>>>(B->spec, M, B->Lb, B->alpha, grad != nullptr,
                                                                     B->uh);
    if (n > 0 && B->point_method == 1) {
        TRY(box_nufft_setup(B, st));
        const int Mf = 2 * M;
        const int64_t MMf = (int64_t)Mf * Mf;
        mhlp::nufft_fine_spectrum_kernel<<<nblocks(2 * MMf, 256), 256, 0, st>>>(B->uh, M, Mf, B->corr, B->fine);
        const size_t sh = sizeof(cplx) * 2 * (size_t)Mf;
        mhlp::fft_lines_kernel<<<dim3(Mf, 2), Mf / 2, sh, st>>>(B->fine, Mf, 1, Mf, MMf, B->twf, 1.0);
        mhlp::fft_lines_kernel<<<dim3(Mf, 2), Mf / 2, sh, st>>>(B->fine, Mf, Mf, 1, MMf, B->twf, 1.0);
        mhlp::nufft_interp_kernel<<<nblocks(n, 128), 128, 0, st>>>(B->fine, Mf, B->Lb / Mf, B->x0, B->y0, px, py, n,
                                                                  up);
    } else if (n > 0) {
        const int nchunk = M / mhlp::FT2_R;
        const int64_t need = 2 * (int64_t)nchunk * n;
        if (need > B->part_cap) {
            HIPCHECK(hipStreamSynchronize(st));
            if (B->part) (void)hipFree(B->part);
            B->part = nullptr;
            B->part_cap = 0;
            TRY(dalloc(&B->part, need));
            B->part_cap = need;
        }
        mhlp::type2_points_kernel<<<dim3(nblocks(n, mhlp::FT2_T), nchunk), mhlp::FT2_T, 0, st>>>(
            B->uh, M, B->Lb, B->x0, B->y0, px, py, n, B->part);
        mhlp::type2_reduce_kernel<<<nblocks(n, 256), 256, 0, st>>>(B->part, nchunk, n, up);
    }
    if (u) {
        fft2_fields(B, B->uh, 2, 1.0, st);
        mhlp::fft_store_real_kernel<<<nblocks(2 * MM, 256), 256, 0, st>>>(B->uh, 2 * MM, u);
    }
    if (grad) {
        fft2_fields(B, B->uh + 2 * MM, 4, 1.0, st);
        mhlp::fft_store_real_kernel<<<nblocks(4 * MM, 256), 256, 0, st>>>(B->uh + 2 * MM, 4 * MM, grad);
    }
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_box_destroy(mhlp_box *B)
{
    delete B;
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* SISDC time step of the Navier-Stokes equations on the periodic box         */
/* ------------------------------------------------------------------------ */
/* q[m][j] = (1/dts) int_{t_m}^{t_{m+1}} l_j(t) dt, t_i = i dts: the Lagrange basis
   polynomial of node j expanded in monomials and integrated exactly */
static void sisdc_weights(int p, std::vector<double> &q)
{
    q.assign((size_t)p * (p + 1), 0.0);
    for (int j = 0; j <= p; ++j) {
        std::vector<double> c(1, 1.0); /* coefficients of prod_{i != j} (t - i)/(j - i), ascending */
        for (int i = 0; i <= p; ++i) {
            if (i == j) continue;
            std::vector<double> nc(c.size() + 1, 0.0);
            for (size_t d = 0; d < c.size(); ++d) {
                nc[d + 1] += c[d] / (double)(j - i);
                nc[d] -= c[d] * (double)i / (double)(j - i);
            }
            c.swap(nc);
        }
        for (int m = 0; m < p; ++m) {
            double s = 0.0;
            for (size_t d = 0; d < c.size(); ++d)
                s += c[d] * (std::pow((double)(m + 1), (double)(d + 1)) - std::pow((double)m, (double)(d + 1))) /
                     (double)(d + 1);
            q[(size_t)m * (p + 1) + j] = s;
        }
    }
}

static void lincomb(const std::vector<std::pair<double, const double *>> &terms, int64_t n, double *out,
                    hipStream_t st)
{
    mhlp::LinComb T{};
    T.nterm = (int)terms.size();
    for (int k = 0; k < T.nterm; ++k) {
        T.c[k] = terms[k].first;
        T.x[k] = terms[k].second;
    }
    mhlp::lincomb_kernel<<<nblocks(n, 256), 256, 0, st>>>(T, n, out);
}

extern "C" mhlp_status mhlp_sisdc_step(mhlp_box *B, double Re, double dt, int32_t K, double *u, double *grad,
                                       double *lap, void *stream)
{
    if (!B) return fail(MHLP_INVALID_ARG, "box is NULL");
    if (!u || !grad || !lap) return fail(MHLP_INVALID_ARG, "u, grad and lap are required");
    if (K < 2 || K > 5) return fail(MHLP_INVALID_ARG, "K must be in [2, 5]");
    if (!(Re > 0.0) || !(dt > 0.0) || !std::isfinite(Re) || !std::isfinite(dt))
        return fail(MHLP_INVALID_ARG, "Re and dt must be finite and > 0");
    const int p = K - 1;
    const double dts = dt / p, a2 = Re / dts;
    if (std::fabs(B->alpha * B->alpha - a2) > 1e-12 * a2)
        return fail(MHLP_INVALID_ARG, "the box's alpha must satisfy alpha^2 = Re K'/dt, K' = K - 1 substeps");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n2 = 2 * (int64_t)B->M * B->M;
    /* workspace: N, L of the previous sweep, U, N, L of the new one (p + 1 each), F */
    const int64_t need = (5 * (int64_t)(p + 1) + 1) * n2;
    if (need > B->sdc_cap) {
        HIPCHECK(hipStreamSynchronize(st));
        if (B->sdc) (void)hipFree(B->sdc);
        B->sdc = nullptr;
        B->sdc_cap = 0;
        TRY(dalloc(&B->sdc, need));
        B->sdc_cap = need;
    }
    double *w = B->sdc;
    auto slot = [&](int k) { return w + (int64_t)k * n2; };
    std::vector<double *> No(p + 1), Lo(p + 1), Un(p + 1), Nn(p + 1), Ln(p + 1);
    for (int m = 0; m <= p; ++m) {
        No[m] = slot(m);
        Lo[m] = slot(p + 1 + m);
        Un[m] = slot(2 * (p + 1) + m);
        Nn[m] = slot(3 * (p + 1) + m);
        Ln[m] = slot(4 * (p + 1) + m);
    }
    double *F = slot(5 * (p + 1));
    std::vector<double> q;
    sisdc_weights(p, q);
    const unsigned nb = nblocks(n2 / 2, 256);
    /* start of the step: u0, N0 = (u0.grad) u0, L0 = lap */
    HIPCHECK(hipMemcpyAsync(Un[0], u, sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
    mhlp::advect_kernel<<<nb, 256, 0, st>>>(u, grad, n2 / 2, Nn[0]);
    HIPCHECK(hipMemcpyAsync(Ln[0], lap, sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
    auto solve_into = [&](int m) -> mhlp_status {
        /* (alpha^2 - Delta) U_{m+1} + Re grad p = F; N_{m+1}, L_{m+1} = alpha^2 U_{m+1} - F */
        TRY(mhlp_box_particular(B, F, Un[m + 1], grad, 0, nullptr, nullptr, nullptr, stream));
        mhlp::advect_kernel<<<nb, 256, 0, st>>>(Un[m + 1], grad, n2 / 2, Nn[m + 1]);
        lincomb({{a2, Un[m + 1]}, {-1.0, F}}, n2, Ln[m + 1], st);
        return MHLP_OK;
    };
    for (int m = 0; m < p; ++m) { /* first sweep: implicit-explicit Euler */
        lincomb({{a2, Un[m]}, {-Re, Nn[m]}}, n2, F, st);
        TRY(solve_into(m));
    }
    for (int k = 1; k < K; ++k) { /* corrections */
        std::swap(No, Nn);
        std::swap(Lo, Ln);
        /* the new sweep starts from the same initial values */
        HIPCHECK(hipMemcpyAsync(Nn[0], No[0], sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
        HIPCHECK(hipMemcpyAsync(Ln[0], Lo[0], sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
        for (int m = 0; m < p; ++m) {
            std::vector<std::pair<double, const double *>> t = {
                {a2, Un[m]}, {-Re, Nn[m]}, {Re, No[m]}, {-1.0, Lo[m + 1]}};
            for (int j = 0; j <= p; ++j) {
                t.push_back({q[(size_t)m * (p + 1) + j], Lo[j]});
                t.push_back({-Re * q[(size_t)m * (p + 1) + j], No[j]});
            }
            lincomb(t, n2, F, st);
            TRY(solve_into(m));
        }
    }
    HIPCHECK(hipMemcpyAsync(u, Un[p], sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipMemcpyAsync(lap, Ln[p], sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* Launch shape of the volume sum: one thread per target in blocks of
   FT_THREADS; when that leaves fewer than 1024 blocks the sources are split
   into ranges of whole LDS tiles evaluated by separate blocks (partials
   [nsplit][n], summed in fixed order by volume_finalize).  Returns nsplit. */
static int volume_shape(VolArgs &A)
{
    const int64_t n = A.n;
    const int64_t tblocks = (n + FT_THREADS - 1) / FT_THREADS;
    int64_t ns = (1024 + tblocks - 1) / tblocks;
    if (ns > (n + FT_SRC - 1) / FT_SRC) ns = (n + FT_SRC - 1) / FT_SRC;
    if (ns < 1) ns = 1;
    A.per_split = ((n + ns - 1) / ns + FT_SRC - 1) / FT_SRC * FT_SRC;
    return (int)((n + A.per_split - 1) / A.per_split);
}

static void volume_launch(const VolArgs &A, int nsplit, int32_t precision, hipStream_t st)
{
    const unsigned tblocks = (unsigned)((A.n + FT_THREADS - 1) / FT_THREADS);
    if (nsplit > 1) {
        dim3 grid(tblocks, nsplit);
        if (precision == MHLP_MIXED)
            volume_kernel<true, true><<<grid, FT_THREADS, 0, st>>>(A);
        else
            volume_kernel<false, true><<<grid, FT_THREADS, 0, st>>>(A);
        volume_finalize<<<nblocks(A.n, 256), 256, 0, st>>>(A, nsplit);
    } else if (precision == MHLP_MIXED) {
        volume_kernel<true, false><<<tblocks, FT_THREADS, 0, st>>>(A);
    } else {
        volume_kernel<false, false><<<tblocks, FT_THREADS, 0, st>>>(A);
    }
}

static mhlp_status volume_check(const double *x, const double *y, const double *w, const double *f, int64_t n,
                                double alpha, double h, int32_t precision, const double *u)
{
    if (!x || !y || !w || !f || !u) return fail(MHLP_INVALID_ARG, "NULL argument");
    if (n < 1) return fail(MHLP_INVALID_ARG, "n must be >= 1");
    if (!(alpha > 0.0) || !std::isfinite(alpha) || !(h > 0.0)) return fail(MHLP_INVALID_ARG, "alpha and h must be > 0");
    if (precision != MHLP_FP64 && precision != MHLP_MIXED) return fail(MHLP_INVALID_ARG, "unknown precision");
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_volume_eval(const double *x, const double *y, const double *w, const double *f, int64_t n,
                                        double alpha, double h, int32_t precision, double *u, double *self_cell,
                                        void *stream)
{
    TRY(volume_check(x, y, w, f, n, alpha, h, precision, u));
    hipStream_t st = (hipStream_t)stream;
    double *dev = nullptr;
    TRY(dalloc(&dev, 1));
    self_cell_kernel<<<1, 64, 0, st>>>(alpha, h, dev, nullptr);
    double wc = 0.0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&wc, dev, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("volume self cell: ") + hipGetErrorString(e));
    if (self_cell) *self_cell = wc;
    VolArgs A;
    A.x = x;
    A.y = y;
    A.w = w;
    A.f = f;
    A.n = n;
    A.alpha = alpha;
    A.selfc = wc / (h * h);
    A.u = u;
    A.selfc_dev = nullptr;
    A.part = nullptr;
    const int nsplit = volume_shape(A);
    if (nsplit > 1) {
        TRY(dalloc(&A.part, (int64_t)nsplit * n));
        volume_launch(A, nsplit, precision, st);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(A.part);
        if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("volume_eval: ") + hipGetErrorString(e));
        return MHLP_OK;
    }
    volume_launch(A, nsplit, precision, st);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* Fixed device scratch of the allocation-free volume sum, one copy per device
   (a file-scope device array lives in every device's copy of the code
   object).  Slot 0 holds Wcell/h^2; the split partials start at VOL_HEAD.
   volume_shape() never needs more than 523,776 partial values (nsplit = 2 at
   n = 261,888), below VOL_PART_MAX.  Host code must not pass `scratch` itself
   to a kernel: it names a host-side stand-in; the device address comes from
   hipGetSymbolAddress, once per device. */
constexpr int64_t VOL_HEAD = 32; /* doubles: keeps the partials 256-byte aligned */
constexpr int64_t VOL_PART_MAX = (int64_t)1 << 19;
static __device__ __align__(256) double scratch[VOL_HEAD + VOL_PART_MAX];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[SCRATCH_MAX_DEVICES];

/* Device address of `scratch` on the current device (looked up on the first
   call per device, then reused). */
static mhlp_status scratch_address(double **out)
{
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(MHLP_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MHLP_HIP_ERROR, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_volume_eval_noalloc(const double *x, const double *y, const double *w, const double *f,
                                                int64_t n, double alpha, double h, int32_t precision, double *u,
                                                void *stream)
{
    TRY(volume_check(x, y, w, f, n, alpha, h, precision, u));
    hipStream_t st = (hipStream_t)stream;
    VolArgs A;
    A.x = x;
    A.y = y;
    A.w = w;
    A.f = f;
    A.n = n;
    A.alpha = alpha;
    A.selfc = 0.0;
    A.u = u;
    const int nsplit = volume_shape(A);
    if (nsplit > 1 && (int64_t)nsplit * n > VOL_PART_MAX)
        return fail(MHLP_INVALID_ARG, "volume_eval_noalloc: partial sums exceed the fixed scratch (" +
                                          std::to_string(VOL_PART_MAX) + " values)");
    double *S = nullptr;
    TRY(scratch_address(&S));
    A.selfc_dev = S;
    A.part = nsplit > 1 ? S + VOL_HEAD : nullptr;
    /* slot 0 and every partial are written before they are read: nothing to clear */
    self_cell_kernel<<<1, 64, 0, st>>>(alpha, h, nullptr, S);
    volume_launch(A, nsplit, precision, st);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* batched on-surface operator and lockstep GMRES over many geometries and   */
/* right-hand sides                                                          */
/*                                                                           */
/* Batched vector layout: for each geometry g, a block [R][N_g] at offset     */
/* voff_g (R right-hand sides of the same geometry are contiguous systems).   */
/* One grouped launch applies (1/2 I + D) to every system: each block owns    */
/* (geometry, target tile, source split); every kernel value is shared by the */
/* R right-hand sides of its geometry.                                        */
/* ------------------------------------------------------------------------ */
constexpr int BATCH_R_MAX = 4;

struct BatchGeo {
    const double *x, *y, *w, *nx, *ny;
    const int32_t *nptr, *npan;
    const double *wdl;
    int64_t N, Np;
    double alpha;
    int64_t voff; /* offset of the geometry's [R][N] block in batched vectors */
    int64_t poff; /* offset of its partial sums [nsplit][R][N]                 */
    int32_t nsplit, pps;
};

struct BatchWork {
    int32_t g, tb, split, pad;
};

/* A geometry takes part in a batched operator application unless a gate is
   given and all its right-hand sides are gated off (gate[g*R + r] == 0:
   systems that have converged in the current GMRES cycle). */
template <int R>
__device__ __forceinline__ bool batch_gated_off(const double *__restrict__ gate, int g)
{
    if (!gate) return false;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (gate[(int64_t)g * R + r] != 0.0) return false;
    return true;
}

/* Device state of a lockstep batched GMRES cycle. */
struct BState {
    int32_t j;     /* current Arnoldi column (common to all systems)         */
    int32_t kmax;  /* columns allowed in this cycle                          */
    int32_t done;  /* all systems converged / broken down, or kmax reached   */
    int32_t nact;  /* systems still active after the last step               */
    int32_t steps; /* lockstep steps taken in this cycle                     */
    int32_t pad[3];
};

/* density of a batched launch: fixed, or basis column bs->j; false = no-op */
__device__ __forceinline__ bool batch_density(const BState *bs, int64_t jstride, const double *__restrict__ &mu)
{
    if (bs) {
        if (bs->done) return false;
        mu += (int64_t)bs->j * jstride;
    }
    return true;
}

/* The batched far field of one work item (geometry g, target tile tb, source
   split): TPL targets per lane (tile of FT_THREADS * TPL targets; lane t takes
   t, t + FT_THREADS, ...), sources staged in LDS SRC at a time (a multiple of
   16), R right-hand sides sharing every kernel value; a target skips the
   panels it lists as near.  Partial sums per (split, right-hand side, node). */
template <int R, int TPL, int SRC>
__global__ __launch_bounds__(FT_THREADS) void batch_far_dlp(const BatchGeo *__restrict__ G,
                                                            const BatchWork *__restrict__ W,
                                                            const double *__restrict__ mu, double *__restrict__ part,
                                                            const double *__restrict__ gate, const BState *bs,
                                                            int64_t jstride)
{
    static_assert(SRC % 16 == 0 && SRC <= FT_THREADS, "whole panels, one source per thread");
    if (batch_gated_off<R>(gate, W[blockIdx.x].g) || !batch_density(bs, jstride, mu)) return;
    __shared__ double lx[SRC], ly[SRC];
    __shared__ double ldx[R][SRC], ldy[R][SRC];
    const BatchWork wk = W[blockIdx.x];
    const BatchGeo geo = G[wk.g];
    const int64_t pb = (int64_t)wk.split * geo.pps;
    const int64_t pe = min(geo.Np, pb + geo.pps);
    int64_t i[TPL];
    bool valid[TPL];
    double x[TPL], y[TPL];
    int32_t k[TPL], kend[TPL], nxt[TPL];
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
        i[q] = (int64_t)wk.tb * (FT_THREADS * TPL) + q * FT_THREADS + threadIdx.x;
        valid[q] = i[q] < geo.N;
        x[q] = valid[q] ? geo.x[i[q]] : 0.0;
        y[q] = valid[q] ? geo.y[i[q]] : 0.0;
        k[q] = kend[q] = 0;
        if (valid[q]) {
            k[q] = geo.nptr[i[q]];
            kend[q] = geo.nptr[i[q] + 1];
            while (k[q] < kend[q] && geo.npan[k[q]] >= 0 && geo.npan[k[q]] < pb) ++k[q];
        }
        nxt[q] = (k[q] < kend[q]) ? geo.npan[k[q]] : INT_MAX;
    }
    const FarConst fc = far_const(geo.alpha);
    const double *mug = mu + geo.voff;
    double acc[TPL][R];
#pragma unroll
    for (int q = 0; q < TPL; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[q][r] = 0.0;
    for (int64_t base = 16 * pb; base < 16 * pe; base += SRC) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (threadIdx.x < SRC && j < 16 * pe) {
            const double wj = geo.w[j];
            lx[threadIdx.x] = geo.x[j];
            ly[threadIdx.x] = geo.y[j];
            const double nxj = geo.nx[j], nyj = geo.ny[j];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double m = (geo.alpha * wj) * mug[r * geo.N + j]; /* the pair gives K1(z)/r */
                ldx[r][threadIdx.x] = m * nxj;
                ldy[r][threadIdx.x] = m * nyj;
            }
        }
        __syncthreads();
        const int32_t p0 = (int32_t)(base / 16);
        const int npl = (pe - p0) < SRC / 16 ? (int)(pe - p0) : SRC / 16;
        for (int pl = 0; pl < npl; ++pl) {
            bool use[TPL];
            bool any = false;
#pragma unroll
            for (int q = 0; q < TPL; ++q) {
                use[q] = p0 + pl != nxt[q];
                if (!use[q]) {
                    ++k[q];
                    nxt[q] = (k[q] < kend[q]) ? geo.npan[k[q]] : INT_MAX;
                }
                any = any || use[q];
            }
            if (!any) continue;
#pragma unroll 1
            for (int s = 0; s < 16; s += 2) {
                const FarTab T = far_table();
                const int l0 = pl * 16 + s, l1 = l0 + 1;
#pragma unroll
                for (int q = 0; q < TPL; ++q) {
                    if (!use[q]) continue;
                    const double ex0 = x[q] - lx[l0], ey0 = y[q] - ly[l0];
                    const double ex1 = x[q] - lx[l1], ey1 = y[q] - ly[l1];
                    K01 o0, o1;
                    k01_far2<false, true, true, true>(T, fc, fma(ex0, ex0, ey0 * ey0), fma(ex1, ex1, ey1 * ey1), o0,
                                                      o1);
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        acc[q][r] = fma(o1.ak1r, fma(ex1, ldx[r][l1], ey1 * ldy[r][l1]),
                                        fma(o0.ak1r, fma(ex0, ldx[r][l0], ey0 * ldy[r][l0]), acc[q][r]));
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
        if (!valid[q]) continue;
#pragma unroll
        for (int r = 0; r < R; ++r) part[geo.poff + ((int64_t)wk.split * R + r) * geo.N + i[q]] = acc[q][r];
    }
}

/* out = (1/2 I + D) mu for every system: split partials + corrections + identity */
template <int R>
__global__ void batch_finalize(const BatchGeo *__restrict__ G, const BatchWork *__restrict__ W,
                               const double *__restrict__ part, const double *__restrict__ mu,
                               double *__restrict__ out, const double *__restrict__ gate, const BState *bs,
                               int64_t jstride)
{
    if (batch_gated_off<R>(gate, W[blockIdx.x].g) || !batch_density(bs, jstride, mu)) return;
    const BatchWork wk = W[blockIdx.x];
    const BatchGeo geo = G[wk.g];
    const int64_t i = (int64_t)wk.tb * FT_THREADS + threadIdx.x;
    if (i >= geo.N) return;
    const double *mug = mu + geo.voff;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = 0.0;
    for (int sp = 0; sp < geo.nsplit; ++sp)
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] += part[geo.poff + ((int64_t)sp * R + r) * geo.N + i];
    double c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) c[r] = 0.0;
    for (int32_t q = geo.nptr[i]; q < geo.nptr[i + 1]; ++q) {
        const int64_t p = geo.npan[q];
        if (p < 0) continue;
        for (int jj = 0; jj < 16; ++jj) {
            const double wq = geo.wdl[16 * (int64_t)q + jj];
#pragma unroll
            for (int r = 0; r < R; ++r) c[r] = fma(wq, mug[r * geo.N + 16 * p + jj], c[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) out[geo.voff + r * geo.N + i] = fma(INV_2PI, v[r], c[r]) + 0.5 * mug[r * geo.N + i];
}

/* per-system BLAS-1 over batched vectors: system s spans [off[s], off[s] + n[s]) */
__global__ __launch_bounds__(256) void bdot_kernel(const double *__restrict__ V, int64_t ld,
                                                   const double *__restrict__ w, const int64_t *__restrict__ off,
                                                   const int64_t *__restrict__ n, int ldh, double *__restrict__ out)
{
    __shared__ double red[256];
    const int s = blockIdx.x, c = blockIdx.y;
    const double *v = V + c * ld + off[s];
    const double *ww = w + off[s];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n[s]; i += 256) acc = fma(v[i], ww[i], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)s * ldh + c] = red[0];
}

/* w_s -= sum_{c<ncol} h[s][c] V_c  (sign = -1) or x_s += sum_{c<k_s} y[s][c] V_c (sign = +1) */
__global__ void bcombo_kernel(const double *__restrict__ V, int64_t ld, int ncol, const int32_t *__restrict__ kcol,
                              const double *__restrict__ h, int ldh, double sign, double *__restrict__ w,
                              const int64_t *__restrict__ off, const int64_t *__restrict__ n)
{
    const int s = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n[s]) return;
    const int nc = kcol ? kcol[s] : ncol;
    const int64_t e = off[s] + i;
    double acc = w[e];
    for (int c = 0; c < nc; ++c) acc = fma(sign * h[(int64_t)s * ldh + c], V[c * ld + e], acc);
    w[e] = acc;
}

/* out_s = scale[s] * in_s */
__global__ void bscale_kernel(const double *__restrict__ in, const double *__restrict__ scale,
                              double *__restrict__ out, const int64_t *__restrict__ off,
                              const int64_t *__restrict__ n)
{
    const int s = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n[s]) return;
    out[off[s] + i] = scale[s] * in[off[s] + i];
}

/* ---- device-driven lockstep GMRES over the batch (no-ops once done; a
   system with gate[s] == 0 has converged in this cycle and is skipped) ---- */
__global__ __launch_bounds__(256) void bdot_dev_kernel(const BState *__restrict__ bs, const double *__restrict__ V,
                                                       int64_t ld, const double *__restrict__ w,
                                                       const int64_t *__restrict__ off,
                                                       const int64_t *__restrict__ n, int ldh,
                                                       double *__restrict__ out, const double *__restrict__ gate)
{
    const int s = blockIdx.x, c = blockIdx.y;
    if (bs->done || c > bs->j || gate[s] == 0.0) return;
    __shared__ double red[256];
    const double *v = V + c * ld + off[s];
    const double *ww = w + off[s];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n[s]; i += 256) acc = fma(v[i], ww[i], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)s * ldh + c] = red[0];
}

/* w_s -= sum_{c<=j} h[s][c] V_c */
__global__ void bsub_dev_kernel(const BState *__restrict__ bs, const double *__restrict__ V, int64_t ld,
                                const double *__restrict__ h, int ldh, double *__restrict__ w,
                                const int64_t *__restrict__ off, const int64_t *__restrict__ n,
                                const double *__restrict__ gate)
{
    const int s = blockIdx.y;
    if (bs->done || gate[s] == 0.0) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n[s]) return;
    const int nc = bs->j + 1;
    const int64_t e = off[s] + i;
    double acc = w[e];
    for (int c = 0; c < nc; ++c) acc = fma(-h[(int64_t)s * ldh + c], V[c * ld + e], acc);
    w[e] = acc;
}

/* Hessenberg column j of every active system, its Givens rotations, the
   rotated right-hand side and the per-system stopping test; gate[s] becomes
   1/h_{j+1,j} (next basis vector scale) or 0 (converged).  One block. */
__global__ __launch_bounds__(256) void bfinish_kernel(BState *__restrict__ bs, int S, int m, int ldh,
                                                      double *__restrict__ H, double *__restrict__ cs,
                                                      double *__restrict__ sn, double *__restrict__ gv,
                                                      const double *__restrict__ h1, const double *__restrict__ h2,
                                                      const double *__restrict__ hn, const double *__restrict__ thresh,
                                                      double *__restrict__ resest, double *__restrict__ gate,
                                                      int32_t *__restrict__ dk)
{
    __shared__ int cnt[256];
    const bool skip = bs->done != 0;
    const int k = bs->j;
    int mine = 0;
    if (!skip) {
        for (int s = threadIdx.x; s < S; s += 256) {
            if (gate[s] == 0.0) continue;
            double *Hs = H + (int64_t)s * (m + 1) * m, *c_ = cs + (int64_t)s * m, *s_ = sn + (int64_t)s * m;
            double *g_ = gv + (int64_t)s * (m + 1);
            for (int j = 0; j <= k; ++j) Hs[(int64_t)j * m + k] = h1[(int64_t)s * ldh + j] + h2[(int64_t)s * ldh + j];
            const double hk = sqrt(hn[(int64_t)s * ldh]);
            Hs[(int64_t)(k + 1) * m + k] = hk;
            for (int j = 0; j < k; ++j) {
                const double a = Hs[(int64_t)j * m + k], c = Hs[(int64_t)(j + 1) * m + k];
                Hs[(int64_t)j * m + k] = c_[j] * a + s_[j] * c;
                Hs[(int64_t)(j + 1) * m + k] = -s_[j] * a + c_[j] * c;
            }
            const double a = Hs[(int64_t)k * m + k], c = Hs[(int64_t)(k + 1) * m + k];
            const double den = hypot(a, c);
            c_[k] = den > 0.0 ? a / den : 1.0;
            s_[k] = den > 0.0 ? c / den : 0.0;
            Hs[(int64_t)k * m + k] = den;
            Hs[(int64_t)(k + 1) * m + k] = 0.0;
            g_[k + 1] = -s_[k] * g_[k];
            g_[k] = c_[k] * g_[k];
            dk[s] = k + 1;
            resest[s] = fabs(g_[k + 1]);
            if (resest[s] <= thresh[s] || hk == 0.0) {
                gate[s] = 0.0;
            } else {
                gate[s] = 1.0 / hk;
                ++mine;
            }
        }
    }
    cnt[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && !skip) {
        bs->nact = cnt[0];
        bs->steps = k + 1;
        if (cnt[0] == 0 || k + 1 >= bs->kmax) bs->done = 1;
    }
}

/* V_{j+1, s} = gate[s] * w_s */
__global__ void bscale_dev_kernel(const BState *__restrict__ bs, const double *__restrict__ w,
                                  const double *__restrict__ gate, double *__restrict__ V, int64_t ld,
                                  const int64_t *__restrict__ off, const int64_t *__restrict__ n)
{
    const int s = blockIdx.y;
    if (bs->done) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n[s]) return;
    V[(int64_t)(bs->j + 1) * ld + off[s] + i] = gate[s] * w[off[s] + i];
}

__global__ void badvance_kernel(BState *__restrict__ bs)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && !bs->done) bs->j += 1;
}

/* y_s = R^{-1} g_s over the dk[s] leading columns; one wave per system */
__global__ __launch_bounds__(64) void bsolve_kernel(int m, int ldh, const double *__restrict__ H,
                                                    const double *__restrict__ gv, const int32_t *__restrict__ dk,
                                                    double *__restrict__ y)
{
    const int s = blockIdx.x, k = dk[s];
    const double *Hs = H + (int64_t)s * (m + 1) * m, *g_ = gv + (int64_t)s * (m + 1);
    double *y_ = y + (int64_t)s * ldh;
    for (int i = k - 1; i >= 0; --i) {
        double acc = 0.0;
        for (int c = i + 1 + (int)threadIdx.x; c < k; c += 64) acc = fma(Hs[(int64_t)i * m + c], y_[c], acc);
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (threadIdx.x == 0) {
            const double d = Hs[(int64_t)i * m + i];
            y_[i] = d != 0.0 ? (g_[i] - acc) / d : 0.0;
        }
        __syncthreads();
    }
}

struct mhlp_batch {
    int n_geom = 0, R = 0, S = 0;
    int64_t total = 0, max_n = 0;
    std::vector<int64_t> off, n;
    BatchGeo *dgeo = nullptr;
    BatchWork *dwork = nullptr, *dfin = nullptr;
    int64_t nwork = 0, nfin = 0;
    double *part = nullptr;
    int64_t *doff = nullptr, *dn = nullptr;
    /* GMRES workspace */
    int m = 0;
    double *V = nullptr, *w = nullptr, *r = nullptr;
    double *dh = nullptr, *hh = nullptr; /* [3][S][ldh] device / pinned host */
    double *dsc = nullptr;               /* per-system scalars */
    int32_t *dk = nullptr;
    int ldh = 0;
    std::vector<BatchGeo> hgeo; /* host copy of the per-geometry descriptors */
    int64_t target = 0;         /* block target of the current work list    */
    int tpl = 1, src = FT_SRC;  /* tile shape of the far launch: targets per lane, sources per LDS stage */
    uint64_t version = 0;       /* bumped by every work-list build (keys the captured graphs) */
    struct TuneRec {
        int64_t target;
        int tpl, src;
        double ms;
    };
    std::vector<TuneRec> tune; /* the autotuner's candidates */
    /* device-driven GMRES: state, per-system Hessenberg data, step graphs */
    char *gd = nullptr;         /* BState, H, cs, sn, gv, y, thresh, resest  */
    char *hpin = nullptr;       /* pinned: BState + resest (down), gv + thresh (up) */
    hipStream_t cap_stream = nullptr;
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        const void *V = nullptr, *work = nullptr, *part = nullptr, *gd = nullptr;
        int m = 0, S = 0;
        uint64_t version = 0;
    } graphs[4];
};

static mhlp_status batch_build_work(mhlp_batch *B, int64_t target, int tpl, int src, hipStream_t st);

extern "C" mhlp_status mhlp_batch_destroy(mhlp_batch *B)
{
    if (!B) return MHLP_OK;
    for (auto &gr : B->graphs)
        if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    void *ptrs[] = {B->dgeo, B->dwork, B->dfin, B->part, B->doff, B->dn, B->V,
                    B->w,    B->r,     B->dh,   B->dsc,  B->dk,   B->gd};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (B->hh) (void)hipHostFree(B->hh);
    if (B->hpin) (void)hipHostFree(B->hpin);
    delete B;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_batch_create(int32_t n_geom, const mhlp_plan *const *plans, int32_t n_rhs, void *stream,
                                         mhlp_batch **out)
{
    if (!out) return fail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_geom < 1 || !plans) return fail(MHLP_INVALID_ARG, "need at least one plan");
    if (n_rhs < 1 || n_rhs > BATCH_R_MAX) return fail(MHLP_INVALID_ARG, "n_rhs must be 1..4");
    for (int g = 0; g < n_geom; ++g)
        if (!plans[g] || !plans[g]->onsurf || plans[g]->stokes)
            return fail(MHLP_INVALID_ARG, "batch needs on-surface scalar plans");
    hipStream_t st = (hipStream_t)stream;
    mhlp_batch *B = new mhlp_batch();
    B->n_geom = n_geom;
    B->R = n_rhs;
    B->S = n_geom * n_rhs;
    B->hgeo.resize(n_geom);
    int64_t voff = 0;
    for (int g = 0; g < n_geom; ++g) {
        const mhlp_plan *P = plans[g];
        const mhlp_geometry *G = P->g;
        BatchGeo &b = B->hgeo[g];
        b.x = G->soa;
        b.y = G->soa + G->N;
        b.w = G->w;
        b.nx = G->nx;
        b.ny = G->ny;
        b.nptr = P->near_ptr;
        b.npan = P->near_panel;
        b.wdl = P->wdlp;
        b.N = G->N;
        b.Np = G->Np;
        b.alpha = P->alpha;
        b.voff = voff;
        for (int r = 0; r < n_rhs; ++r) {
            B->off.push_back(voff + (int64_t)r * G->N);
            B->n.push_back(G->N);
        }
        B->max_n = std::max<int64_t>(B->max_n, G->N);
        voff += (int64_t)n_rhs * G->N;
    }
    B->total = voff;
    mhlp_status s;
    if ((s = dalloc(&B->dgeo, n_geom)) || (s = dalloc(&B->doff, B->S)) || (s = dalloc(&B->dn, B->S))) {
        mhlp_batch_destroy(B);
        return s;
    }
    hipError_t e = hipMemcpyAsync(B->doff, B->off.data(), sizeof(int64_t) * B->S, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(B->dn, B->n.data(), sizeof(int64_t) * B->S, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        mhlp_batch_destroy(B);
        return fail(MHLP_HIP_ERROR, std::string("batch_create: ") + hipGetErrorString(e));
    }
    if ((s = batch_build_work(B, 2048, 1, FT_SRC, st))) {
        mhlp_batch_destroy(B);
        return s;
    }
    *out = B;
    return MHLP_OK;
}

/* Work list of the grouped operator launch for about `target` blocks in total:
   each geometry gets blocks in proportion to its share of the pair work
   (N_g^2), as source splits of its target blocks (at least 4 panels per
   split); items are ordered by decreasing cost so the longest start first. */
static mhlp_status batch_build_work(mhlp_batch *B, int64_t target, int tpl, int src, hipStream_t st)
{
    const int n_geom = B->n_geom, n_rhs = B->R;
    double tot_work = 0;
    for (const BatchGeo &b : B->hgeo) tot_work += (double)b.N * b.N;
    std::vector<BatchWork> hw, hf;
    int64_t poff = 0;
    for (int g = 0; g < n_geom; ++g) {
        BatchGeo &b = B->hgeo[g];
        const int64_t tb = (b.N + FT_THREADS - 1) / FT_THREADS;            /* finalize tiles */
        const int64_t tbf = (b.N + FT_THREADS * tpl - 1) / (FT_THREADS * tpl); /* far tiles */
        const int64_t want = (int64_t)std::ceil((double)target * (double)b.N * b.N / tot_work);
        int64_t ns = (want + tbf - 1) / tbf;
        if (ns > b.Np / 4) ns = b.Np / 4;
        if (ns < 1) ns = 1;
        b.pps = (int32_t)((b.Np + ns - 1) / ns);
        b.nsplit = (int32_t)((b.Np + b.pps - 1) / b.pps);
        b.poff = poff;
        poff += (int64_t)b.nsplit * n_rhs * b.N;
        for (int64_t t = 0; t < tbf; ++t)
            for (int sp = 0; sp < b.nsplit; ++sp) hw.push_back(BatchWork{g, (int32_t)t, sp, 0});
        for (int64_t t = 0; t < tb; ++t) hf.push_back(BatchWork{g, (int32_t)t, 0, 0});
    }
    /* cost of an item ~ panels it sums over (all items have the same target tile) */
    std::stable_sort(hw.begin(), hw.end(), [&](const BatchWork &a, const BatchWork &c) {
        return B->hgeo[a.g].pps > B->hgeo[c.g].pps;
    });
    HIPCHECK(hipStreamSynchronize(st)); /* old buffers may be in use */
    void *old[] = {B->dwork, B->dfin, B->part};
    for (void *p : old)
        if (p) (void)hipFree(p);
    B->dwork = B->dfin = nullptr;
    B->part = nullptr;
    B->nwork = (int64_t)hw.size();
    B->nfin = (int64_t)hf.size();
    B->target = target;
    B->tpl = tpl;
    B->src = src;
    ++B->version;
    TRY(dalloc(&B->dwork, B->nwork));
    TRY(dalloc(&B->dfin, B->nfin));
    TRY(dalloc(&B->part, poff));
    hipError_t e = hipMemcpyAsync(B->dgeo, B->hgeo.data(), sizeof(BatchGeo) * n_geom, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(B->dwork, hw.data(), sizeof(BatchWork) * B->nwork, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(B->dfin, hf.data(), sizeof(BatchWork) * B->nfin, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("batch work list: ") + hipGetErrorString(e));
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_batch_info(const mhlp_batch *B, int64_t *total_len, int32_t *n_systems,
                                       int64_t *offsets, int64_t *lengths)
{
    if (!B) return fail(MHLP_INVALID_ARG, "batch is NULL");
    if (total_len) *total_len = B->total;
    if (n_systems) *n_systems = B->S;
    for (int s = 0; s < B->S; ++s) {
        if (offsets) offsets[s] = B->off[s];
        if (lengths) lengths[s] = B->n[s];
    }
    return MHLP_OK;
}

template <int R>
static void batch_apply_t(const mhlp_batch *B, const double *mu, double *out, const double *gate,
                          const BState *bs, int64_t jstride, hipStream_t st)
{
    const unsigned nw = (unsigned)B->nwork;
    if (B->tpl == 2 && B->src == 128)
        batch_far_dlp<R, 2, 128><<<nw, FT_THREADS, 0, st>>>(B->dgeo, B->dwork, mu, B->part, gate, bs, jstride);
    else if (B->tpl == 2)
        batch_far_dlp<R, 2, FT_SRC><<<nw, FT_THREADS, 0, st>>>(B->dgeo, B->dwork, mu, B->part, gate, bs, jstride);
    else if (B->src == 128)
        batch_far_dlp<R, 1, 128><<<nw, FT_THREADS, 0, st>>>(B->dgeo, B->dwork, mu, B->part, gate, bs, jstride);
    else
        batch_far_dlp<R, 1, FT_SRC><<<nw, FT_THREADS, 0, st>>>(B->dgeo, B->dwork, mu, B->part, gate, bs, jstride);
    batch_finalize<R><<<(unsigned)B->nfin, FT_THREADS, 0, st>>>(B->dgeo, B->dfin, B->part, mu, out, gate, bs,
                                                                  jstride);
}

/* out = (1/2 I + D) mu for every system; with a gate, geometries whose
   systems are all gated off are skipped (their part of out is left as is);
   with a GMRES state, mu is the basis and column bs->j is applied */
static mhlp_status batch_apply_impl(const mhlp_batch *B, const double *mu, double *out, hipStream_t st,
                                    const double *gate = nullptr, const BState *bs = nullptr, int64_t jstride = 0)
{
    switch (B->R) {
    case 1: batch_apply_t<1>(B, mu, out, gate, bs, jstride, st); break;
    case 2: batch_apply_t<2>(B, mu, out, gate, bs, jstride, st); break;
    case 3: batch_apply_t<3>(B, mu, out, gate, bs, jstride, st); break;
    default: batch_apply_t<4>(B, mu, out, gate, bs, jstride, st); break;
    }
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_batch_apply_bie(const mhlp_batch *B, const double *mu, double *out, void *stream)
{
    if (!B || !mu || !out) return fail(MHLP_INVALID_ARG, "NULL argument");
    if (mu == out) return fail(MHLP_INVALID_ARG, "mu and out must not alias");
    return batch_apply_impl(B, mu, out, (hipStream_t)stream);
}

extern "C" mhlp_status mhlp_batch_autotune(mhlp_batch *B, int32_t reps, void *stream, int64_t *best_target,
                                           double *best_ms)
{
    if (!B) return fail(MHLP_INVALID_ARG, "batch is NULL");
    if (reps < 1 || reps > 1000) return fail(MHLP_INVALID_ARG, "reps must be in [1, 1000]");
    hipStream_t st = (hipStream_t)stream;
    double *mu = nullptr, *out = nullptr;
    TRY(dalloc(&mu, B->total));
    mhlp_status s = dalloc(&out, B->total);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s == MHLP_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        s = fail(MHLP_HIP_ERROR, "hipEventCreate");
    if (s == MHLP_OK) fill_kernel<<<nblocks(B->total, 256), 256, 0, st>>>(mu, 1.0, B->total);
    struct Cand {
        int64_t target;
        int tpl, src;
        double ms;
    };
    std::vector<Cand> tim;
    for (int tpl : {1, 2})
        for (int src : {128, FT_SRC})
            for (int64_t tg : {512LL, 1024LL, 2048LL, 4096LL, 8192LL, 16384LL}) {
                if (s) break;
                if ((s = batch_build_work(B, tg, tpl, src, st))) break;
                if ((s = batch_apply_impl(B, mu, out, st))) break;
                float ms = 0.f;
                hipError_t e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess && s == MHLP_OK; ++r) s = batch_apply_impl(B, mu, out, st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess && s == MHLP_OK)
                    s = fail(MHLP_HIP_ERROR, std::string("batch autotune: ") + hipGetErrorString(e));
                if (s == MHLP_OK) tim.push_back(Cand{tg, tpl, src, (double)ms / reps});
            }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(mu);
    if (out) (void)hipFree(out);
    if (s) return s;
    double bms = 1e300;
    for (const auto &t : tim) bms = std::min(bms, t.ms);
    /* fewest blocks within 1% of the fastest (the first such in the search
       order: one target per lane and the larger stage first) */
    const Cand *best = nullptr;
    for (const auto &t : tim)
        if (t.ms <= 1.01 * bms && (!best || t.target < best->target)) best = &t;
    B->tune.clear();
    for (const auto &t : tim) B->tune.push_back(mhlp_batch::TuneRec{t.target, t.tpl, t.src, t.ms});
    TRY(batch_build_work(B, best->target, best->tpl, best->src, st));
    if (best_target) *best_target = best->target;
    if (best_ms) *best_ms = best->ms;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_batch_set_tile(mhlp_batch *B, int64_t target, int32_t tpl, int32_t src, void *stream)
{
    if (!B) return fail(MHLP_INVALID_ARG, "batch is NULL");
    if (target < 1 || target > (1LL << 24)) return fail(MHLP_INVALID_ARG, "block target must be in [1, 2^24]");
    if (tpl != 1 && tpl != 2) return fail(MHLP_INVALID_ARG, "targets per lane must be 1 or 2");
    if (src != 128 && src != FT_SRC) return fail(MHLP_INVALID_ARG, "sources per stage must be 128 or 256");
    return batch_build_work(B, target, tpl, src, (hipStream_t)stream);
}

/* The tile shape chosen for a batch (targets per lane, sources per LDS stage)
   and the autotuner's measured candidates (host outputs, may be NULL; up to
   cap rows of {block target, targets per lane, sources per stage} and their
   ms per operator application). */
extern "C" mhlp_status mhlp_batch_tile(const mhlp_batch *B, int64_t *target, int32_t *tpl, int32_t *src,
                                       int64_t *cand, double *cand_ms, int32_t cap, int32_t *n_cand)
{
    if (!B) return fail(MHLP_INVALID_ARG, "batch is NULL");
    if (target) *target = B->target;
    if (tpl) *tpl = B->tpl;
    if (src) *src = B->src;
    const int32_t n = (int32_t)B->tune.size();
    if (n_cand) *n_cand = n;
    for (int32_t c = 0; c < n && c < cap; ++c) {
        if (cand) {
            cand[3 * c] = B->tune[c].target;
            cand[3 * c + 1] = B->tune[c].tpl;
            cand[3 * c + 2] = B->tune[c].src;
        }
        if (cand_ms) cand_ms[c] = B->tune[c].ms;
    }
    return MHLP_OK;
}

/* Device data of the batched GMRES for restart m (layout stride B->m). */
struct BDev {
    BState *bs;
    double *H, *cs, *sn, *gv, *y, *thresh, *resest;
};

static BDev bdev_view(const mhlp_batch *B)
{
    const int64_t S = B->S, m = B->m, ldh = B->ldh;
    BDev d;
    d.bs = reinterpret_cast<BState *>(B->gd);
    double *p = reinterpret_cast<double *>(B->gd + 64);
    d.H = p;
    p += S * (m + 1) * m;
    d.cs = p;
    p += S * m;
    d.sn = p;
    p += S * m;
    d.gv = p;
    p += S * (m + 1);
    d.y = p;
    p += S * ldh;
    d.thresh = p;
    p += S;
    d.resest = p;
    return d;
}

/* one lockstep Arnoldi step of every active system, enqueued on st */
static mhlp_status enqueue_bstep(mhlp_batch *B, hipStream_t st)
{
    const int S = B->S, m = B->m, ldh = B->ldh;
    const int64_t T = B->total;
    const BDev d = bdev_view(B);
    double *h1 = B->dh, *h2 = B->dh + (int64_t)S * ldh, *hn = B->dh + 2 * (int64_t)S * ldh;
    const dim3 gS((unsigned)((B->max_n + 255) / 256), (unsigned)S);
    TRY(batch_apply_impl(B, B->V, B->w, st, B->dsc, d.bs, T));
    bdot_dev_kernel<<<dim3((unsigned)S, (unsigned)m), 256, 0, st>>>(d.bs, B->V, T, B->w, B->doff, B->dn, ldh, h1,
                                                                     B->dsc);
    bsub_dev_kernel<<<gS, 256, 0, st>>>(d.bs, B->V, T, h1, ldh, B->w, B->doff, B->dn, B->dsc);
    bdot_dev_kernel<<<dim3((unsigned)S, (unsigned)m), 256, 0, st>>>(d.bs, B->V, T, B->w, B->doff, B->dn, ldh, h2,
                                                                     B->dsc);
    bsub_dev_kernel<<<gS, 256, 0, st>>>(d.bs, B->V, T, h2, ldh, B->w, B->doff, B->dn, B->dsc);
    bdot_dev_kernel<<<dim3((unsigned)S, 1), 256, 0, st>>>(d.bs, B->w, 0, B->w, B->doff, B->dn, ldh, hn, B->dsc);
    bfinish_kernel<<<1, 256, 0, st>>>(d.bs, S, m, ldh, d.H, d.cs, d.sn, d.gv, h1, h2, hn, d.thresh, d.resest, B->dsc,
                                      B->dk);
    bscale_dev_kernel<<<gS, 256, 0, st>>>(d.bs, B->w, B->dsc, B->V, T, B->doff, B->dn);
    badvance_kernel<<<1, 64, 0, st>>>(d.bs);
    HIPCHECK(hipGetLastError());
    return MHLP_OK;
}

/* executable graph of 2^si lockstep steps, captured once per batch state */
static mhlp_status bstep_graph(mhlp_batch *B, int si, hipGraphExec_t *out)
{
    const int S = 1 << si;
    mhlp_batch::StepGraph &G = B->graphs[si];
    if (G.exec && G.V == B->V && G.work == B->dwork && G.part == B->part && G.gd == B->gd && G.m == B->m &&
        G.S == S && G.version == B->version) {
        *out = G.exec;
        return MHLP_OK;
    }
    if (G.exec) {
        (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
    }
    if (!B->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
    HIPCHECK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    mhlp_status s = MHLP_OK;
    for (int k = 0; k < S && s == MHLP_OK; ++k) s = enqueue_bstep(B, B->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(B->cap_stream, &graph);
    if (s != MHLP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(MHLP_HIP_ERROR, std::string("batch step capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        G.exec = nullptr;
        return fail(MHLP_HIP_ERROR, std::string("batch step graph: ") + hipGetErrorString(e));
    }
    G.V = B->V;
    G.work = B->dwork;
    G.part = B->part;
    G.gd = B->gd;
    G.m = B->m;
    G.S = S;
    G.version = B->version;
    *out = G.exec;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_batch_gmres_solve(mhlp_batch *B, const double *g, double *mu, const mhlp_gmres_opts *opts,
                                              mhlp_gmres_info *infos, void *stream)
{
    if (!B || !g || !mu || !opts || !infos) return fail(MHLP_INVALID_ARG, "NULL argument");
    if (!(opts->tol > 0.0) || opts->max_iter < 1 || opts->restart < 1) return fail(MHLP_INVALID_ARG, "bad options");
    if (opts->precision != MHLP_FP64) return fail(MHLP_UNSUPPORTED, "batched GMRES runs in FP64");
    hipStream_t st = (hipStream_t)stream;
    const int S = B->S;
    const int mreq = std::min(opts->restart, 64);
    const int64_t T = B->total;
    if (B->m < mreq) {
        HIPCHECK(hipDeviceSynchronize());
        void *ptrs[] = {B->V, B->w, B->r, B->dh, B->dsc, B->dk, B->gd};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        if (B->hh) (void)hipHostFree(B->hh);
        if (B->hpin) (void)hipHostFree(B->hpin);
        B->V = B->w = B->r = B->dh = B->dsc = nullptr;
        B->dk = nullptr;
        B->gd = nullptr;
        B->hh = nullptr;
        B->hpin = nullptr;
        const int m = mreq;
        B->ldh = m + 2;
        B->m = m;
        const int64_t ngd = (int64_t)S * (m + 1) * m + 2 * (int64_t)S * m + (int64_t)S * (m + 1) +
                            (int64_t)S * B->ldh + 2 * (int64_t)S;
        TRY(dalloc(&B->V, (int64_t)(m + 1) * T));
        TRY(dalloc(&B->w, T));
        TRY(dalloc(&B->r, T));
        TRY(dalloc(&B->dh, 3 * (int64_t)S * B->ldh));
        TRY(dalloc(&B->dsc, S));
        TRY(dalloc(&B->dk, S));
        TRY(dalloc(&B->gd, 64 + 8 * ngd));
        HIPCHECK(hipHostMalloc((void **)&B->hh, sizeof(double) * 3 * (size_t)S * B->ldh, hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void **)&B->hpin, 64 + sizeof(double) * ((size_t)S * (m + 3) + S), hipHostMallocDefault));
    }
    const int m = B->m, ldh = B->ldh;
    const int mcyc = std::min(opts->restart, m);
    const BDev d = bdev_view(B);
    const dim3 gS((unsigned)((B->max_n + 255) / 256), (unsigned)S);
    double *hn = B->dh + 2 * (int64_t)S * ldh;
    BState *bsh = reinterpret_cast<BState *>(B->hpin);
    double *res_h = reinterpret_cast<double *>(B->hpin + 64);    /* [S] resest, device -> host */
    double *up_h = res_h + S;                                     /* [S][m+1] gv then [S] thresh  */
    std::vector<double> bn(S), rel(S, 1.0), x0res(S, 1.0), sc(S), last(S);
    std::vector<int32_t> iters(S, 0), cyc(S, 0), kk(S);
    std::vector<char> conv(S, 0);
    auto norms = [&](const double *v, std::vector<double> &outv) -> mhlp_status {
        bdot_kernel<<<dim3((unsigned)S, 1), 256, 0, st>>>(v, 0, v, B->doff, B->dn, ldh, hn);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(B->hh, hn, sizeof(double) * (size_t)S * ldh, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        for (int s2 = 0; s2 < S; ++s2) outv[s2] = std::sqrt(B->hh[(size_t)s2 * ldh]);
        return MHLP_OK;
    };
    TRY(norms(g, bn));
    /* x0: a guess whose residual is >= 1 (relative) is replaced by zero, per system */
    std::vector<double> rn(S);
    if (opts->use_x0) {
        TRY(batch_apply_impl(B, mu, B->w, st));
        residual_kernel<<<nblocks(T, 256), 256, 0, st>>>(g, B->w, B->r, T);
        TRY(norms(B->r, rn));
        bool any_bad = false;
        for (int s2 = 0; s2 < S; ++s2) {
            x0res[s2] = bn[s2] > 0 ? rn[s2] / bn[s2] : 0.0;
            sc[s2] = (x0res[s2] < 1.0) ? 1.0 : 0.0;
            any_bad |= sc[s2] == 0.0;
        }
        if (any_bad) {
            HIPCHECK(hipMemcpyAsync(B->dsc, sc.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
            bscale_kernel<<<gS, 256, 0, st>>>(mu, B->dsc, mu, B->doff, B->dn);
        }
    } else {
        fill_kernel<<<nblocks(T, 256), 256, 0, st>>>(mu, 0.0, T);
    }
    int total_it = 0;
    for (;;) {
        TRY(batch_apply_impl(B, mu, B->w, st));
        residual_kernel<<<nblocks(T, 256), 256, 0, st>>>(g, B->w, B->r, T);
        TRY(norms(B->r, rn));
        int nact = 0;
        for (int s2 = 0; s2 < S; ++s2) {
            rel[s2] = bn[s2] > 0 ? rn[s2] / bn[s2] : 0.0;
            conv[s2] = rel[s2] <= opts->tol;
            sc[s2] = conv[s2] ? 0.0 : 1.0 / rn[s2];
            nact += !conv[s2];
            cyc[s2] += !conv[s2];
            last[s2] = rn[s2];
        }
        if (nact == 0 || total_it >= opts->max_iter) break;
        /* cycle start: V_0 = r / ||r||, g = ||r|| e_1, thresholds, state */
        for (int s2 = 0; s2 < S; ++s2) {
            double *gs_ = up_h + (size_t)s2 * (m + 1);
            std::fill(gs_, gs_ + m + 1, 0.0);
            gs_[0] = rn[s2];
            up_h[(size_t)S * (m + 1) + s2] = 0.5 * opts->tol * bn[s2];
        }
        *bsh = BState{0, std::min(mcyc, opts->max_iter - total_it), 0, nact, 0, {0, 0, 0}};
        HIPCHECK(hipMemcpyAsync(B->dsc, sc.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
        bscale_kernel<<<gS, 256, 0, st>>>(B->r, B->dsc, B->V, B->doff, B->dn);
        HIPCHECK(hipMemcpyAsync(d.gv, up_h, sizeof(double) * (size_t)S * (m + 1), hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(d.thresh, up_h + (size_t)S * (m + 1), sizeof(double) * S, hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(d.bs, bsh, sizeof(BState), hipMemcpyHostToDevice, st));
        fill_i32_kernel<<<nblocks(S, 256), 256, 0, st>>>(B->dk, 0, S);
        HIPCHECK(hipGetLastError());
        int chunk = 2, done_steps = 0;
        for (;;) {
            int si = 0;
            while ((1 << si) < chunk && si < 3) ++si;
            hipGraphExec_t ex;
            TRY(bstep_graph(B, si, &ex));
            HIPCHECK(hipGraphLaunch(ex, st));
            HIPCHECK(hipMemcpyAsync(bsh, d.bs, sizeof(BState), hipMemcpyDeviceToHost, st));
            HIPCHECK(hipMemcpyAsync(res_h, d.resest, sizeof(double) * S, hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            if (bsh->done) break;
            /* steps the slowest active system still needs at its observed rate */
            const int ran = bsh->steps - done_steps;
            done_steps = bsh->steps;
            int need = 1;
            for (int s2 = 0; s2 < S; ++s2) {
                if (sc[s2] == 0.0) continue;
                const double th = 0.5 * opts->tol * bn[s2], est = res_h[s2];
                if (est <= th) continue;
                int ns2 = 8;
                if (ran > 0 && est > 0.0 && est < last[s2])
                    ns2 = (int)std::ceil(std::log(th / est) / std::log(std::pow(est / last[s2], 1.0 / ran)));
                need = std::max(need, ns2);
                last[s2] = est;
            }
            chunk = std::max(1, std::min(need, 8));
        }
        total_it += bsh->steps;
        HIPCHECK(hipMemcpy(kk.data(), B->dk, sizeof(int32_t) * S, hipMemcpyDeviceToHost));
        for (int s2 = 0; s2 < S; ++s2) iters[s2] += kk[s2];
        bsolve_kernel<<<(unsigned)S, 64, 0, st>>>(m, ldh, d.H, d.gv, B->dk, d.y);
        bcombo_kernel<<<gS, 256, 0, st>>>(B->V, T, 0, B->dk, d.y, ldh, 1.0, mu, B->doff, B->dn);
        HIPCHECK(hipGetLastError());
    }
    bool all = true;
    for (int s2 = 0; s2 < S; ++s2) {
        infos[s2].iters = iters[s2];
        infos[s2].restarts = cyc[s2];
        infos[s2].rel_residual = rel[s2];
        infos[s2].x0_residual = opts->use_x0 ? x0res[s2] : 1.0;
        infos[s2].converged = conv[s2];
        infos[s2].used_x0 = opts->use_x0 ? (x0res[s2] < 1.0) : 0;
        all &= conv[s2] != 0;
    }
    return all ? MHLP_OK : MHLP_NOT_CONVERGED;
}
