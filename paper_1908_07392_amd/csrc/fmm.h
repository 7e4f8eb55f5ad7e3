/* Fast multipole far field for the Yukawa sums of the layer potentials and of
   the volume sum (Sec. 3.2.1, "Fast summation"), scalar kernel, FP64.

   The field of charges q_j and dipoles d_j at y_j,
       phi(x) = sum_j q_j K0(alpha |x - y_j|) + d_j . grad_y K0(alpha |x - y_j|),
   is split on a uniform quadtree: each leaf box takes the sources of its 3x3
   neighbourhood directly (P2P, with the caller's exclusion rule) and all
   other sources through local expansions built from multipole expansions by
   interaction lists at levels lstart..L.  Expansions are the paper's multipole
   and local expansions restricted to modified-Helmholtz fields, with outgoing
   O_n(z) = K_n(alpha |z|) e^{i n arg z} and regular R_n(z) = I_n(alpha |z|) e^{i n arg z}:
     P2M  charge: M_n += q R_{-n}(y - c); dipole: M_n += (alpha/2)[conj(d) R_{1-n} + d R_{-1-n}](y - c)
     M2M  M_k = sum_n M'_n R_{n-k}(c' - c)          (child c' -> parent c)
     M2L  L_l = (-1)^l sum_n M_n O_{n-l}(c_t - c_s)
     L2L  L'_m = sum_l L_l R_{l-m}(c' - c)           (parent c -> child c')
     L2P  phi = sum_l L_l R_l(x - c)
   (Graf's addition theorem for K_n and I_n), truncated to |n| <= p.  Fields are
   real, so coefficients with n < 0 are the conjugates of those with n > 0 and
   only n = 0..p are stored.

   Scaling.  Level l has the scale s_l = min(1, alpha side_l); stored
   coefficients are M~_n = M_n / s^|n| and L~_n = L_n s^|n|, tables hold
   O~_k = O_k s^|k| and R~_k = R_k / s^|k|, and each translation multiplies by
   the leftover powers of s (all <= 1), so no intermediate overflows for small
   alpha side, where K_n grows like (n-1)! (2/(alpha r))^n.

   Decay.  Well-separated boxes at level l are at least 0.586 side_l apart
   (centres 2 sides apart, radii 0.707 side); where alpha 0.586 side_l > 40 every
   such pair is below K0(40) ~ 4e-19 and the level's interactions are dropped
   (lstart is the coarsest level where they are kept; with lstart > L only the
   3x3 neighbourhoods remain).

   Root square (fixed from the inputs alone): centre at the midpoint of the
   bounding box of all sources and targets, side S = (largest extent)(1 + 2^-20)
   (S = 1 if all points coincide); leaf coordinates
   ix = floor((x - (cx - S/2)) / (S / 2^L)) clamped to [0, 2^L - 1].  Boxes are
   numbered iy 2^l + ix; a child's index within its parent is (ix & 1) + 2 (iy & 1). */
#pragma once

#include "fmm_math.h"

namespace mhlp {

constexpr int FMM_PMAX = 60;    /* largest expansion order p */
constexpr int FMM_LMAX = 10;    /* deepest leaf level        */
constexpr int FMM_TILE = 64;    /* leaf kernel: targets per work item, sources per LDS tile */

struct FmmDev {
    int L, p, lstart, nwork;
    double alpha, x0, y0, S;                 /* lower-left corner and side of the root square */
    double side[FMM_LMAX + 1], sig[FMM_LMAX + 1];
    int64_t eoff[FMM_LMAX + 1];              /* expansion offset of level l (cplx units, all fields) */
    int64_t t2l[FMM_LMAX + 1];               /* M2L table of level l: [49][3p+1] */
    int64_t tmm[FMM_LMAX + 1], tll[FMM_LMAX + 1]; /* shift tables of parent level l: [4][3p+1] */
    const int32_t *socc, *tocc;              /* per-level source / target counts, level l at lev4(l) */
    const int32_t *sstart, *tstart;          /* leaf CSR [4^L + 1] */
    const int32_t *sidx;                     /* sorted source -> caller source index */
    const int32_t *tidx;                     /* sorted target -> caller (internal) target index */
    const int32_t *wbox, *wt0;               /* leaf work items: box, first sorted target (<= FMM_TILE each) */
    const double *lx, *ly, *lw, *lnx, *lny;  /* sources in leaf order */
    const int32_t *lpan;                     /* panel of each sorted source (plans) */
    cplx *mexp, *lexp;                       /* expansions [level][field][box][p+1]; lexp holds nch[l] */
    int64_t lch;                             /* partial local expansions, lch apart (their sum is L) */
    int nch[FMM_LMAX + 1];                   /* partials (blocks per box) of level l's downward pass */
    const cplx *tab;                         /* translation tables */
};

__host__ __device__ inline int64_t lev4(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; } /* sum_{k<l} 4^k */

/* ------------------------------------------------------------------------ */
/* translation tables: one thread per row                                   */
/* ------------------------------------------------------------------------ */
__global__ void fmm_tables_kernel(const FmmRow *__restrict__ rows, int nrows, int p, double alpha,
                                  cplx *__restrict__ tab, double *__restrict__ scratch)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    fmm_table_row(rows[r], p, alpha, tab, scratch + (int64_t)r * (2 * p + 1));
}

/* gather of the sources into leaf order */
__global__ void fmm_gather_kernel(const int32_t *__restrict__ sidx, int64_t n, const double *__restrict__ x,
                                  const double *__restrict__ y, const double *__restrict__ w,
                                  const double *__restrict__ nx, const double *__restrict__ ny, double *__restrict__ ox,
                                  double *__restrict__ oy, double *__restrict__ ow, double *__restrict__ onx,
                                  double *__restrict__ ony, int32_t *__restrict__ opan)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t o = sidx[j];
    ox[j] = x[o];
    oy[j] = y[o];
    ow[j] = w[o];
    if (onx) onx[j] = nx[o];
    if (ony) ony[j] = ny[o];
    if (opan) opan[j] = (int32_t)(o / 16);
}

__device__ __forceinline__ cplx fmm_center(const FmmDev &T, int l, int ix, int iy)
{
    return mk(T.x0 + (ix + 0.5) * T.side[l], T.y0 + (iy + 0.5) * T.side[l]);
}

/* ------------------------------------------------------------------------ */
/* P2M at the leaves: one wave per leaf box; lanes take 64 sources at a time  */
/* (their R~_n into LDS), then lane n sums over them in order.                */
/* field 0: charges w sigma (SLP), field 1: dipoles w mu n (DLP)              */
/* ------------------------------------------------------------------------ */
template <bool SLP, bool DLP>
__global__ __launch_bounds__(64) void fmm_p2m_kernel(FmmDev T, const double *__restrict__ sigma,
                                                     const double *__restrict__ mu)
{
    __shared__ double lre[64][FMM_PMAX + 2], lim[64][FMM_PMAX + 2];
    __shared__ double lq[64], ldx[64], ldy[64];
    const int L = T.L, p = T.p, nb = 1 << L;
    const int box = blockIdx.x, lane = threadIdx.x;
    const int ix = box % nb, iy = box / nb;
    const cplx c = fmm_center(T, L, ix, iy);
    const double s = T.sig[L], al = T.alpha;
    cplx aS = mk(0.0, 0.0), aD = mk(0.0, 0.0);
    const int b0 = T.sstart[box], b1 = T.sstart[box + 1];
    for (int base = b0; base < b1; base += 64) {
        const int j = base + lane;
        if (j < b1) {
            const int64_t o = T.sidx[j];
            const double dxv = T.lx[j] - c.re, dyv = T.ly[j] - c.im;
            const double rr = sqrt(dxv * dxv + dyv * dyv);
            const cplx u = rr > 0.0 ? mk(dxv / rr, dyv / rr) : mk(1.0, 0.0);
            fmm_iscaled_store(al * rr, s, p + 1, &lre[lane][0], 1);
            cplx e = mk(1.0, 0.0);
            for (int n = 0; n <= p + 1; ++n) {
                const double m = lre[lane][n];
                lre[lane][n] = m * e.re;
                lim[lane][n] = m * e.im;
                e = e * u;
            }
            const double w = T.lw[j];
            lq[lane] = SLP ? w * sigma[o] : 0.0;
            if (DLP) {
                const double m = w * mu[o];
                ldx[lane] = m * T.lnx[j];
                ldy[lane] = m * T.lny[j];
            } else {
                ldx[lane] = 0.0;
                ldy[lane] = 0.0;
            }
        }
        __syncthreads();
        const int cnt = min(64, b1 - base);
        if (lane <= p) {
            const int n = lane;
            for (int t = 0; t < cnt; ++t) {
                const cplx Rn = mk(lre[t][n], -lim[t][n]); /* conj R~_n */
                if (SLP) aS = aS + lq[t] * Rn;
                if (DLP) {
                    const cplx d = mk(ldx[t], ldy[t]);
                    if (n == 0) {
                        /* alpha s Re(conj(d) R~_1) */
                        const cplx r1 = mk(lre[t][1], lim[t][1]);
                        aD.re = fma(al * s, (conj(d) * r1).re, aD.re);
                    } else {
                        const cplx rm = mk(lre[t][n - 1], -lim[t][n - 1]), rp = mk(lre[t][n + 1], -lim[t][n + 1]);
                        aD = aD + (0.5 * al / s) * (conj(d) * rm) + (0.5 * al * s) * (d * rp);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (lane <= p) {
        const int64_t nbx = (int64_t)nb * nb;
        if (SLP) T.mexp[T.eoff[L] + (0 * nbx + box) * (p + 1) + lane] = aS;
        if (DLP) T.mexp[T.eoff[L] + (1 * nbx + box) * (p + 1) + lane] = aD;
    }
}

/* M2M into parent level l: one block per parent box, wave w takes child w
   (lane k), the four partial sums are added in child order. */
template <bool SLP, bool DLP>
__global__ __launch_bounds__(256) void fmm_m2m_kernel(FmmDev T, int l)
{
    __shared__ cplx lm[4][2][FMM_PMAX + 1], part[4][2][FMM_PMAX + 1];
    __shared__ cplx lt[4][3 * FMM_PMAX + 1];
    __shared__ double pr[FMM_PMAX + 1], pp2[FMM_PMAX + 1];
    const int p = T.p, nb = 1 << l, nbc = nb << 1, rl = 3 * p + 1;
    const int box = blockIdx.x, tid = threadIdx.x, w = tid >> 6, k = tid & 63;
    const int ix = box % nb, iy = box / nb;
    const double sp_ = T.sig[l], sc = T.sig[l + 1];
    if (tid <= p) {
        pr[tid] = pow(sc / sp_, (double)tid);
        pp2[tid] = pow(sp_, 2.0 * tid);
    }
    const int cx = 2 * ix + (w & 1), cy = 2 * iy + (w >> 1);
    const int cb = cy * nbc + cx;
    const bool occ = T.socc[lev4(l + 1) + cb] != 0;
    const int64_t nbcx = (int64_t)nbc * nbc;
    if (occ) {
        if (k <= p) {
            lm[w][0][k] = SLP ? T.mexp[T.eoff[l + 1] + (0 * nbcx + cb) * (p + 1) + k] : mk(0.0, 0.0);
            lm[w][1][k] = DLP ? T.mexp[T.eoff[l + 1] + (1 * nbcx + cb) * (p + 1) + k] : mk(0.0, 0.0);
        }
        for (int j = k; j < rl; j += 64) lt[w][j] = T.tab[T.tmm[l] + (int64_t)w * rl + j];
    }
    __syncthreads();
    cplx acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
    if (occ && k <= p) {
        for (int n = -p; n <= p; ++n) {
            const int an = n >= 0 ? n : -n;
            const double f = pr[an] * (n >= 0 ? pp2[max(0, n - k)] : pp2[an]);
            const cplx t = f * lt[w][n - k + 2 * p];
            if (SLP) acc[0] = acc[0] + (n >= 0 ? lm[w][0][n] : conj(lm[w][0][-n])) * t;
            if (DLP) acc[1] = acc[1] + (n >= 0 ? lm[w][1][n] : conj(lm[w][1][-n])) * t;
        }
    }
    if (k <= p) {
        part[w][0][k] = acc[0];
        part[w][1][k] = acc[1];
    }
    __syncthreads();
    if (w == 0 && k <= p) {
        const int64_t nbx = (int64_t)nb * nb;
        cplx s0 = part[0][0][k], s1 = part[0][1][k];
        for (int c = 1; c < 4; ++c) {
            s0 = s0 + part[c][0][k];
            s1 = s1 + part[c][1][k];
        }
        if (SLP) T.mexp[T.eoff[l] + (0 * nbx + box) * (p + 1) + k] = s0;
        if (DLP) T.mexp[T.eoff[l] + (1 * nbx + box) * (p + 1) + k] = s1;
    }
}

/* downward pass at level l, one block per box that holds targets: L2L from
   the parent (l > lstart, wave 0) plus M2L over the occupied boxes of the
   interaction list, FMM_DW waves taking one list box each per round (its
   multipole and table row staged in LDS); per-wave sums are added in wave
   order, so the result does not depend on timing. */
constexpr int FMM_DW = 8;
/* blocks per box in the downward pass of the coarse levels (fewer than
   FMM_CH_BOXES boxes, too few blocks to fill the chip): block c of nch takes
   interactions c, c + nch, ... of the box's list (one round of FMM_DW waves for
   up to 27 entries) and writes partial local expansion c; chunk 0 also carries
   the L2L term.  The consumers (the children's L2L, the leaf's L2P) add the
   level's partials in order.  Finer levels run one block per box. */
constexpr int FMM_CH = 4, FMM_CH_BOXES = 256;

template <bool SLP, bool DLP>
__global__ __launch_bounds__(64 * FMM_DW) void fmm_down_kernel(FmmDev T, int l)
{
    __shared__ cplx lm[FMM_DW][2][FMM_PMAX + 1], lmp[FMM_DW][2][FMM_PMAX + 1], part[FMM_DW][2][FMM_PMAX + 1];
    __shared__ cplx lt[FMM_DW][3 * FMM_PMAX + 1];
    __shared__ double pw[FMM_PMAX + 1], pr[FMM_PMAX + 1];
    __shared__ int il_box[27], il_off[27], il_flag[36], n_il;
    const int p = T.p, nb = 1 << l, rl = 3 * p + 1;
    const int box = blockIdx.x, chunk = blockIdx.y, tid = threadIdx.x, w = tid >> 6, m = tid & 63;
    if (T.tocc[lev4(l) + box] == 0) return; /* whole block */
    const int ix = box % nb, iy = box / nb, px = ix >> 1, py = iy >> 1;
    const double s = T.sig[l];
    const double sp_ = l > 0 ? T.sig[l - 1] : 1.0;
    if (tid <= p) {
        pw[tid] = pow(s, 2.0 * tid);        /* M2L: s^{2 min(n, m)}; L2L: s_c^{2 j} */
        pr[tid] = pow(s / sp_, (double)tid); /* L2L: (s_c/s_p)^|l| */
    }
    /* interaction list: the 36 children of the parent's neighbours, one thread
       each (occupancy read in parallel), compacted in a fixed order */
    if (tid < 36) {
        const int jx = 2 * (px - 1) + tid % 6, jy = 2 * (py - 1) + tid / 6;
        int ok = jx >= 0 && jx < nb && jy >= 0 && jy < nb && (abs(jx - ix) > 1 || abs(jy - iy) > 1);
        if (ok) ok = T.socc[lev4(l) + jy * nb + jx] != 0;
        il_flag[tid] = ok;
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0;
        for (int c = 0; c < 36; ++c) {
            if (!il_flag[c]) continue;
            const int jx = 2 * (px - 1) + c % 6, jy = 2 * (py - 1) + c / 6;
            il_box[n] = jy * nb + jx;
            il_off[n] = (jx - ix + 3) * 7 + (jy - iy + 3);
            ++n;
        }
        n_il = n;
    }
    const int64_t nbx = (int64_t)nb * nb;
    const bool l2l = l > T.lstart && chunk == 0;
    if (l2l) {
        const int pnb = nb >> 1, pb = py * pnb + px, ch = (ix & 1) + 2 * (iy & 1);
        const int64_t pbx = (int64_t)pnb * pnb;
        if (tid <= p) {
            cplx a = mk(0.0, 0.0), b = mk(0.0, 0.0);
            for (int c = 0; c < T.nch[l - 1]; ++c) {
                const cplx *lp = T.lexp + c * T.lch + T.eoff[l - 1];
                if (SLP) a = a + lp[(0 * pbx + pb) * (p + 1) + tid];
                if (DLP) b = b + lp[(1 * pbx + pb) * (p + 1) + tid];
            }
            lm[0][0][tid] = a;
            lm[0][1][tid] = b;
        }
        for (int j = tid; j < rl; j += 64 * FMM_DW) lt[0][j] = T.tab[T.tll[l - 1] + (int64_t)ch * rl + j];
    }
    __syncthreads();
    cplx accl[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
    if (l2l && w == 0 && m <= p) {
        for (int n = -p; n <= p; ++n) {
            const int an = n >= 0 ? n : -n;
            const double f = pr[an] * (n >= m ? 1.0 : (n >= 0 ? pw[m - n] : pw[m]));
            const cplx t = f * lt[0][n - m + 2 * p];
            if (SLP) accl[0] = accl[0] + (n >= 0 ? lm[0][0][n] : conj(lm[0][0][-n])) * t;
            if (DLP) accl[1] = accl[1] + (n >= 0 ? lm[0][1][n] : conj(lm[0][1][-n])) * t;
        }
    }
    __syncthreads(); /* lm[0], lt[0] are reused below */
    cplx acce[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
    /* this block's share of the list: entries chunk, chunk + FMM_CH, ... */
    const int nchk = (int)gridDim.y;
    const int nil = n_il, nk = nil > chunk ? (nil - chunk + nchk - 1) / nchk : 0;
    const int nr = (nk + FMM_DW - 1) / FMM_DW;
    for (int r = 0; r < nr; ++r) {
        const int kc = r * FMM_DW + w, k = chunk + nchk * kc;
        const bool act = kc < nk;
        if (act) {
            const int sb = il_box[k];
            if (m <= p) {
                const cplx a = SLP ? T.mexp[T.eoff[l] + (0 * nbx + sb) * (p + 1) + m] : mk(0.0, 0.0);
                const cplx b = DLP ? T.mexp[T.eoff[l] + (1 * nbx + sb) * (p + 1) + m] : mk(0.0, 0.0);
                lm[w][0][m] = a;
                lm[w][1][m] = b;
                lmp[w][0][m] = pw[m] * a; /* the factor s^{2n} of the terms with 0 <= n < m */
                lmp[w][1][m] = pw[m] * b;
            }
            const cplx *tb = T.tab + T.t2l[l] + (int64_t)il_off[k] * rl;
            for (int j = m; j < rl; j += 64) lt[w][j] = tb[j];
        }
        __syncthreads();
        if (act && m <= p) {
            /* L~_m += (-1)^m [ sum_{n<0} conj(M~_|n|) t_{n-m}
                               + sum_{0<=n<m} s^{2n} M~_n t_{n-m} + s^{2m} sum_{n>=m} M~_n t_{n-m} ]
               (t_k = O~_k of the list box's offset); the multipoles are read as
               broadcasts, the table row by consecutive lanes */
            const cplx *tw = &lt[w][2 * p - m];
            cplx a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0), h0 = mk(0.0, 0.0), h1 = mk(0.0, 0.0);
#pragma unroll 4
            for (int n = 1; n <= p; ++n) {
                const cplx t = tw[-n];
                if (SLP) a0 = a0 + conj(lm[w][0][n]) * t;
                if (DLP) a1 = a1 + conj(lm[w][1][n]) * t;
            }
#pragma unroll 4
            for (int n = 0; n <= p; ++n) {
                const cplx t = tw[n];
                const bool lo = n < m;
                if (SLP) {
                    const cplx v = lo ? lmp[w][0][n] : lm[w][0][n];
                    if (lo) a0 = a0 + v * t;
                    else h0 = h0 + v * t;
                }
                if (DLP) {
                    const cplx v = lo ? lmp[w][1][n] : lm[w][1][n];
                    if (lo) a1 = a1 + v * t;
                    else h1 = h1 + v * t;
                }
            }
            acce[0] = acce[0] + a0 + pw[m] * h0;
            acce[1] = acce[1] + a1 + pw[m] * h1;
        }
        __syncthreads();
    }
    if (m <= p) {
        const double sg = (m & 1) ? -1.0 : 1.0;
        part[w][0][m] = accl[0] + sg * acce[0];
        part[w][1][m] = accl[1] + sg * acce[1];
    }
    __syncthreads();
    if (w == 0 && m <= p) {
        cplx s0 = part[0][0][m], s1 = part[0][1][m];
        for (int ww = 1; ww < FMM_DW; ++ww) {
            s0 = s0 + part[ww][0][m];
            s1 = s1 + part[ww][1][m];
        }
        cplx *lo = T.lexp + chunk * T.lch + T.eoff[l];
        if (SLP) lo[(0 * nbx + box) * (p + 1) + m] = s0;
        if (DLP) lo[(1 * nbx + box) * (p + 1) + m] = s1;
    }
}

/* Leaf work: L2P plus the direct sum over the 3x3 neighbourhood.
   MODE 0 (plans): sources of the target's near panels are skipped and the
   near-panel corrections, 1/(2 pi) and the caller order are applied by the
   far-field epilogue; MODE 1 (volume): coincident points are skipped and
   u = phi/(2 pi) + selfc w f. */
struct FmmVol {
    const double *f;
    double selfc;
    double *u;
};

constexpr int FMM_LW = 4; /* waves per leaf work item */

template <bool SLP, bool DLP, int MODE>
__global__ __launch_bounds__(64 * FMM_LW) void fmm_leaf_kernel(FmmDev T, FarArgs A, FmmVol V)
{
    /* FMM_LW waves share the work item's FMM_TILE targets (lane = target) and
       split its tasks: the source tiles of the 3x3 neighbourhood and, as the
       last task, the local expansion; partial sums are added in wave order */
    static_assert(FMM_TILE == 64, "one target per lane");
    __shared__ double sx[FMM_LW][FMM_TILE], sy[FMM_LW][FMM_TILE], sq[FMM_LW][FMM_TILE], sdx[FMM_LW][FMM_TILE],
        sdy[FMM_LW][FMM_TILE];
    __shared__ int32_t spn[FMM_LW][FMM_TILE];
    __shared__ double ps[FMM_LW][FMM_TILE], pd[FMM_LW][FMM_TILE];
    __shared__ cplx lcs[FMM_PMAX + 1], lcd[FMM_PMAX + 1];
    __shared__ int nbox_b0[9], nbox_b1[9], tpre[10];
    const int L = T.L, p = T.p, nb = 1 << L;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int box = T.wbox[blockIdx.x], t0 = T.wt0[blockIdx.x];
    const int t1 = min(t0 + FMM_TILE, T.tstart[box + 1]);
    const int ix = box % nb, iy = box / nb;
    const int tt = t0 + lane;
    const bool valid = tt < t1;
    const int64_t i = valid ? (MODE == 0 ? (int64_t)T.tidx[tt] : (int64_t)tt) : 0;
    const double x = valid ? (MODE == 0 ? A.tx[i] : T.lx[tt]) : 0.0;
    const double y = valid ? (MODE == 0 ? A.ty[i] : T.ly[tt]) : 0.0;
    const double *mu = A.mu;
    const bool local = T.lstart <= L;
    if (local && tid <= p) {
        const int64_t nbx = (int64_t)nb * nb;
        cplx a = mk(0.0, 0.0), b = mk(0.0, 0.0);
        for (int c = 0; c < T.nch[L]; ++c) { /* the partial local expansions, in order */
            const cplx *lp = T.lexp + c * T.lch + T.eoff[L];
            if (SLP) a = a + lp[(0 * nbx + box) * (p + 1) + tid];
            if (DLP) b = b + lp[(1 * nbx + box) * (p + 1) + tid];
        }
        if (SLP) lcs[tid] = a;
        if (DLP) lcd[tid] = b;
    }
    /* the neighbourhood's source ranges (one thread per box) and their tile
       counts, in a fixed order */
    if (tid < 9) {
        const int jx = ix + tid % 3 - 1, jy = iy + tid / 3 - 1;
        int b0 = 0, b1 = 0;
        if (jx >= 0 && jx < nb && jy >= 0 && jy < nb) {
            b0 = T.sstart[jy * nb + jx];
            b1 = T.sstart[jy * nb + jx + 1];
        }
        nbox_b0[tid] = b0;
        nbox_b1[tid] = b1;
    }
    __syncthreads();
    if (tid == 0) {
        tpre[0] = 0;
        for (int k = 0; k < 9; ++k) tpre[k + 1] = tpre[k] + (nbox_b1[k] - nbox_b0[k] + FMM_TILE - 1) / FMM_TILE;
    }
    /* near list of the target (MODE 0), up to 8 entries in registers */
    int32_t nl[8];
    int32_t nlo = 0, nln = 0;
    if (MODE == 0 && valid) {
        nlo = A.nptr[i];
        nln = A.nptr[i + 1] - nlo;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) nl[q] = (q < nln) ? A.npan[nlo + q] : -3;
    __syncthreads();
    const int ntile = tpre[9], ntask = ntile + (local ? 1 : 0);
    const FarConst fc = far_const(T.alpha);
    double accs = 0.0, accd = 0.0;
    const int nr = (ntask + FMM_LW - 1) / FMM_LW;
    for (int r = 0; r < nr; ++r) {
        const int k = r * FMM_LW + w;
        const bool tile = k < ntile;
        int cnt = 0;
        if (tile) {
            int j9 = 0;
            while (tpre[j9 + 1] <= k) ++j9;
            const int base = nbox_b0[j9] + (k - tpre[j9]) * FMM_TILE, b1 = nbox_b1[j9];
            cnt = min(FMM_TILE, b1 - base);
            const int j = base + lane;
            if (lane < cnt) {
                const int64_t o = T.sidx[j];
                const double wj = T.lw[j];
                sx[w][lane] = T.lx[j];
                sy[w][lane] = T.ly[j];
                if (MODE == 0) {
                    sq[w][lane] = SLP ? wj * A.sigma[o] : 0.0;
                    const double m = DLP ? wj * mu[o] : 0.0;
                    sdx[w][lane] = DLP ? m * T.lnx[j] : 0.0;
                    sdy[w][lane] = DLP ? m * T.lny[j] : 0.0;
                    spn[w][lane] = T.lpan[j];
                } else {
                    sq[w][lane] = wj * V.f[o];
                    sdx[w][lane] = 0.0;
                    sdy[w][lane] = 0.0;
                    spn[w][lane] = -1;
                }
            } else { /* padding slot of an odd count: skipped */
                sx[w][lane] = 0.0;
                sy[w][lane] = 0.0;
                sq[w][lane] = 0.0;
                sdx[w][lane] = 0.0;
                sdy[w][lane] = 0.0;
                spn[w][lane] = -2;
            }
        }
        __syncthreads();
        if (tile && valid) {
#pragma unroll 1
            for (int l = 0; l < cnt; l += 2) {
                const FarTab Tb = far_table();
                const double ex0 = x - sx[w][l], ey0 = y - sy[w][l];
                const double ex1 = x - sx[w][l + 1], ey1 = y - sy[w][l + 1];
                double r20 = fma(ex0, ex0, ey0 * ey0), r21 = fma(ex1, ex1, ey1 * ey1);
                bool k0_ = true, k1_ = true;
                if (MODE == 0) {
                    const int32_t pa = spn[w][l], pb = spn[w][l + 1];
                    bool ea = false, eb = false;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        ea |= pa == nl[q];
                        eb |= pb == nl[q];
                    }
                    for (int q = 8; q < nln; ++q) { /* long near lists (rare) */
                        const int32_t v = A.npan[nlo + q];
                        ea |= pa == v;
                        eb |= pb == v;
                    }
                    k0_ = !ea && pa != -2;
                    k1_ = !eb && pb != -2;
                } else {
                    k0_ = r20 != 0.0 && spn[w][l] != -2;
                    k1_ = r21 != 0.0 && spn[w][l + 1] != -2;
                }
                r20 = k0_ ? r20 : 1.0;
                r21 = k1_ ? r21 : 1.0;
                K01 o0, o1;
                k01_far2<SLP, DLP>(Tb, fc, r20, r21, o0, o1);
                if (SLP) {
                    const double q0 = k0_ ? sq[w][l] : 0.0, q1 = k1_ ? sq[w][l + 1] : 0.0;
                    accs = fma(o1.k0, q1, fma(o0.k0, q0, accs));
                }
                if (DLP) {
                    const double a0 = k0_ ? o0.ak1r : 0.0, a1 = k1_ ? o1.ak1r : 0.0;
                    accd = fma(a1, fma(ex1, sdx[w][l + 1], ey1 * sdy[w][l + 1]),
                               fma(a0, fma(ex0, sdx[w][l], ey0 * sdy[w][l]), accd));
                }
            }
        } else if (k == ntile && local && valid) {
            const cplx c = fmm_center(T, L, ix, iy);
            const double dxv = x - c.re, dyv = y - c.im, rr = sqrt(dxv * dxv + dyv * dyv);
            const cplx u = rr > 0.0 ? mk(dxv / rr, dyv / rr) : mk(1.0, 0.0);
            double a2[2];
            fmm_l2p<SLP, DLP>(lcs, lcd, p, T.alpha * rr, T.sig[L], u, a2);
            accs += a2[0];
            accd += a2[1];
        }
        __syncthreads();
    }
    ps[w][lane] = accs;
    pd[w][lane] = accd;
    __syncthreads();
    if (w != 0 || !valid) return;
    double s_ = ps[0][lane], d_ = pd[0][lane];
    for (int ww = 1; ww < FMM_LW; ++ww) {
        s_ += ps[ww][lane];
        d_ += pd[ww][lane];
    }
    if (MODE == 0) {
        far_epilogue<SLP, DLP>(A, mu, i, s_, d_);
    } else {
        const int64_t o = T.sidx[tt];
        V.u[o] = fma(INV_2PI, s_, V.selfc * T.lw[tt] * V.f[o]);
    }
}

} // namespace mhlp
