/* Particular solution of the modified Stokes equations on a periodic box
   (Sec. 2.1, the periodic stokeslet multiplier; Sec. 3.1.2, grid transforms and
   type-2 sums at the boundary nodes), FP64.

   Box [x0, x0 + Lb) x [y0, y0 + Lb), grid x_a = x0 + a Lb/M, y_b = y0 + b Lb/M,
   fields stored [b][a] (row = y).  Coefficients F^(k) = (1/M^2) sum F e^{-i k.(x - x0)},
   k = (2 pi/Lb)(k1, k2), k1, k2 in [-M/2, M/2) in FFT order; Nyquist coefficients are
   zeroed in every result.
     u^_j = S^_jl F^_l,  S^_jl = (delta_jl - k_j k_l/|k|^2)/(alpha^2 + |k|^2),  S^(0) = I/alpha^2,
     d u_j/d x_m  <-  i k_m u^_j,   u_j(x) = sum_k u^_j(k) e^{i k.(x - x0)} at points.
   FFTs: Stockham radix-2 in LDS, one block per line (rows, then columns read
   with a stride), twiddles e^{-2 pi i j/M} from a host table. */
#pragma once

namespace mhlp {

/* one length-M FFT per block along a line of a complex array: element e of
   line l at base[l * line_stride + e * elem_stride]; sign -1 forward, +1 inverse
   (no scaling); M/2 threads; tw[j] = e^{-2 pi i j/M}, j < M/2 */
__global__ void fft_lines_kernel(cplx *__restrict__ data, int M, int64_t elem_stride, int64_t line_stride,
                                 int64_t field_stride, const cplx *__restrict__ tw, double sign)
{
    extern __shared__ cplx fsh[];
    cplx *a = fsh, *b = fsh + M;
    cplx *base = data + (int64_t)blockIdx.y * field_stride + (int64_t)blockIdx.x * line_stride;
    const int j = threadIdx.x, h = M >> 1;
    a[j] = base[(int64_t)j * elem_stride];
    a[j + h] = base[(int64_t)(j + h) * elem_stride];
    __syncthreads();
    for (int Ns = 1; Ns < M; Ns <<= 1) {
        const int k = j & (Ns - 1);
        cplx w = tw[k * (h / Ns)];
        if (sign > 0.0) w = conj(w);
        const cplx in0 = a[j], in1 = a[j + h] * w;
        const int d = (j - k) * 2 + k;
        b[d] = in0 + in1;
        b[d + Ns] = in0 - in1;
        __syncthreads();
        cplx *t = a;
        a = b;
        b = t;
    }
    base[(int64_t)j * elem_stride] = a[j];
    base[(int64_t)(j + h) * elem_stride] = a[j + h];
}

/* real grid fields [nf][M*M] -> complex */
__global__ void fft_load_real_kernel(const double *__restrict__ f, int64_t n, cplx *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = mk(f[i], 0.0);
}

/* spectra of the two forcing components (unnormalised forward FFTs) -> u^_1, u^_2
   and, if grad, i k_x u^_1, i k_y u^_1, i k_x u^_2, i k_y u^_2 */
__global__ void stokes_multiplier_kernel(const cplx *__restrict__ Fh, int M, double Lb, double alpha, bool grad,
                                         cplx *__restrict__ Uh)
{
    const int64_t MM = (int64_t)M * M;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= MM) return;
    const int r = (int)(i / M), c = (int)(i % M);
    const bool nyq = r == M / 2 || c == M / 2;
    const double w = 2.0 * PI / Lb;
    const double k1 = w * (c < M / 2 ? c : c - M), k2 = w * (r < M / 2 ? r : r - M);
    const double inv = 1.0 / ((double)M * (double)M);
    const cplx f1 = inv * Fh[i], f2 = inv * Fh[MM + i];
    const double kk = k1 * k1 + k2 * k2, den = 1.0 / (alpha * alpha + kk);
    cplx u1 = mk(0.0, 0.0), u2 = mk(0.0, 0.0);
    if (!nyq) {
        if (kk > 0.0) {
            const double ikk = 1.0 / kk;
            const double p11 = 1.0 - k1 * k1 * ikk, p22 = 1.0 - k2 * k2 * ikk, p12 = -k1 * k2 * ikk;
            u1 = den * (p11 * f1 + p12 * f2);
            u2 = den * (p12 * f1 + p22 * f2);
        } else {
            u1 = den * f1;
            u2 = den * f2;
        }
    }
    Uh[i] = u1;
    Uh[MM + i] = u2;
    if (grad) {
        const cplx iu1 = mk(-u1.im, u1.re), iu2 = mk(-u2.im, u2.re); /* i u^ */
        Uh[2 * MM + i] = k1 * iu1;
        Uh[3 * MM + i] = k2 * iu1;
        Uh[4 * MM + i] = k1 * iu2;
        Uh[5 * MM + i] = k2 * iu2;
    }
}

__global__ void fft_store_real_kernel(const cplx *__restrict__ in, int64_t n, double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i].re;
}

/* type-2 sums of u^_1, u^_2 at points: block (point chunk, row chunk of FT2_R
   rows); columns in tiles of FT2_C staged in LDS; per thread e^{i k1 x'} by
   recurrence re-anchored with sincos at every tile, one accumulator per row;
   partial[chunk][comp][point] */
constexpr int FT2_R = 8, FT2_C = 32, FT2_T = 256;

__global__ __launch_bounds__(FT2_T) void type2_points_kernel(const cplx *__restrict__ Uh, int M, double Lb,
                                                             double x0, double y0, const double *__restrict__ px,
                                                             const double *__restrict__ py, int64_t n,
                                                             double *__restrict__ partial)
{
    __shared__ cplx tile[2][FT2_R][FT2_C];
    const int64_t MM = (int64_t)M * M;
    const int64_t i = blockIdx.x * (int64_t)FT2_T + threadIdx.x;
    const bool valid = i < n;
    const int r0 = blockIdx.y * FT2_R;
    const double w = 2.0 * PI / Lb;
    const double xr = valid ? px[i] - x0 : 0.0, yr = valid ? py[i] - y0 : 0.0;
    double sr, cr;
    sincos(w * xr, &sr, &cr);
    const cplx ex1 = mk(cr, sr);
    cplx acc1[FT2_R], acc2[FT2_R];
#pragma unroll
    for (int q = 0; q < FT2_R; ++q) acc1[q] = acc2[q] = mk(0.0, 0.0);
    for (int c0 = 0; c0 < M; c0 += FT2_C) {
        const int nc = min(FT2_C, M);
        __syncthreads();
        for (int t = threadIdx.x; t < 2 * FT2_R * nc; t += FT2_T) {
            const int comp = t / (FT2_R * nc), rem = t % (FT2_R * nc), q = rem / nc, cc = rem % nc;
            tile[comp][q][cc] = Uh[comp * MM + (int64_t)(r0 + q) * M + c0 + cc];
        }
        __syncthreads();
        /* e^{i k1 x'} at the tile's first column, exactly */
        const int cs = c0 < M / 2 ? c0 : c0 - M;
        double s0, c0v;
        sincos(w * cs * xr, &s0, &c0v);
        cplx e = mk(c0v, s0);
        for (int cc = 0; cc < nc; ++cc) {
            if (cc > 0) {
                const int cg = c0 + cc;
                if (cg == M / 2) { /* the negative frequencies start here */
                    double s1, c1;
                    sincos(w * (double)(cg - M) * xr, &s1, &c1);
                    e = mk(c1, s1);
                } else {
                    e = e * ex1;
                }
            }
#pragma unroll
            for (int q = 0; q < FT2_R; ++q) {
                acc1[q] = acc1[q] + tile[0][q][cc] * e;
                acc2[q] = acc2[q] + tile[1][q][cc] * e;
            }
        }
    }
    if (!valid) return;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < FT2_R; ++q) {
        const int r = r0 + q;
        const int ks = r < M / 2 ? r : r - M;
        double sy, cy;
        sincos(w * ks * yr, &sy, &cy);
        const cplx ey = mk(cy, sy);
        s1 += (acc1[q] * ey).re;
        s2 += (acc2[q] * ey).re;
    }
    partial[((int64_t)blockIdx.y * 2 + 0) * n + i] = s1;
    partial[((int64_t)blockIdx.y * 2 + 1) * n + i] = s2;
}

__global__ void type2_reduce_kernel(const double *__restrict__ partial, int nchunk, int64_t n, double *__restrict__ up)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nchunk; ++k) {
        s1 += partial[((int64_t)k * 2 + 0) * n + i];
        s2 += partial[((int64_t)k * 2 + 1) * n + i];
    }
    up[i] = s1;
    up[n + i] = s2;
}

/* ---- type-2 sums at points by a non-uniform FFT (spreading kernel) ----
   The exponential-of-semicircle kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)),
   |z| < 1, spans NU_W points of a fine grid of Mf = 2M points (spacing hf):
     b(y_l) = sum_k c(k) e^{i k (y_l - x0)},  c(k) = u^(k) hf^2 / (psi^(k1) psi^(k2)),
     u(x) ~ sum_{l near x} b(y_l) phi_h(x1 - y_l1) phi_h(x2 - y_l2),
   psi^ the Fourier transform of phi_h(x) = phi(2x/(NU_W hf)) (Poisson summation;
   the 2x oversampling and the kernel's decay keep the aliased terms ~1e-14 of
   sum |u^|).  b comes from an inverse FFT of size Mf of the zero-padded c. */
constexpr int NU_W = 14;
constexpr double NU_BETA = 2.30 * NU_W;

/* c = u^ corr(k1) corr(k2) placed in the fine spectrum (zero outside |k| < M/2);
   corr[j] = hf / psi^(k_j) in coarse FFT order */
__global__ void nufft_fine_spectrum_kernel(const cplx *__restrict__ Uh, int M, int Mf, const double *__restrict__ corr,
                                           cplx *__restrict__ fine)
{
    const int64_t MMf = (int64_t)Mf * Mf;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 2 * MMf) return;
    const int comp = (int)(i / MMf);
    const int64_t e = i % MMf;
    const int r = (int)(e / Mf), c = (int)(e % Mf);
    const int h = M / 2;
    const int jr = r < h ? r : (r >= Mf - h ? r - Mf + M : -1);
    const int jc = c < h ? c : (c >= Mf - h ? c - Mf + M : -1);
    cplx v = mk(0.0, 0.0);
    if (jr >= 0 && jc >= 0) v = (corr[jr] * corr[jc]) * Uh[(int64_t)comp * M * M + (int64_t)jr * M + jc];
    fine[i] = v;
}

__device__ __forceinline__ double nu_phi(double z)
{
    const double q = 1.0 - z * z;
    return q > 0.0 ? exp(NU_BETA * (sqrt(q) - 1.0)) : 0.0;
}

/* u at the points from the fine-grid values b (real parts), NU_W x NU_W stencil */
__global__ void nufft_interp_kernel(const cplx *__restrict__ fine, int Mf, double hf, double x0, double y0,
                                    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
                                    double *__restrict__ up)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xf = (px[i] - x0) / hf, yf = (py[i] - y0) / hf;
    const int ix0 = (int)floor(xf) - NU_W / 2 + 1, iy0 = (int)floor(yf) - NU_W / 2 + 1;
    double wx[NU_W], wy[NU_W];
#pragma unroll
    for (int a = 0; a < NU_W; ++a) {
        wx[a] = nu_phi((xf - (ix0 + a)) * (2.0 / NU_W));
        wy[a] = nu_phi((yf - (iy0 + a)) * (2.0 / NU_W));
    }
    const int64_t MMf = (int64_t)Mf * Mf;
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < NU_W; ++b) {
        const int ry = ((iy0 + b) % Mf + Mf) % Mf;
        double t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int a = 0; a < NU_W; ++a) {
            const int cx = ((ix0 + a) % Mf + Mf) % Mf;
            const int64_t o = (int64_t)ry * Mf + cx;
            t1 = fma(wx[a], fine[o].re, t1);
            t2 = fma(wx[a], fine[MMf + o].re, t2);
        }
        s1 = fma(wy[b], t1, s1);
        s2 = fma(wy[b], t2, s2);
    }
    up[i] = s1;
    up[n + i] = s2;
}

/* (u.grad) u from u [2][n] and its gradient g [4][n] (du1/dx, du1/dy, du2/dx, du2/dy) */
__global__ void advect_kernel(const double *__restrict__ u, const double *__restrict__ g, int64_t n,
                              double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u1 = u[i], u2 = u[n + i];
    out[i] = fma(u1, g[i], u2 * g[n + i]);
    out[n + i] = fma(u1, g[2 * n + i], u2 * g[3 * n + i]);
}

/* out = sum_{k < nterm} c_k x_k over n elements (terms added in order) */
constexpr int LC_MAX = 16;
struct LinComb {
    const double *x[LC_MAX];
    double c[LC_MAX];
    int nterm;
};

__global__ void lincomb_kernel(LinComb T, int64_t n, double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = T.c[0] * T.x[0][i];
    for (int k = 1; k < T.nterm; ++k) s = fma(T.c[k], T.x[k][i], s);
    out[i] = s;
}

} // namespace mhlp
