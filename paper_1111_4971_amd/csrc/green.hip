// green.hip -- FP64 evaluation of the pipe Green function on the mesh and the
// kernels that turn it into the cached spectra.
//
// R(u, v, w) = 1/(2 pi a b) sum_{m<=mx, n<=my} kappa_mn^{-1} cos(m pi u/a) cos(n pi v/b) g(kappa_mn, w)
// (Eq. 9; Eq. 16 for the z-integrated kind), kappa_mn^2 = (m pi/a)^2 + (n pi/b)^2,
// is needed at the differences u = p hx (p < nx) and sums u = 2 x0 + (p + 2) hx
// (p <= 2nx - 2) of node positions x0 + (i+1) hx, likewise in y, and w = r hz (r < nz):
//   Rbar[p][q][r] = sum_m Cx[p][m] sum_n Cy[q][n] D[m][n][r],
//   Cx[p][m] = cos(pi m u_p / a),  Cy[q][n] = cos(pi n v_q / b),
//   D[m][n][r] = g(kappa_mn, r hz) / (2 pi a b kappa_mn),
// computed as two FP64 matrix products (y contraction per m, then x).
// g is e^{-kappa |w|} (Eq. 9) or the IGF z-kernel of Eq. 15, evaluated in a form
// free of cancellation:
//   r = 0:  g = 2 (x - 1 + e^{-x}) / x^2,  x = kappa hz  (Taylor series for x < 0.5)
//   r >= 1: g = e^{-x (r - 1)} (expm1(-x) / x)^2
// (the bracket of Eq. 15 is e^{-kappa(|w| - hz)} (1 - e^{-x})^2 for |w| >= hz).
#include <cmath>

#include "pipe_internal.h"

namespace pipe {

// cos(pi * t * s) for integer t, with the product reduced modulo 2 exactly:
// t*s = hi + lo (two-product), hi - 2 round(hi/2) is exact.
__device__ __forceinline__ double cospi_prod(double t, double s) {
    const double hi = t * s;
    const double lo = fma(t, s, -hi);
    const double red = hi - 2.0 * rint(0.5 * hi);
    return cospi(red + lo);
}

// t * s reduced modulo 2 (exactly, then the rounding error of the product added back)
__device__ __forceinline__ double red2_prod(double t, double s) {
    const double hi = t * s;
    const double lo = fma(t, s, -hi);
    return (hi - 2.0 * rint(0.5 * hi)) + lo;
}

// Cosines of the distances the four terms need along one axis, for modes m = 1..M:
// rows p < nconv:  cos(pi m p h / a)                        (differences, p h)
// rows nconv + p:  cos(pi m (2 x0 + (p + 2) h) / a), p < ncorr  (sums X_i + X_i')
// with s = h / a and off = 2 x0 / a.
__global__ void cos_table_kernel(double* out, int nconv, int ncorr, int m, double s, double off) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)(nconv + ncorr) * m) return;
    const int p = (int)(i / m), mm = (int)(i % m) + 1;
    if (p < nconv) {
        out[i] = cospi_prod((double)p * (double)mm, s);
    } else {
        const double t = red2_prod((double)(p - nconv + 2) * (double)mm, s) + red2_prod((double)mm, off);
        out[i] = cospi(t);
    }
}

__device__ __forceinline__ double igf_g(double x, int r) {
    if (r == 0) {
        if (x < 0.5) {
            // 2 sum_{j>=0} (-x)^j / (j+2)!
            double term = 1.0, fact = 2.0, acc = 0.0;
#pragma unroll
            for (int j = 0; j < 22; ++j) {
                acc += term / fact;
                term *= -x;
                fact *= (double)(j + 3);
            }
            return 2.0 * acc;
        }
        return 2.0 * (x + expm1(-x)) / (x * x);
    }
    const double q = expm1(-x) / x;
    return exp(-x * (double)(r - 1)) * q * q;
}

__global__ void modes_kernel(double* d, int mx, int my, int rz, double a, double b, double hz, int igf,
                             double norm) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)mx * my * rz;
    if (i >= total) return;
    const int r = (int)(i % rz);
    const int n = (int)((i / rz) % my) + 1;
    const int m = (int)(i / ((long)rz * my)) + 1;
    const double km = (double)m / a, kn = (double)n / b;
    const double kap = M_PI * sqrt(km * km + kn * kn);
    double g;
    if (igf)
        g = igf_g(kap * hz, r);
    else
        g = exp(-kap * ((double)r * hz));
    d[i] = norm * g / kap;
}

// C[b] (M x N) = A[b] (M x K) * B[b] (K x N), row-major FP64, 64 x 64 tiles, 4 x 4 per thread.
constexpr int GT = 64, GK = 16;
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double* __restrict__ A, const double* __restrict__ B,
                                                        double* __restrict__ C, int M, int N, int K, long lda,
                                                        long ldb, long ldc, long sA, long sB, long sC) {
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int bz = blockIdx.z;
    A += bz * sA;
    B += bz * sB;
    C += bz * sC;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += GK) {
        for (int i = threadIdx.x; i < GT * GK; i += 256) {
            const int mm = i / GK, kk = i % GK;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < M && gk < K) ? A[gm * lda + gk] : 0.0;
            const int kb = i / GT, nn = i % GT;
            const int gkb = k0 + kb, gn = n0 + nn;
            Bs[kb][nn] = (gkb < K && gn < N) ? B[gkb * ldb + gn] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty + 16 * i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx + 16 * j;
            if (gn < N) C[gm * ldc + gn] = acc[i][j];
        }
    }
}

// xi[p][q][s] = Rbar at term ab's distance for slot (p, q, s), zero in unused slots
// (Appendix, Eq. A.3 for convolution slots, remark A.9 for correlation slots).
// Rbar rows along x: 0..n-1 the differences |m| h, n..3n-2 the sums 2 x0 + (p + 2) h:
//   convolution slot p: m = p (p <= L/2) or p - L; used when |m| <= n - 1 -> row |m|;
//   correlation slot p: used when p <= 2n - 2 (p = i + i') -> row n + p.
__device__ __forceinline__ int conv_slot(int p, int L, int n) {
    const int m = (p <= L / 2) ? p : p - L;
    const int am = m < 0 ? -m : m;
    return am <= n - 1 ? am : -1;
}
__device__ __forceinline__ int corr_slot(int p, int n) { return p <= 2 * n - 2 ? n + p : -1; }

// zid: the z index is the plane distance itself (lz = nz planes, no mirror
// slots), for the banded spectra, which are transformed in x and y only.
__global__ void arrange_kernel(double* xi, const double* __restrict__ rbar, int nx, int ny, int nz, int lx,
                               int ly, int lz, int xcorr, int ycorr, int zid) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)lx * ly * lz;
    if (i >= total) return;
    const int s = (int)(i % lz);
    const int q = (int)((i / lz) % ly);
    const int p = (int)(i / ((long)lz * ly));
    const int ip = xcorr ? corr_slot(p, nx) : conv_slot(p, lx, nx);
    const int iq = ycorr ? corr_slot(q, ny) : conv_slot(q, ly, ny);
    const int is = zid ? s : conv_slot(s, lz, nz);
    double v = 0.0;
    if (ip >= 0 && iq >= 0 && is >= 0) v = rbar[((long)ip * (3 * ny - 1) + iq) * nz + is];
    xi[i] = v;
}

// Free-space Green array of Eq. 5: slot (p, q, s) holds G = 1/r at the grid
// distance (|m| hx, |n| hy, |l| hz) of its convolution slot (Appendix A.3),
// g0 at zero distance (Eq. 3 is singular there), zero in unused slots.
__global__ void free_arrange_kernel(double* xi, int nx, int ny, int nz, int lx, int ly, int lz, double hx,
                                    double hy, double hz, double g0) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)lx * ly * lz;
    if (i >= total) return;
    const int s = (int)(i % lz);
    const int q = (int)((i / lz) % ly);
    const int p = (int)(i / ((long)lz * ly));
    const int ip = conv_slot(p, lx, nx), iq = conv_slot(q, ly, ny), is = conv_slot(s, lz, nz);
    double v = 0.0;
    if (ip >= 0 && iq >= 0 && is >= 0) {
        if (ip == 0 && iq == 0 && is == 0) {
            v = g0;
        } else {
            const double u = ip * hx, w = iq * hy, z = is * hz;
            v = 1.0 / sqrt(u * u + w * w + z * z);
        }
    }
    xi[i] = v;
}

// Orbit table from the full forward spectrum S[lx][ly][nh] (FP64 complex, kz = lz/2
// packed into slot 0 as A + iB).  term: 0 cc, 1 cr, 2 rc, 3 rr.
// nval = 9 (the four terms) or 1 (T_cc only: free space).
template <typename out_t>
__global__ void compress_kernel(const double2* __restrict__ S, out_t* table, out_t* nyq, int term, int lx, int ly,
                                int nh, int tile, int nval) {
    const int kxo_n = lx / 2 + 1, kyo_n = ly / 2 + 1;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)kxo_n * kyo_n * nh;
    if (i >= total) return;
    const int kz = (int)(i % nh);
    const int kyo = (int)((i / nh) % kyo_n);
    const int kxo = (int)(i / ((long)nh * kyo_n));
    const int ntiles = (nh + tile - 1) / tile;
    // tile-blocked position of (kxo, kyo, kz), plane p at ti + p * tile; kz = lz/2 at ni + p
    const long ti = ((((long)kyo * ntiles + kz / tile) * kxo_n + kxo) * nval) * tile + kz % tile;
    const long ni = ((long)kyo * kxo_n + kxo) * nval;
    auto at = [&](int kx, int ky) { return S[((long)kx * ly + ky) * nh + kz]; };
    // value at (kx, ky): main (kz) and, for kz = 0, the kz = lz/2 part
    auto split = [&](int kx, int ky, double2& A, double2& B) {
        const double2 p = at(kx, ky);
        if (kz != 0) {
            A = p;
            B = make_double2(0.0, 0.0);
            return;
        }
        const double2 m = at((lx - kx) % lx, (ly - ky) % ly);  // P(-k)
        A = make_double2(0.5 * (p.x + m.x), 0.5 * (p.y - m.y));
        // (p - conj m) / (2i) = -i (p - conj m) / 2
        const double dx = p.x - m.x, dy = p.y + m.y;
        B = make_double2(0.5 * dy, -0.5 * dx);
    };
    double2 A, B, A2, B2;
    split(kxo, kyo, A, B);
    auto put = [&](int pl, double va, double vb) {
        if (pl >= nval) return;
        table[ti + (long)pl * tile] = (out_t)va;
        if (kz == 0) nyq[ni + pl] = (out_t)vb;
    };
    switch (term) {
        case 0: put(0, A.x, B.x); break;
        case 1: put(1, A.x, B.x); put(2, A.y, B.y); break;
        case 2: put(3, A.x, B.x); put(4, A.y, B.y); break;
        default:
            split((lx - kxo) % lx, kyo, A2, B2);
            put(5, A.x, B.x);
            put(6, A.y, B.y);
            put(7, A2.x, B2.x);
            put(8, A2.y, B2.y);
            break;
    }
}

// Tile-blocked table -> 9 planes [p][kx][ky][kz] followed by 9 planes [p][kx][ky] (kz = lz/2);
// planes p >= nval (absent terms) are zero.
template <typename T_>
__global__ void untile_kernel(const T_* __restrict__ table, const T_* __restrict__ nyq, T_* out, int lx, int ly,
                              int nh, int tile, int nval) {
    const int kxo_n = lx / 2 + 1, kyo_n = ly / 2 + 1;
    const long plane = (long)kxo_n * kyo_n * nh;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane) return;
    const int kz = (int)(i % nh);
    const int kyo = (int)((i / nh) % kyo_n);
    const int kxo = (int)(i / ((long)nh * kyo_n));
    const int ntiles = (nh + tile - 1) / tile;
    const long ti = ((((long)kyo * ntiles + kz / tile) * kxo_n + kxo) * nval) * tile + kz % tile;
    for (int p = 0; p < 9; ++p) out[p * plane + i] = p < nval ? table[ti + (long)p * tile] : (T_)0;
    if (kz == 0) {
        const long np_ = (long)kxo_n * kyo_n, ni = (long)kxo * kyo_n + kyo;
        for (int p = 0; p < 9; ++p)
            out[9 * plane + p * np_ + ni] = p < nval ? nyq[((long)kyo * kxo_n + kxo) * nval + p] : (T_)0;
    }
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_cos_table(double* out, int nconv, int ncorr, int m, double s, double off, hipStream_t st) {
    const long n = (long)(nconv + ncorr) * m;
    hipLaunchKernelGGL(cos_table_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, out, nconv, ncorr, m, s, off);
    return hipGetLastError();
}

hipError_t launch_modes(double* d, int mx, int my, int rz, double a, double b, double hz, int igf, double norm,
                        hipStream_t st) {
    const long n = (long)mx * my * rz;
    hipLaunchKernelGGL(modes_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, mx, my, rz, a, b, hz, igf,
                       norm);
    return hipGetLastError();
}

hipError_t launch_gemm_f64(const double* A, const double* B, double* C, int M, int N, int K, long lda, long ldb,
                           long ldc, long sA, long sB, long sC, int batch, hipStream_t st) {
    dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)batch);
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, A, B, C, M, N, K, lda, ldb, ldc, sA, sB, sC);
    return hipGetLastError();
}

hipError_t launch_arrange(double* xi, const double* rbar, int nx, int ny, int nz, int lx, int ly, int lz, int xcorr,
                          int ycorr, hipStream_t st, bool z_identity) {
    const long n = (long)lx * ly * lz;
    if (z_identity && lz != nz) return hipErrorInvalidValue;
    hipLaunchKernelGGL(arrange_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, xi, rbar, nx, ny, nz, lx, ly,
                       lz, xcorr, ycorr, (int)z_identity);
    return hipGetLastError();
}

hipError_t launch_free_arrange(double* xi, int nx, int ny, int nz, int lx, int ly, int lz, double hx, double hy,
                              double hz, double g0, hipStream_t st) {
    const long n = (long)lx * ly * lz;
    hipLaunchKernelGGL(free_arrange_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, xi, nx, ny, nz, lx, ly, lz,
                       hx, hy, hz, g0);
    return hipGetLastError();
}

hipError_t launch_compress(const void* spec, void* table, void* nyq, int real_bytes, int term, int lx, int ly,
                           int nh, int tile, hipStream_t st, int nval) {
    const long n = (long)(lx / 2 + 1) * (ly / 2 + 1) * nh;
    if (tile < 1) return hipErrorInvalidValue;
    if (real_bytes == 8)
        hipLaunchKernelGGL(compress_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           (const double2*)spec, (double*)table, (double*)nyq, term, lx, ly, nh, tile, nval);
    else
        hipLaunchKernelGGL(compress_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           (const double2*)spec, (float*)table, (float*)nyq, term, lx, ly, nh, tile, nval);
    return hipGetLastError();
}

hipError_t launch_untile(const void* table, const void* nyq, void* out, int real_bytes, int lx, int ly, int nh,
                         int tile, hipStream_t st, int nval) {
    const long n = (long)(lx / 2 + 1) * (ly / 2 + 1) * nh;
    if (tile < 1) return hipErrorInvalidValue;
    if (real_bytes == 8)
        hipLaunchKernelGGL(untile_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const double*)table,
                           (const double*)nyq, (double*)out, lx, ly, nh, tile, nval);
    else
        hipLaunchKernelGGL(untile_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const float*)table,
                           (const float*)nyq, (float*)out, lx, ly, nh, tile, nval);
    return hipGetLastError();
}

}  // namespace pipe
