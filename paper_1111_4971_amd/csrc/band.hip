// band.hip -- neighbouring-plane z sums (Eq. 17-18).  When the z dependence of
// the Green function is negligible beyond nb planes, the potential on plane k is
//   phi[., ., k] = hx hy hz sum_{d=-nb..nb} (2-D mixed conv/corr of rho[., ., k-d]
//                                            with the slice of G at z distance |d| hz)
// so the z transform drops out: the planes are transformed in y and x only, the
// product sums 2 nb + 1 plane products per output plane, and the Green spectra
// are nb + 1 two-dimensional slices.
//
//   B1 y forward, real planes -> A (nx, ly, nz) complex      [strided_real_kernel<fwd>]
//   B2 x forward of planes z0-nb .. z0+T+nb-1, banded product,
//      x inverse of planes z0 .. z0+T-1, A -> B               [xband_kernel]
//   B3 y inverse B -> real planes, scaled                     [strided_real_kernel<inv>]
#include "pass_common.h"

namespace pipe {

// y pass with real input (forward: rho -> complex) or real output (inverse:
// complex -> scaled real part).  Same block shape as the complex y pass.
template <typename real, int N, int T, bool INV>
__global__ __launch_bounds__(ce_max(1, 256 / ((N / Plan<N>::E) * T)) * (N / Plan<N>::E) * T)
void strided_real_kernel(const void* in, void* out, int n_in, int n_out, long in_es, long out_es, long ncols,
                         long in_ss, long out_ss, long nslabs, real scale, const cplx<real>* __restrict__ tw) {
    using C = cplx<real>;
    constexpr int P = N / Plan<N>::E, SPW = ce_max(1, 256 / (P * T));
    __shared__ C lds[SPW * N * T];
    __shared__ C s_tw[N];
    tw = stage_twiddles(s_tw, tw, N);
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, s = threadIdx.x / (T * P);
    const long slab = (long)blockIdx.y * SPW + s;
    const long col = (long)blockIdx.x * T + c;
    const bool active = slab < nslabs && col < ncols;
    const long ioff = active ? slab * in_ss + col : 0;
    const long ooff = active ? slab * out_ss + col : 0;
    LdsCol<C, T> view{lds + s * N * T + c};
    fft_line<N, INV, false>(
        t, tw,
        [&](int e) -> C {
            if (!(active && e < n_in)) return cmake<C>(0, 0);
            if constexpr (INV) return reinterpret_cast<const C*>(in)[ioff + e * in_es];
            else return cmake<C>(reinterpret_cast<const real*>(in)[ioff + e * in_es], (real)0);
        },
        [&](int e, C v) {
            if (!(active && e < n_out)) return;
            if constexpr (INV) reinterpret_cast<real*>(out)[ooff + e * out_es] = v.x * scale;
            else reinterpret_cast<C*>(out)[ooff + e * out_es] = v;
        },
        view);
}

// Planes per block of the banded x pass: a power of two <= 16 with at most
// 512 threads (two ky lines x P threads x T planes) and 2 N T complex of LDS
// within PIPE_LDS_CAP.
template <typename real, int N> constexpr int band_T() {
    constexpr int P = N / Plan<N>::E;
    int t = 16;
    while (t > 1 && (2 * P * t > 512 || 2 * N * t * 2 * (int)sizeof(real) > PIPE_LDS_CAP)) t /= 2;
    return t;
}

// Block (tile, ky): the two lines ky and -ky of T consecutive output planes
// z0 = tile T ...  The input planes z0 - nb .. z0 + T + nb - 1 are transformed
// along x T at a time into LDS; after each chunk every (kx orbit, output plane)
// item of this thread adds the products of the chunk's planes within nb of it
// to register accumulators.  The accumulators then replace the LDS lines and
// are transformed back.  Banded table: 9 values per (ky orbit, |d|, kx orbit)
// at ((kyo (nb + 1) + |d|) (N/2 + 1) + kxo) 9, same plane order as the 3-D
// orbit table.
template <typename real, int N, bool ADJ>
__global__ __launch_bounds__((2 * (N / Plan<N>::E) * band_T<real, N>()))
void xband_kernel(const cplx<real>* __restrict__ in, cplx<real>* __restrict__ out, int nx, int ly, int nz, int nb,
                  const real* __restrict__ table, const cplx<real>* __restrict__ tw) {
    using C = cplx<real>;
    constexpr int T = band_T<real, N>();
    constexpr int P = N / Plan<N>::E, NT = 2 * P * T, NKX = N / 2 + 1;
    constexpr int IMAX = (NKX * T + NT - 1) / NT;   // (orbit, plane) items per thread
    __shared__ C lds[2 * N * T];
    __shared__ C s_tw[N];
    tw = stage_twiddles(s_tw, tw, N);
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, l = threadIdx.x / (T * P);
    const unsigned ntile = gridDim.x;
    const unsigned lid = xcd_remap(blockIdx.x + ntile * blockIdx.y, ntile * gridDim.y);
    const int tile = (int)(lid % ntile);
    const int ky = (int)(lid / ntile);
    const int kyl = l == 0 ? ky : (ly - ky) % ly;
    const bool self = (ky == 0) || (2 * ky == ly);
    const int z0 = tile * T;
    const long xs = (long)ly * nz;
    const real* trow = table + (long)ky * (nb + 1) * NKX * 9;
    LdsCol<C, T> view{lds + l * N * T + c};

    C acc[IMAX][4];
#pragma unroll
    for (int i = 0; i < IMAX; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = cmake<C>(0, 0);

    // input column cc (0 <= cc < T + 2 nb) is plane z0 - nb + cc; output plane
    // z0 + c2 takes column cc = c2 + nb - d for d in [-nb, nb]
    const int ncol = T + 2 * nb;
    const int nchunk = (ncol + T - 1) / T;
    for (int ch = 0; ch < nchunk; ++ch) {
        if (ch > 0) __syncthreads();   // previous chunk's products have read the LDS
        const int z = z0 - nb + ch * T + c;
        const bool act = ch * T + c < ncol && z >= 0 && z < nz;
        const C* line = in + (act ? (long)kyl * nz + z : 0);
        fft_line<N, false, false>(
            t, tw, [&](int e) -> C { return (act && e < nx) ? line[e * xs] : cmake<C>(0, 0); },
            [&](int e, C v) { view.set(e, v); }, view);
        __syncthreads();
        // planes of this chunk that lie inside the mesh
        const int zc0 = z0 - nb + ch * T;
        const int jmin = ce_max(0, -zc0);
        const int jmax = min(T, min(ncol - ch * T, nz - zc0));   // exclusive
#pragma unroll
        for (int i = 0; i < IMAX; ++i) {
            const int w = threadIdx.x + i * NT;
            if (w >= NKX * T) break;
            const int c2 = w % T, o = w / T;
            const int on = (N - o) % N;
            // column j of the chunk is cc = ch T + j, d = c2 + nb - cc
            const int lo = ce_max(jmin, c2 - ch * T);
            const int hi = min(jmax, c2 - ch * T + 2 * nb + 1);
            for (int j = lo; j < hi; ++j) {
                const int d = c2 + nb - ch * T - j;
                const int ad = d < 0 ? -d : d;
                const C r[4] = {lds[o * T + j], lds[on * T + j], lds[(N + o) * T + j], lds[(N + on) * T + j]};
                const Orbit<real> ob = load_orbit(trow + ((long)ad * NKX + o) * 9, 1);
                C p[4];
                orbit_product<ADJ>(ob, r, p);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] = cadd(acc[i][q], p[q]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
        const int w = threadIdx.x + i * NT;
        if (w >= NKX * T) break;
        const int c2 = w % T, o = w / T;
        const int on = (N - o) % N;
        // o = 0 and o = N/2 are their own mirror: acc[i][0] and acc[i][1] agree there
        lds[o * T + c2] = acc[i][0];
        lds[(N + o) * T + c2] = acc[i][2];
        if (on != o) {
            lds[on * T + c2] = acc[i][1];
            lds[(N + on) * T + c2] = acc[i][3];
        }
    }
    __syncthreads();

    // inverse x transforms of the T output planes, rows i < nx
    const int zo = z0 + c;
    const bool oact = zo < nz && !(l == 1 && self);
    C* oline = out + (oact ? (long)kyl * nz + zo : 0);
    fft_line<N, true, true>(
        t, tw, [&](int e) -> C { return view.get(e); },
        [&](int e, C v) {
            if (oact && e < nx) oline[e * xs] = v;
        },
        view);
}

// Banded orbit table from the 2-D forward spectra S[lx][ly][D] (FP64 complex)
// of one term's arrangement; term: 0 cc, 1 cr, 2 rc, 3 rr.
template <typename out_t>
__global__ void compress_band_kernel(const double2* __restrict__ S, out_t* table, int term, int lx, int ly, int D) {
    const int kxo_n = lx / 2 + 1, kyo_n = ly / 2 + 1;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)kxo_n * kyo_n * D;
    if (i >= total) return;
    const int d = (int)(i % D);
    const int kyo = (int)((i / D) % kyo_n);
    const int kxo = (int)(i / ((long)D * kyo_n));
    out_t* e = table + (((long)kyo * D + d) * kxo_n + kxo) * 9;
    const double2 v = S[((long)kxo * ly + kyo) * D + d];
    switch (term) {
        case 0: e[0] = (out_t)v.x; break;
        case 1: e[1] = (out_t)v.x; e[2] = (out_t)v.y; break;
        case 2: e[3] = (out_t)v.x; e[4] = (out_t)v.y; break;
        default: {
            const double2 m = S[((long)((lx - kxo) % lx) * ly + kyo) * D + d];
            e[5] = (out_t)v.x;
            e[6] = (out_t)v.y;
            e[7] = (out_t)m.x;
            e[8] = (out_t)m.y;
            break;
        }
    }
}

// ---------------------------------------------------------------- launchers

template <typename real>
hipError_t launch_strided_real(int n, bool inverse, const void* in, void* out, int n_in, int n_out, long in_es,
                               long out_es, long ncols, long in_ss, long out_ss, long nslabs, real scale,
                               const TwiddleBank& twb, hipStream_t s) {
    using C = cplx<real>;
    const C* tw = twb.get<C>(n);
    if (!tw || ncols <= 0 || nslabs <= 0) return hipErrorInvalidValue;
    switch (n) {
#define X(N_)                                                                                        \
    case N_: {                                                                                       \
        constexpr int T = strided_T<real, N_>();                                                     \
        constexpr int P = N_ / Plan<N_>::E, SPW = ce_max(1, 256 / (P * T));                          \
        dim3 grid((unsigned)((ncols + T - 1) / T), (unsigned)((nslabs + SPW - 1) / SPW));            \
        if (inverse)                                                                                 \
            hipLaunchKernelGGL((strided_real_kernel<real, N_, T, true>), grid, dim3(SPW * P * T), 0, \
                               s, in, out, n_in, n_out, in_es, out_es, ncols, in_ss, out_ss, nslabs,  \
                               scale, tw);                                                           \
        else                                                                                         \
            hipLaunchKernelGGL((strided_real_kernel<real, N_, T, false>), grid, dim3(SPW * P * T),   \
                               0, s, in, out, n_in, n_out, in_es, out_es, ncols, in_ss, out_ss,       \
                               nslabs, scale, tw);                                                   \
        return hipGetLastError();                                                                    \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

int band_tile(int lx, int real_bytes) {
    switch (lx) {
#define X(N_) \
    case N_: return real_bytes == 8 ? band_T<double, N_>() : band_T<float, N_>();
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return 0;
}

template <typename real>
hipError_t launch_xband(int lx, bool adjoint, const void* in, void* out, int nx, int ly, int nz, int nb,
                        const real* table, const TwiddleBank& twb, hipStream_t s) {
    using C = cplx<real>;
    const C* tw = twb.get<C>(lx);
    if (!tw || nb < 0 || nx > lx || nz < 1) return hipErrorInvalidValue;
    switch (lx) {
#define X(N_)                                                                                        \
    case N_: {                                                                                       \
        constexpr int T = band_T<real, N_>();                                                        \
        constexpr int P = N_ / Plan<N_>::E;                                                          \
        dim3 grid((unsigned)((nz + T - 1) / T), (unsigned)(ly / 2 + 1));                             \
        if (adjoint)                                                                                 \
            hipLaunchKernelGGL((xband_kernel<real, N_, true>), grid, dim3(2 * P * T), 0, s,          \
                               (const C*)in, (C*)out, nx, ly, nz, nb, table, tw);                    \
        else                                                                                         \
            hipLaunchKernelGGL((xband_kernel<real, N_, false>), grid, dim3(2 * P * T), 0, s,         \
                               (const C*)in, (C*)out, nx, ly, nz, nb, table, tw);                    \
        return hipGetLastError();                                                                    \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

static unsigned blocks_for(long n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_compress_band(const void* spec, void* table, int real_bytes, int term, int lx, int ly, int D,
                                hipStream_t st) {
    const long n = (long)(lx / 2 + 1) * (ly / 2 + 1) * D;
    if (D < 1) return hipErrorInvalidValue;
    if (real_bytes == 8)
        hipLaunchKernelGGL(compress_band_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           (const double2*)spec, (double*)table, term, lx, ly, D);
    else
        hipLaunchKernelGGL(compress_band_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           (const double2*)spec, (float*)table, term, lx, ly, D);
    return hipGetLastError();
}

#define PIPE_INST(real)                                                                                      \
    template hipError_t launch_strided_real<real>(int, bool, const void*, void*, int, int, long, long, long, \
                                                  long, long, long, real, const TwiddleBank&, hipStream_t);  \
    template hipError_t launch_xband<real>(int, bool, const void*, void*, int, int, int, int, const real*,   \
                                           const TwiddleBank&, hipStream_t);
PIPE_INST(float)
PIPE_INST(double)
#undef PIPE_INST

}  // namespace pipe
