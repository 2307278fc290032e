// band.hip -- neighbouring-plane z sums (Eq. 17-18).  When the z dependence of
// the Green function is negligible beyond N planes, the potential on plane k is
//   phi[., ., k] = hx hy hz sum_{d=-N..N} (2-D mixed conv/corr of rho[., ., k-d]
//                                          with the slice of G at z distance |d| hz)
// so the z transform drops out: the planes are transformed in y and x only, the
// product sums 2N + 1 plane products per output plane, and the Green spectra
// are N + 1 two-dimensional slices.
//
// The planes are real, so two of them travel as one complex plane: packed
// column p holds rho[., ., 2p] + i rho[., ., 2p+1].  Its 2-D spectrum F splits
// into the two planes' Hermitian spectra, R_even(k) = (F(k) + conj F(-k)) / 2
// and R_odd(k) = (F(k) - conj F(-k)) / 2i; the products are needed at only two
// points of each orbit (the other two are their conjugates), and the outputs
// are packed the same way before the inverse transforms.
//
//   B1 y forward of packed pairs, rho -> A (ly, nx, ceil(nz/2)) complex  [strided_pair_kernel<fwd>]
//   B2 x forward, split, banded product, pack, x inverse, A -> B         [xband0_kernel (N = 0),
//                                                                         xband1_kernel / xband_kernel]
//   B3 y inverse, unpack to the real planes, scaled                      [strided_pair_kernel<inv>]
#include "pass_common.h"

// Compiled as one unit (PIPE_TU undefined) or as two: PIPE_TU = 1 (FP32
// kernels and the precision-independent functions), PIPE_TU = 2 (FP64 kernels).
#if !defined(PIPE_TU) || PIPE_TU == 1
#define PIPE_TU_FP32 1
#endif
#if !defined(PIPE_TU) || PIPE_TU == 2
#define PIPE_TU_FP64 1
#endif

namespace pipe {

// y pass between real planes (pairs of z columns) and packed complex columns.
// Real side: element (slab, e, z) at slab * r_ss + e * r_es + z, z < nz.
// Complex side: (slab, e, p) at slab * c_ss + e * c_es + p, p < ncols = ceil(nz/2).
// Forward: real in, complex out (all ly rows, zero-padded beyond n_in).
// Inverse: complex in, real out (rows e < n_out), times scale.
template <typename real, int N, int T, bool INV>
__global__ __launch_bounds__(ce_max(1, 256 / ((N / Plan<N, strided_V<real, N>()>::E) * T)) *
                             (N / Plan<N, strided_V<real, N>()>::E) * T)
void strided_pair_kernel(const void* in, void* out, int n_in, int n_out, long r_es, long c_es, long ncols,
                         long r_ss, long c_ss, long nslabs, int nz, real scale, const twid<real>* __restrict__ tw) {
    using C = cplx<real>;
    using PL = Plan<N, strided_V<real, N>()>;
    constexpr int P = N / PL::E, SPW = ce_max(1, 256 / (P * T));
    __shared__ C lds[SPW * N * T];
    __shared__ twid<real> s_tw[N];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<PL>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, s = threadIdx.x / (T * P);
    const long slab = (long)blockIdx.y * SPW + s;
    const long col = (long)blockIdx.x * T + c;
    const bool active = slab < nslabs && col < ncols;
    const bool pair = 2 * col + 1 < nz;            // the odd plane exists
    // pairs start on a 2-real boundary: one vector access per pair
    const void* rp = INV ? (const void*)out : in;
    const bool vec = (nz % 2) == 0 && (reinterpret_cast<uintptr_t>(rp) % (2 * sizeof(real))) == 0;
    const long roff = active ? slab * r_ss + 2 * col : 0;
    const long coff = active ? slab * c_ss + col : 0;
    LdsCol<C, T> view{lds + s * N * T + c};
    fft_line<PL, INV, false>(
        t, tw,
        [&](int e) -> C {
            if (!(active && e < n_in)) return cmake<C>(0, 0);
            if constexpr (INV) {
                return reinterpret_cast<const C*>(in)[coff + e * c_es];
            } else {
                const real* r = reinterpret_cast<const real*>(in) + roff + e * r_es;
                if (vec) return *reinterpret_cast<const C*>(r);
                return cmake<C>(r[0], pair ? r[1] : (real)0);
            }
        },
        [&](int e, C v) {
            if (!(active && e < n_out)) return;
            if constexpr (INV) {
                real* r = reinterpret_cast<real*>(out) + roff + e * r_es;
                if (vec) {
                    *reinterpret_cast<C*>(r) = cmake<C>(v.x * scale, v.y * scale);
                } else {
                    r[0] = v.x * scale;
                    if (pair) r[1] = v.y * scale;
                }
            } else {
                reinterpret_cast<C*>(out)[coff + e * c_es] = v;
            }
        },
        view);
}

#ifndef PIPE_BAND_TMAX
#define PIPE_BAND_TMAX 16     // widest packed-column tile of the banded x pass
#endif

// Packed columns per block of the banded x pass: a power of two <= PIPE_BAND_TMAX
// with at most 512 threads (two ky lines x P threads x T columns), the padded
// LDS lines (2 N (T + 1) complex) within PIPE_LDS_CAP + 8 KB, and the whole
// block's LDS (lines, twiddles, one distance's coefficients) within 156 KB.
template <typename real, int N> constexpr int band_T() {
    constexpr int P = N / Plan<N>::E, cs = 2 * (int)sizeof(real);
    constexpr int fixed = N * cs + 10 * (N / 2 + 1) * (int)sizeof(real);
    int t = PIPE_BAND_TMAX;
    while (t > 1 && (2 * P * t > 512 || 2 * N * (t + 1) * cs > PIPE_LDS_CAP + 8192 ||
                     2 * N * (t + 1) * cs + fixed > 156 * 1024))
        t /= 2;
    return t;
}

__device__ __forceinline__ int floor_half(int x) { return x >= 0 ? x / 2 : -((1 - x) / 2); }

// Block (tile, ky): lines ky and -ky of the 2 to output planes z0 = 2 to tile ...
// z0 + 2 to - 1 (packed columns to tile ..., to <= T).  The packed input
// columns holding planes z0 - nb .. z0 + 2 to - 1 + nb (to + nb + (nb odd)
// of them) are transformed along x, T at a time, into
// LDS (element e of column j at e (T+1) + j: the padding keeps both the
// transforms' column-wise and the products' orbit-wise accesses free of bank
// conflicts).  Each chunk is split into the planes' spectra in place; then
// every (kx orbit, output column) item adds the products of its two output
// planes with the chunk's planes within nb of them to register accumulators.
// Lanes of a wave run over kx orbits, so the plane bookkeeping is uniform per
// wave and the table reads are coalesced.  The accumulators are finally packed
// into the LDS lines and transformed back.
//
// The product.  With R real-plane spectra (Hermitian), the four-term product
// at the orbit points (kx, ky) and (-kx, ky) of an output plane needs only
// x0 = R(kx, ky) = a + ib and x1 = R(-kx, ky) = c + id of the input plane:
//   Phi(kx, ky)  = T_cc x0 - T_cr conj x1 - T_rc x1 + T_rr conj x0,
//   Phi(-kx, ky) = T_cc x1 - T_cr conj x0 - conj(T_rc) x0 + T_rr(-kx, ky) conj x1,
// (the other two points are the conjugates), a real-linear map of (a, b, c, d)
// whose 4 x 4 matrix is symmetric with ten distinct entries K0..K9
// (band_coefficients).  The adjoint therefore applies the same matrices.
//
// Banded table: K_k of (ky orbit kyo, plane distance d, kx orbit kxo) at
// ((kyo (nb + 1) + d) 10 + k) (N/2 + 1) + kxo.  The split leaves a factor 2
// on the spectra, which the inverse y pass removes with its scale.
template <typename real, int N>
__global__ __launch_bounds__((2 * (N / Plan<N>::E) * band_T<real, N>()))
void xband_kernel(const cplx<real>* __restrict__ in, cplx<real>* __restrict__ out, int nx, int ly, int nz, long pitch,
                  int nb, int to, const real* __restrict__ table, const twid<real>* __restrict__ tw) {
    using C = cplx<real>;
    constexpr int T = band_T<real, N>(), TS = T + 1;
    constexpr int P = N / Plan<N>::E, NT = 2 * P * T, NH = N / 2, NKX = NH + 1;
    // items (orbit o < N/2, output column c2): exactly IM per thread; the
    // orbit o = N/2 of output column c2 goes to thread c2 as one more item
    constexpr int IM = NH * T / NT;
    static_assert(IM * NT == NH * T, "the E/4 items per thread must tile the orbits");
    constexpr int KPT = (10 * NKX + NT - 1) / NT;   // coefficients each thread stages per distance
    __shared__ C lds[2 * N * TS];
    __shared__ twid<real> s_tw[N];
    __shared__ real sK[10 * NKX];   // K0..K9 of one plane distance, this block's ky
    tw = stage_twiddles(s_tw, tw, stage_tw_size<Plan<N>>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, l = threadIdx.x / (T * P);
    const unsigned ntile = gridDim.x;
    const unsigned lid = xcd_remap(blockIdx.x + ntile * blockIdx.y, ntile * gridDim.y);
    const int tile = (int)(lid % ntile);
    const int ky = (int)(lid / ntile);
    const int kyl = l == 0 ? ky : (ly - ky) % ly;
    const bool self = (ky == 0) || (2 * ky == ly);
    const int nzp = (nz + 1) / 2;
    const int z0 = 2 * to * tile;   // to <= T output columns per block
    const long xs = pitch;   // row (x) stride of the packed arrays
    const real* trow = table + (long)ky * (nb + 1) * 10 * NKX;
    for (int idx = threadIdx.x; idx < 10 * NKX; idx += NT) sK[idx] = trow[idx];   // distance 0 (barriers follow)
    LdsCol<C, TS> view{lds + l * N * TS + c};
    const bool extra = threadIdx.x < T;   // owns item (N/2, c2 = threadIdx.x)
    auto item = [&](int i, int& o, int& c2) {
        if (i < IM) {
            const int w = threadIdx.x + i * NT;
            o = w % NH;
            c2 = w / NH;
        } else {
            o = NH;
            c2 = threadIdx.x;
        }
    };

    C acc[IM + 1][4];   // per item: Phi_even at (kx,ky), (-kx,ky); Phi_odd at the same
#pragma unroll
    for (int i = 0; i <= IM; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = cmake<C>(0, 0);

    // packed input columns pbase .. pbase + ncolp - 1 hold planes z0 - nb .. z0 + 2 to - 1 + nb
    const int pbase = floor_half(z0 - nb);
    const int ncolp = floor_half(z0 + 2 * to - 1 + nb) - pbase + 1;
    const int nchunk = (ncolp + T - 1) / T;
    for (int ch = 0; ch < nchunk; ++ch) {
        if (ch > 0) __syncthreads();   // previous chunk's products have read the LDS
        const int pc = pbase + ch * T + c;
        const bool act = ch * T + c < ncolp && pc >= 0 && pc < nzp;
        const C* line = in + (act ? (long)kyl * nx * pitch + pc : 0);
        fft_line<Plan<N>, false, false>(
            t, tw, [&](int e) -> C { return (act && e < nx) ? line[e * xs] : cmake<C>(0, 0); },
            [&](int e, C v) { view.set(e, v); }, view);
        __syncthreads();
        // split every packed column into 2 R_even (line 0) and 2 R_odd (line 1)
        // at slots o, -o: F(k) +- conj F(-k), times -i for the odd plane; the
        // item of orbit o owns all four slots
#pragma unroll
        for (int i = 0; i <= IM; ++i) {
            if (i == IM && !extra) break;
            int o, j;
            item(i, o, j);
            const int on = (N - o) % N;
            const C f0 = lds[o * TS + j], f1 = lds[on * TS + j];
            const C g0 = lds[(N + o) * TS + j], g1 = lds[(N + on) * TS + j];
            const C u0 = csub(f0, cconj(g1)), u1 = csub(f1, cconj(g0));
            lds[o * TS + j] = cadd(f0, cconj(g1));
            lds[(N + o) * TS + j] = cmake<C>(u0.y, -u0.x);
            if (on != o) {
                lds[on * TS + j] = cadd(f1, cconj(g0));
                lds[(N + on) * TS + j] = cmake<C>(u1.y, -u1.x);
            }
        }
        __syncthreads();
        // products: output plane ze + h (ze = z0 + 2 c2) with input plane
        // z = ze + h - d, |d| <= nb, when z lies in this chunk and in the mesh.
        // The coefficients of distance ad sit in sK; those of ad + 1 are
        // fetched into registers meanwhile and stored after the products.
        const int p0 = pbase + ch * T;
        const int jlim = min(T, ncolp - ch * T);
        for (int ad = 0; ad <= nb; ++ad) {
            real pre[KPT];
            if (ad < nb) {
                const real* src = trow + (long)(ad + 1) * 10 * NKX;
#pragma unroll
                for (int u = 0; u < KPT; ++u) {
                    const int idx = threadIdx.x + u * NT;
                    if (idx < 10 * NKX) pre[u] = src[idx];
                }
            }
#pragma unroll
            for (int i = 0; i <= IM; ++i) {
                if (i == IM && !extra) break;
                int o, c2;
                item(i, o, c2);
                if (c2 >= to) continue;
                const int on = (N - o) % N;
                const int ze = z0 + 2 * c2;
                // the (up to) four pairs at this distance: d = +-ad, h = 0, 1
                int zk[4];
                bool any = false;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int z = ze + (k & 1) - ((k & 2) ? -ad : ad);
                    const int j = (z >> 1) - p0;
                    const bool ok = !((k & 2) && ad == 0) && z >= 0 && z < nz && j >= 0 && j < jlim;
                    zk[k] = ok ? z : -1;
                    any |= ok;
                }
                if (!any) continue;
                real q[10];
#pragma unroll
                for (int m = 0; m < 10; ++m) q[m] = sK[m * NKX + o];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int z = zk[k];
                    if (z < 0) continue;
                    const int j = (z >> 1) - p0, sN = (z & 1) * N;
                    const C x0 = lds[(sN + o) * TS + j], x1 = lds[(sN + on) * TS + j];
                    C& y0 = acc[i][2 * (k & 1)];
                    C& y1 = acc[i][2 * (k & 1) + 1];
                    y0.x += q[0] * x0.x + q[1] * x0.y + q[3] * x1.x + q[4] * x1.y;
                    y0.y += q[1] * x0.x + q[2] * x0.y + q[5] * x1.x + q[6] * x1.y;
                    y1.x += q[3] * x0.x + q[5] * x0.y + q[7] * x1.x + q[8] * x1.y;
                    y1.y += q[4] * x0.x + q[6] * x0.y + q[8] * x1.x + q[9] * x1.y;
                }
            }
            __syncthreads();   // every product of distance ad has read sK
            if (ad < nb) {
#pragma unroll
                for (int u = 0; u < KPT; ++u) {
                    const int idx = threadIdx.x + u * NT;
                    if (idx < 10 * NKX) sK[idx] = pre[u];
                }
            } else if (ch + 1 < nchunk && nb > 0) {
                // next chunk starts again at distance 0
                const real* src = trow;
                for (int idx = threadIdx.x; idx < 10 * NKX; idx += NT) sK[idx] = src[idx];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // G = Phi_even + i Phi_odd; Phi Hermitian: Phi(kx,-ky) = conj Phi(-kx,ky), Phi(-kx,-ky) = conj Phi(kx,ky)
    auto pack = [](C e, C d) { return cmake<C>(e.x - d.y, e.y + d.x); };   // e + i d
#pragma unroll
    for (int i = 0; i <= IM; ++i) {
        if (i == IM && !extra) break;
        int o, c2;
        item(i, o, c2);
        const int on = (N - o) % N;
        const C e0 = acc[i][0], e1 = acc[i][1], d0 = acc[i][2], d1 = acc[i][3];
        lds[o * TS + c2] = pack(e0, d0);
        lds[(N + o) * TS + c2] = pack(cconj(e1), cconj(d1));
        if (on != o) {   // o = 0 and o = N/2 are their own mirror
            lds[on * TS + c2] = pack(e1, d1);
            lds[(N + on) * TS + c2] = pack(cconj(e0), cconj(d0));
        }
    }
    __syncthreads();

    // inverse x transforms of the output columns c < to, rows i < nx
    const int pco = to * tile + c;
    const bool oact = c < to && pco < nzp && !(l == 1 && self);
    C* oline = out + (oact ? (long)kyl * nx * pitch + pco : 0);
    fft_line<Plan<N>, true, true>(
        t, tw, [&](int e) -> C { return view.get(e); },
        [&](int e, C v) {
            if (oact && e < nx) oline[e * xs] = v;
        },
        view);
}

// N = 0 (Eq. 17: independent planes).  Each output column depends on its
// own input column only, so the split, the product and the packing happen in
// place, one orbit at a time, between the two transforms, with no halo, no
// accumulators and the 3-D fused pass's block shape: T packed columns of the
// two lines ky, -ky.  Coefficients as xband_kernel (distance 0).
template <typename real, int N> constexpr int band0_T() {
    constexpr int P = N / Plan<N>::E;
    int t = PIPE_XPROD_TMAX;
    while (t > 1 && (2 * N * t * 2 * (int)sizeof(real) > PIPE_LDS_CAP || 2 * P * t > 1024)) t /= 2;
    return t;
}

// T: the widest tile (band0_T) or half of it; the plan picks by timing.  The
// ten coefficients of each of a thread's orbits are loaded with the rows,
// before the forward transform (they depend on ky and kx only); the Nyquist
// orbit kx = N/2, whose T items go to the first T threads, is staged in LDS.
// Waves per SIMD the register allocation must allow (1: no constraint): as the
// 3-D fused pass, the FP32 length-512 kernel fits one 1024-thread block per CU
// at its natural 72 registers although the LDS holds two; at 64 (no spills at
// T = 8) two fit (256x256x1024, N = 0: 472 -> 438 us).
template <typename real, int N> constexpr int xband0_waves() { return (sizeof(real) == 4 && N == 512) ? 8 : 1; }
template <typename real, int N, int T>
__global__ __launch_bounds__((2 * (N / Plan<N>::E) * T)) __attribute__((amdgpu_waves_per_eu(xband0_waves<real, N>())))
void xband0_kernel(const cplx<real>* __restrict__ in, cplx<real>* __restrict__ out, int nx, int ly, int nz,
                   long pitch, const real* __restrict__ table, const twid<real>* __restrict__ tw) {
    using C = cplx<real>;
    constexpr int P = N / Plan<N>::E, NT = 2 * P * T, NKX = N / 2 + 1, NO = N / 2;
    constexpr int IT = (NO * T + NT - 1) / NT, KN = (10 + NT - 1) / NT;
    static_assert(N % 2 == 0, "banded lengths are even");
    __shared__ C lds[2 * N * T];
    __shared__ twid<real> s_tw[N];
    __shared__ real s_kn[10];   // the Nyquist orbit's coefficients
    tw = stage_twiddles(s_tw, tw, stage_tw_size<Plan<N>>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, l = threadIdx.x / (T * P);
    const unsigned ntile = gridDim.x;
    const unsigned lid = xcd_remap(blockIdx.x + ntile * blockIdx.y, ntile * gridDim.y);
    const int tile = (int)(lid % ntile);
    const int ky = (int)(lid / ntile);
    const int kyl = l == 0 ? ky : (ly - ky) % ly;
    const bool self = (ky == 0) || (2 * ky == ly);
    const int nzp = (nz + 1) / 2;
    const int pc = tile * T + c;
    const bool active = pc < nzp;
    const long xs = pitch;   // row (x) stride of the packed arrays
    const C* iline = in + (active ? (long)kyl * nx * pitch + pc : 0);
    C* oline = out + (active ? (long)kyl * nx * pitch + pc : 0);
    LdsCol<C, T> view{lds + l * N * T + c};

    const real* trow = table + (long)ky * 10 * NKX;
    real qs[IT][10];
    real kn[KN];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int w = threadIdx.x + it * NT;
        if (w < NO * T) {
#pragma unroll
            for (int m = 0; m < 10; ++m) qs[it][m] = trow[m * NKX + w / T];
        }
    }
#pragma unroll
    for (int k = 0; k < KN; ++k) {
        const int m = threadIdx.x + k * NT;
        if (m < 10) kn[k] = trow[m * NKX + NO];
    }

    fft_line<Plan<N>, false, false>(
        t, tw, [&](int e) -> C { return (active && e < nx) ? iline[e * xs] : cmake<C>(0, 0); },
        [&](int e, C v) { view.set(e, v); }, view);
#pragma unroll
    for (int k = 0; k < KN; ++k) {
        const int m = threadIdx.x + k * NT;
        if (m < 10) s_kn[m] = kn[k];
    }
    __syncthreads();

    auto orbit_item = [&](int o, int j, const real* q) {
        const int on = (N - o) % N;
        const C f0 = lds[o * T + j], f1 = lds[on * T + j];
        const C g0 = lds[(N + o) * T + j], g1 = lds[(N + on) * T + j];
        // 2 R of the even and the odd plane at (kx,ky), (-kx,ky)
        const C u0 = csub(f0, cconj(g1)), u1 = csub(f1, cconj(g0));
        const C xe0 = cadd(f0, cconj(g1)), xe1 = cadd(f1, cconj(g0));
        const C xo0 = cmake<C>(u0.y, -u0.x), xo1 = cmake<C>(u1.y, -u1.x);
        auto apply = [&](C x0, C x1, C& y0, C& y1) {
            y0 = cmake<C>(q[0] * x0.x + q[1] * x0.y + q[3] * x1.x + q[4] * x1.y,
                          q[1] * x0.x + q[2] * x0.y + q[5] * x1.x + q[6] * x1.y);
            y1 = cmake<C>(q[3] * x0.x + q[5] * x0.y + q[7] * x1.x + q[8] * x1.y,
                          q[4] * x0.x + q[6] * x0.y + q[8] * x1.x + q[9] * x1.y);
        };
        C e0, e1, d0, d1;
        apply(xe0, xe1, e0, e1);
        apply(xo0, xo1, d0, d1);
        // G = Phi_even + i Phi_odd at the four points (Phi Hermitian)
        auto pack = [](C e, C d) { return cmake<C>(e.x - d.y, e.y + d.x); };
        lds[o * T + j] = pack(e0, d0);
        lds[(N + o) * T + j] = pack(cconj(e1), cconj(d1));
        if (on != o) {
            lds[on * T + j] = pack(e1, d1);
            lds[(N + on) * T + j] = pack(cconj(e0), cconj(d0));
        }
    };
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int w = threadIdx.x + it * NT;
        if (w < NO * T) orbit_item(w / T, w % T, qs[it]);
    }
    if (threadIdx.x < T) {
        real q[10];
#pragma unroll
        for (int m = 0; m < 10; ++m) q[m] = s_kn[m];
        orbit_item(NO, threadIdx.x, q);
    }
    __syncthreads();

    fft_line<Plan<N>, true, true>(
        t, tw, [&](int e) -> C { return view.get(e); },
        [&](int e, C v) {
            if (active && e < nx && !(l == 1 && self)) oline[e * xs] = v;
        },
        view);
}

// Small N: the whole input window of a block -- `to` output columns plus the
// halo, to + N + (N odd) <= T packed columns -- is one transform chunk, so all
// transforms finish before the products start and the accumulators are never
// live together with a transform's registers.  Same block shape as the N = 0
// pass (T packed columns of the lines ky, -ky, padded LDS columns so the
// orbit-wise product reads are conflict-free); the coefficients of each plane
// distance are read from global memory, coalesced over orbits.
// As xband0: the FP32 length-512 kernel fits one 1024-thread block per CU at
// its natural 76 registers; held to 64 (9 spilled) two fit (256x256x1024,
// N = 1: 1096 -> 918 us).
template <typename real, int N> constexpr int xband1_waves() { return (sizeof(real) == 4 && N == 512) ? 8 : 1; }
template <typename real, int N>
__global__ __launch_bounds__((2 * (N / Plan<N>::E) * band0_T<real, N>()))
__attribute__((amdgpu_waves_per_eu(xband1_waves<real, N>())))
void xband1_kernel(const cplx<real>* __restrict__ in, cplx<real>* __restrict__ out, int nx, int ly, int nz,
                   long pitch, int nb, int to, const real* __restrict__ table, const twid<real>* __restrict__ tw) {
    using C = cplx<real>;
    constexpr int T = band0_T<real, N>(), TS = T + 1;
    constexpr int P = N / Plan<N>::E, NT = 2 * P * T, NH = N / 2, NKX = NH + 1;
    constexpr int IM = (NH * T + NT - 1) / NT;   // (orbit < N/2, output column) items per thread, at most
    __shared__ C lds[2 * N * TS];
    __shared__ twid<real> s_tw[N];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<Plan<N>>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, l = threadIdx.x / (T * P);
    const unsigned ntile = gridDim.x;
    const unsigned lid = xcd_remap(blockIdx.x + ntile * blockIdx.y, ntile * gridDim.y);
    const int tile = (int)(lid % ntile);
    const int ky = (int)(lid / ntile);
    const int kyl = l == 0 ? ky : (ly - ky) % ly;
    const bool self = (ky == 0) || (2 * ky == ly);
    const int nzp = (nz + 1) / 2;
    const int z0 = 2 * to * tile;
    const long xs = pitch;   // row (x) stride of the packed arrays
    const real* trow = table + (long)ky * (nb + 1) * 10 * NKX;
    LdsCol<C, TS> view{lds + l * N * TS + c};

    // the window: packed columns pbase .. pbase + ncolp - 1 (ncolp <= T)
    const int pbase = floor_half(z0 - nb);
    const int ncolp = floor_half(z0 + 2 * to - 1 + nb) - pbase + 1;
    {
        const int pc = pbase + c;
        const bool act = c < ncolp && pc >= 0 && pc < nzp;
        const C* line = in + (act ? (long)kyl * nx * pitch + pc : 0);
        fft_line<Plan<N>, false, false>(
            t, tw, [&](int e) -> C { return (act && e < nx) ? line[e * xs] : cmake<C>(0, 0); },
            [&](int e, C v) { view.set(e, v); }, view);
    }
    __syncthreads();
    // split every column into 2 R_even (line 0) and 2 R_odd (line 1) at slots o, -o
    for (int w = threadIdx.x; w < NKX * T; w += NT) {
        const int o = w % NKX, j = w / NKX, on = (N - o) % N;
        const C f0 = lds[o * TS + j], f1 = lds[on * TS + j];
        const C g0 = lds[(N + o) * TS + j], g1 = lds[(N + on) * TS + j];
        const C u0 = csub(f0, cconj(g1)), u1 = csub(f1, cconj(g0));
        lds[o * TS + j] = cadd(f0, cconj(g1));
        lds[(N + o) * TS + j] = cmake<C>(u0.y, -u0.x);
        if (on != o) {
            lds[on * TS + j] = cadd(f1, cconj(g0));
            lds[(N + on) * TS + j] = cmake<C>(u1.y, -u1.x);
        }
    }
    __syncthreads();

    // products: item (o, c2 < to), lanes over o; the orbit o = N/2 of column c2 is thread c2's extra item
    auto item = [&](int i, int& o, int& c2) {
        if (i < IM) {
            const int w = threadIdx.x + i * NT;
            o = w % NH;
            c2 = w / NH;
        } else {
            o = NH;
            c2 = threadIdx.x;
        }
    };
    C acc[IM + 1][4];
#pragma unroll
    for (int i = 0; i <= IM; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = cmake<C>(0, 0);
    for (int ad = 0; ad <= nb; ++ad) {
        const real* kp = trow + (long)ad * 10 * NKX;
#pragma unroll
        for (int i = 0; i <= IM; ++i) {
            int o, c2;
            item(i, o, c2);
            if (c2 >= to) continue;
            const int on = (N - o) % N;
            const int ze = z0 + 2 * c2;
            real q[10];
#pragma unroll
            for (int m = 0; m < 10; ++m) q[m] = kp[m * NKX + o];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((k & 2) && ad == 0) continue;
                const int z = ze + (k & 1) - ((k & 2) ? -ad : ad);
                if (z < 0 || z >= nz) continue;
                const int j = (z >> 1) - pbase, sN = (z & 1) * N;
                const C x0 = lds[(sN + o) * TS + j], x1 = lds[(sN + on) * TS + j];
                C& y0 = acc[i][2 * (k & 1)];
                C& y1 = acc[i][2 * (k & 1) + 1];
                y0.x += q[0] * x0.x + q[1] * x0.y + q[3] * x1.x + q[4] * x1.y;
                y0.y += q[1] * x0.x + q[2] * x0.y + q[5] * x1.x + q[6] * x1.y;
                y1.x += q[3] * x0.x + q[5] * x0.y + q[7] * x1.x + q[8] * x1.y;
                y1.y += q[4] * x0.x + q[6] * x0.y + q[8] * x1.x + q[9] * x1.y;
            }
        }
    }
    __syncthreads();   // every product has read the window
    auto pack = [](C e, C d) { return cmake<C>(e.x - d.y, e.y + d.x); };   // e + i d
#pragma unroll
    for (int i = 0; i <= IM; ++i) {
        int o, c2;
        item(i, o, c2);
        if (c2 >= to) continue;
        const int on = (N - o) % N;
        const C e0 = acc[i][0], e1 = acc[i][1], d0 = acc[i][2], d1 = acc[i][3];
        lds[o * TS + c2] = pack(e0, d0);
        lds[(N + o) * TS + c2] = pack(cconj(e1), cconj(d1));
        if (on != o) {
            lds[on * TS + c2] = pack(e1, d1);
            lds[(N + on) * TS + c2] = pack(cconj(e0), cconj(d0));
        }
    }
    __syncthreads();

    const int pco = to * tile + c;
    const bool oact = c < to && pco < nzp && !(l == 1 && self);
    C* oline = out + (oact ? (long)kyl * nx * pitch + pco : 0);
    fft_line<Plan<N>, true, true>(
        t, tw, [&](int e) -> C { return view.get(e); },
        [&](int e, C v) {
            if (oact && e < nx) oline[e * xs] = v;
        },
        view);
}

// y pass with real input (forward: rho -> complex) or real output (inverse:
// complex -> scaled real part), one plane per column (the Green arrangements).
template <typename real, int N, int T, bool INV>
__global__ __launch_bounds__(ce_max(1, 256 / ((N / Plan<N, strided_V<real, N>()>::E) * T)) *
                             (N / Plan<N, strided_V<real, N>()>::E) * T)
void strided_real_kernel(const void* in, void* out, int n_in, int n_out, long in_es, long out_es, long ncols,
                         long in_ss, long out_ss, long nslabs, real scale, const twid<real>* __restrict__ tw) {
    using C = cplx<real>;
    using PL = Plan<N, strided_V<real, N>()>;
    constexpr int P = N / PL::E, SPW = ce_max(1, 256 / (P * T));
    __shared__ C lds[SPW * N * T];
    __shared__ twid<real> s_tw[N];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<PL>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, s = threadIdx.x / (T * P);
    const long slab = (long)blockIdx.y * SPW + s;
    const long col = (long)blockIdx.x * T + c;
    const bool active = slab < nslabs && col < ncols;
    const long ioff = active ? slab * in_ss + col : 0;
    const long ooff = active ? slab * out_ss + col : 0;
    LdsCol<C, T> view{lds + s * N * T + c};
    fft_line<PL, INV, false>(
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

#if PIPE_TU_FP32
// The four terms' 2-D spectra of one plane distance, 9 values per orbit in
// the 3-D orbit table's order (0 T_cc, 1-2 T_cr, 3-4 T_rc, 5-6 T_rr(kx,ky),
// 7-8 T_rr(-kx,ky)), FP64, planar: value p of (kyo, d, kxo) at
// ((kyo D + d) 9 + p) (lx/2 + 1) + kxo.  S[lx][ly][D] is one term's spectrum;
// term: 0 cc, 1 cr, 2 rc, 3 rr.
__global__ void compress_band_kernel(const double2* __restrict__ S, double* tmp, int term, int lx, int ly, int D) {
    const int kxo_n = lx / 2 + 1, kyo_n = ly / 2 + 1;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)kxo_n * kyo_n * D;
    if (i >= total) return;
    const int d = (int)(i % D);
    const int kyo = (int)((i / D) % kyo_n);
    const int kxo = (int)(i / ((long)D * kyo_n));
    double* e = tmp + ((long)kyo * D + d) * 9 * kxo_n + kxo;   // value p at e[p kxo_n]
    const double2 v = S[((long)kxo * ly + kyo) * D + d];
    switch (term) {
        case 0: e[0] = v.x; break;
        case 1: e[1 * kxo_n] = v.x; e[2 * kxo_n] = v.y; break;
        case 2: e[3 * kxo_n] = v.x; e[4 * kxo_n] = v.y; break;
        default: {
            const double2 m = S[((long)((lx - kxo) % lx) * ly + kyo) * D + d];
            e[5 * kxo_n] = v.x;
            e[6 * kxo_n] = v.y;
            e[7 * kxo_n] = m.x;
            e[8 * kxo_n] = m.y;
            break;
        }
    }
}
#endif

// K0..K9 of xband_kernel from the nine values (cc; cr = p + iq; rc = u + iv;
// rr = m + in; rr(-kx) = m2 + i n2), computed in FP64 and rounded once:
//   K0 = cc + m   K1 = n        K2 = cc - m   K3 = -p - u   K4 = -q + v
//   K5 = -q - v   K6 = p - u    K7 = cc + m2  K8 = n2       K9 = cc - m2
template <typename out_t>
__global__ void band_coefficients_kernel(const double* __restrict__ tmp, out_t* table, long n_entries, int kxo_n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_entries * kxo_n) return;
    const long row = i / kxo_n, kxo = i % kxo_n;
    const double* e = tmp + row * 9 * kxo_n + kxo;
    const double cc = e[0], p = e[kxo_n], q = e[2 * kxo_n], u = e[3 * kxo_n], v = e[4 * kxo_n];
    const double m = e[5 * kxo_n], n = e[6 * kxo_n], m2 = e[7 * kxo_n], n2 = e[8 * kxo_n];
    const double K[10] = {cc + m, n, cc - m, -p - u, -q + v, -q - v, p - u, cc + m2, n2, cc - m2};
    out_t* o = table + row * 10 * kxo_n + kxo;
    for (int k = 0; k < 10; ++k) o[k * kxo_n] = (out_t)K[k];
}

// ---------------------------------------------------------------- launchers

template <typename real>
hipError_t launch_strided_pair(int n, bool inverse, const void* in, void* out, int n_in, int n_out, long r_es,
                               long c_es, long r_ss, long c_ss, long nslabs, int nz, real scale,
                               const TwiddleBank& twb, hipStream_t s) {
    using C = cplx<real>;
    const long ncols = (nz + 1) / 2;
    if (nz < 1 || nslabs <= 0) return hipErrorInvalidValue;
    switch (n) {
#define X(N_)                                                                                        \
    case N_: {                                                                                       \
        constexpr int T = strided_T<real, N_>(), V = strided_V<real, N_>();                          \
        constexpr int P = N_ / Plan<N_, V>::E, SPW = ce_max(1, 256 / (P * T));                       \
        const twid<real>* tw = twb.stage<twid<real>>(N_, V);                                                           \
        if (!tw) return hipErrorInvalidValue;                                                        \
        dim3 grid((unsigned)((ncols + T - 1) / T), (unsigned)((nslabs + SPW - 1) / SPW));            \
        if (inverse)                                                                                 \
            hipLaunchKernelGGL((strided_pair_kernel<real, N_, T, true>), grid, dim3(SPW * P * T), 0, \
                               s, in, out, n_in, n_out, r_es, c_es, ncols, r_ss, c_ss, nslabs, nz,    \
                               scale, tw);                                                           \
        else                                                                                         \
            hipLaunchKernelGGL((strided_pair_kernel<real, N_, T, false>), grid, dim3(SPW * P * T),   \
                               0, s, in, out, n_in, n_out, r_es, c_es, ncols, r_ss, c_ss, nslabs, nz, \
                               scale, tw);                                                           \
        return hipGetLastError();                                                                    \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename real>
hipError_t launch_strided_real(int n, bool inverse, const void* in, void* out, int n_in, int n_out, long in_es,
                               long out_es, long ncols, long in_ss, long out_ss, long nslabs, real scale,
                               const TwiddleBank& twb, hipStream_t s) {
    using C = cplx<real>;
    if (ncols <= 0 || nslabs <= 0) return hipErrorInvalidValue;
    switch (n) {
#define X(N_)                                                                                        \
    case N_: {                                                                                       \
        constexpr int T = strided_T<real, N_>(), V = strided_V<real, N_>();                          \
        constexpr int P = N_ / Plan<N_, V>::E, SPW = ce_max(1, 256 / (P * T));                       \
        const twid<real>* tw = twb.stage<twid<real>>(N_, V);                                                           \
        if (!tw) return hipErrorInvalidValue;                                                        \
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

#if PIPE_TU_FP32
int band_tile(int lx, int real_bytes) {
    switch (lx) {
#define X(N_) \
    case N_: return real_bytes == 8 ? band_T<double, N_>() : band_T<float, N_>();
        PIPE_FOR_EACH_BAND_N(X)
#undef X
    }
    return 0;
}

#endif
// Output columns per block of xband_kernel: as many as leave the input window
// (to + nb + (nb odd) packed columns) inside one chunk of T, while that keeps
// at least half the tile; otherwise T, with the window taken in several chunks.
static int band_out_columns(int T, int nb) {
    const int to = T - nb - (nb & 1);
    return 2 * to >= T ? to : T;
}

// Output columns of xband1_kernel (window of to + nb + (nb odd) <= T columns)
// when that leaves at least a quarter of the tile, else 0 (xband_kernel only).
static int band_small_columns(int T, int nb) {
    const int to = T - nb - (nb & 1);
    return 4 * to >= T && to >= 1 ? to : 0;
}

#if PIPE_TU_FP32
int band0_tile(int lx, int real_bytes) {
    switch (lx) {
#define X(N_) \
    case N_: return real_bytes == 8 ? band0_T<double, N_>() : band0_T<float, N_>();
        PIPE_FOR_EACH_BAND_N(X)
#undef X
    }
    return 0;
}

int band_small_columns_for(int lx, int real_bytes, int nb) {
    switch (lx) {
#define X(N_) \
    case N_: return band_small_columns(real_bytes == 8 ? band0_T<double, N_>() : band0_T<float, N_>(), nb);
        PIPE_FOR_EACH_BAND_N(X)
#undef X
    }
    return 0;
}
#endif

template <typename real>
hipError_t launch_xband(int lx, const void* in, void* out, int nx, int ly, int nz, long pitch, int nb,
                        const real* table, const TwiddleBank& twb, hipStream_t s, bool single_window, int tile0) {
    using C = cplx<real>;
    const twid<real>* tw = twb.stage<twid<real>>(lx);
    const int nzp = (nz + 1) / 2;
    if (!tw || nb < 0 || nx > lx || nz < 1 || pitch < nzp) return hipErrorInvalidValue;
    switch (lx) {
#define X(N_)                                                                                        \
    case N_: {                                                                                       \
        constexpr int P = N_ / Plan<N_>::E;                                                          \
        if (nb == 0) {                                                                               \
            constexpr int T = band0_T<real, N_>(), T2 = T > 1 ? T / 2 : 1;                           \
            if (tile0 == T2 && T > 1) {                                                              \
                dim3 grid((unsigned)((nzp + T2 - 1) / T2), (unsigned)(ly / 2 + 1));                  \
                hipLaunchKernelGGL((xband0_kernel<real, N_, T2>), grid, dim3(2 * P * T2), 0, s,      \
                                   (const C*)in, (C*)out, nx, ly, nz, pitch, table, tw);                    \
            } else {                                                                                 \
                dim3 grid((unsigned)((nzp + T - 1) / T), (unsigned)(ly / 2 + 1));                    \
                hipLaunchKernelGGL((xband0_kernel<real, N_, T>), grid, dim3(2 * P * T), 0, s,        \
                                   (const C*)in, (C*)out, nx, ly, nz, pitch, table, tw);                    \
            }                                                                                        \
        } else if (single_window && band_small_columns(band0_T<real, N_>(), nb) > 0) {               \
            constexpr int T = band0_T<real, N_>();                                                   \
            const int to = band_small_columns(T, nb);                                                \
            dim3 grid((unsigned)((nzp + to - 1) / to), (unsigned)(ly / 2 + 1));                      \
            hipLaunchKernelGGL((xband1_kernel<real, N_>), grid, dim3(2 * P * T), 0, s,               \
                               (const C*)in, (C*)out, nx, ly, nz, pitch, nb, to, table, tw);                \
        } else {                                                                                     \
            constexpr int T = band_T<real, N_>();                                                    \
            const int to = band_out_columns(T, nb);                                                  \
            dim3 grid((unsigned)((nzp + to - 1) / to), (unsigned)(ly / 2 + 1));                      \
            hipLaunchKernelGGL((xband_kernel<real, N_>), grid, dim3(2 * P * T), 0, s,                \
                               (const C*)in, (C*)out, nx, ly, nz, pitch, nb, to, table, tw);                \
        }                                                                                            \
        return hipGetLastError();                                                                    \
    }
        PIPE_FOR_EACH_BAND_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

#if PIPE_TU_FP32
static unsigned blocks_for(long n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_compress_band(const void* spec, double* tmp, int term, int lx, int ly, int D, hipStream_t st) {
    const long n = (long)(lx / 2 + 1) * (ly / 2 + 1) * D;
    if (D < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(compress_band_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const double2*)spec, tmp,
                       term, lx, ly, D);
    return hipGetLastError();
}

hipError_t launch_band_coefficients(const double* tmp, void* table, int real_bytes, int lx, int ly, int D,
                                    hipStream_t st) {
    const int kxo_n = lx / 2 + 1;
    const long rows = (long)(ly / 2 + 1) * D;
    const long n = rows * kxo_n;
    if (D < 1) return hipErrorInvalidValue;
    if (real_bytes == 8)
        hipLaunchKernelGGL(band_coefficients_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, tmp,
                           (double*)table, rows, kxo_n);
    else
        hipLaunchKernelGGL(band_coefficients_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, tmp,
                           (float*)table, rows, kxo_n);
    return hipGetLastError();
}
#endif

#define PIPE_INST(real)                                                                                      \
    template hipError_t launch_strided_pair<real>(int, bool, const void*, void*, int, int, long, long, long, \
                                                  long, long, int, real, const TwiddleBank&, hipStream_t);   \
    template hipError_t launch_strided_real<real>(int, bool, const void*, void*, int, int, long, long, long, \
                                                  long, long, long, real, const TwiddleBank&, hipStream_t);  \
    template hipError_t launch_xband<real>(int, const void*, void*, int, int, int, long, int, const real*,   \
                                           const TwiddleBank&, hipStream_t, bool, int);

#if PIPE_TU_FP32
PIPE_INST(float)
#endif
#if PIPE_TU_FP64
PIPE_INST(double)
#endif
#undef PIPE_INST

}  // namespace pipe
