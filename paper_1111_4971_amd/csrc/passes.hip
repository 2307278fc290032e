// passes.hip -- the five transform passes of one open-pipe solve, and their launchers.
//
// Data layout: C-order, z fastest.  A solve is
//   P1 z-forward  real (nx, ny, nz) -> half spectrum (nx, ny, lz/2)       [z_r2c]
//   P2 y-forward  (nx, ny, lz/2)    -> (ly, nx, lz/2), input rows j < ny  [strided]
//   P3 x-forward, mixed product, x-inverse, in place on (ly, nx, lz/2)    [xprod]
//   P4 y-inverse  (ly, nx, lz/2)    -> (nx, ny, lz/2), rows j < ny kept   [strided]
//   P5 z-inverse  (nx, ny, lz/2)    -> real (nx, ny, nz), scaled           [z_c2r]
// The y passes write and read the y-transformed array ky-major, so the rows a
// block of P3 gathers (all x at one ky, a few kz) lie lz/2 values apart inside
// one nx lz/2 run rather than ly lz/2 apart across the whole array; HBM serves
// those short row segments much faster from nearby addresses.
// The half spectrum stores kz = 0 .. lz/2 - 1 with the real kz = lz/2 value
// packed into the imaginary part of the kz = 0 slot (both are real for real
// input), so every z line holds exactly lz/2 complex values.
//
// The four terms of Eq. 10 (convolution or correlation in x and in y) are one
// product: a correlation along a dimension, taken as F^f{F^f(rho) F^b(xi)},
// equals the plain inverse transform of rho_hat(-k) xi_hat(k) (Appendix, A.9:
// swapping both transform directions reflects the spectral index), so
//   Phi(kx,ky) = T_cc rho(kx,ky) - T_cr rho(kx,-ky) - T_rc rho(-kx,ky) + T_rr rho(-kx,-ky)
// with every T_ab the forward transform of its own Green array.  z is always a
// convolution, so no reflection ever leaves the stored half spectrum.
#include "pass_common.h"

namespace pipe {

// One source, compiled as one unit (PIPE_TU undefined) or as two: PIPE_TU = 1
// (the FP32 kernels and the precision-independent functions) and PIPE_TU = 2
// (the FP64 kernels), which halves the longest compile.
#if !defined(PIPE_TU) || PIPE_TU == 1
#define PIPE_TU_FP32 1
#endif
#if !defined(PIPE_TU) || PIPE_TU == 2
#define PIPE_TU_FP64 1
#endif

#if PIPE_TU_FP32
template <typename C> static const C* bank_base(const TwiddleBank& b);
template <> const float2* bank_base<float2>(const TwiddleBank& b) { return reinterpret_cast<const float2*>(b.d32); }
template <> const double2* bank_base<double2>(const TwiddleBank& b) { return reinterpret_cast<const double2*>(b.d64); }
template <> const TwPair32* bank_base<TwPair32>(const TwiddleBank& b) {
    return reinterpret_cast<const TwPair32*>(b.d32c);
}

template <typename C> const C* TwiddleBank::get(int n) const {
    for (int i = 0; i < kNumFft; ++i) {
        if (kFftLengths[i] == n) return bank_base<C>(*this) + offset[i];
        if (2 * kFftLengths[i] == n) return bank_base<C>(*this) + offset2[i];
    }
    return nullptr;
}
template <typename C> const C* TwiddleBank::stage(int n, int variant) const {
    if (variant == 0) {
        for (int i = 0; i < kNumFft; ++i)
            if (kFftLengths[i] == n) return bank_base<C>(*this) + soffset[i];
        return nullptr;
    }
    for (int i = 0; i < kNumVariants; ++i)
        if (kPlanVariants[i].n == n && kPlanVariants[i].v == variant) return bank_base<C>(*this) + voffset[i];
    return nullptr;
}
template const float2* TwiddleBank::get<float2>(int) const;
template const double2* TwiddleBank::get<double2>(int) const;
template const float2* TwiddleBank::stage<float2>(int, int) const;
template const double2* TwiddleBank::stage<double2>(int, int) const;
template const TwPair32* TwiddleBank::get<TwPair32>(int) const;
template const TwPair32* TwiddleBank::stage<TwPair32>(int, int) const;

template <class PL> static int stage_exponents(int* m) {
    constexpr int N = PL::LEN;
    int i = 0;
    for (int s = 1; s < PL::S; ++s) {
        const int R = PL::radix(s), NS = plan_ns<PL>(s);
        for (int r = 1; r < R; ++r)
            for (int k = 0; k < NS; ++k) m[i++] = r * k * (N / (NS * R));
    }
    return i;
}

int fft_stage_exponents(int n, int variant, int* m_out) {
    if (variant == 0) {
        switch (n) {
#define X(N_) \
    case N_: return stage_exponents<Plan<N_>>(m_out);
            PIPE_FOR_EACH_N(X)
#undef X
        }
        return -1;
    }
#define X(N_, V_) \
    if (n == N_ && variant == V_) return stage_exponents<Plan<N_, V_>>(m_out);
    PIPE_FOR_EACH_VARIANT(X)
#undef X
    return -1;
}
#endif

// The z passes are persistent: block b handles line groups b, b + gridDim.x, ...
// (LPW lines per group) and issues the global loads of its next group before
// transforming the current one, so each block keeps reads in flight while it
// computes.  Twiddles are staged into LDS once per block.

#ifndef PIPE_Z_PAIR_STORE
#define PIPE_Z_PAIR_STORE 1
#endif
template <typename real, int NH, int E>
constexpr bool Z_PAIR_STORE = PIPE_Z_PAIR_STORE && sizeof(real) == 4 && NH % 2 == 0 && E % 2 == 0;

// P1 / spectra z pass: real lines of n_in values (zero-padded to 2*NH) -> NH packed bins.
// A real line x of length L = 2 NH is read as z[m] = x[2m] + i x[2m+1]; with
// Z = DFT_NH(z) the half spectrum is
//   X[k] = (Z[k] + conj Z[NH-k]) / 2 - i W_L^k (Z[k] - conj Z[NH-k]) / 2,
//   X[0] = Re Z[0] + Im Z[0],  X[NH] = Re Z[0] - Im Z[0]  (stored as slot 0 = (X[0], X[NH])).
// vec2: n_in and in_pitch even and `in` 2-element aligned, so x[2m], x[2m+1] load as one pair.
template <typename real, int NH>
__global__ __launch_bounds__((z_lines<real, NH>() * (NH / Plan<NH, z_V<real, NH>()>::E)))
__attribute__((amdgpu_waves_per_eu(z_waves<real, NH>() > 1 ? z_waves<real, NH>() : z_waves_big<real, NH>())))
void z_r2c_kernel(const real* in, long in_pitch, int n_in, cplx<real>* out, long out_pitch, long nlines,
                  const twid<real>* __restrict__ tw, const twid<real>* __restrict__ tw2, int vec2,
                  const GroupArgs* __restrict__ group) {
    using C = cplx<real>;
    if (group) {
        in = (const real*)group[blockIdx.z].in;
        out = (C*)group[blockIdx.z].out;
    }
    using PL = Plan<NH, z_V<real, NH>()>;
    constexpr int E = PL::E, P = NH / E, LPW = z_lines<real, NH>();
    constexpr int R0 = PL::radix(0);
    constexpr int PADN = lpad_len<z_pad<NH>()>(NH);
    constexpr Sync ZS = z_sync<real, NH>();
    __shared__ C lds[LPW * PADN];
    constexpr bool TW2L = z_tw2_lds<real, NH>();
    __shared__ twid<real> s_tw[NH], s_tw2[TW2L ? NH : 1];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<PL>());
    if constexpr (TW2L) tw2 = stage_twiddles(s_tw2, tw2, NH);
    const gptr<const twid<real>> gtw2 = to_global(tw2);
    auto w2 = [&](int k) -> twid<real> {
        if constexpr (TW2L) return tw2[k];
        else return gtw2[k];
    };
    if constexpr (ZS == Sync::WAVE) __syncthreads();   // the twiddles, written by every wave
    const int t = threadIdx.x % P, l = threadIdx.x / P;
    LdsLine<C, z_pad<NH>()> view{lds + l * PADN};
    const long ngroups = (nlines + LPW - 1) / LPW;
    // stage-0 inputs of line `line` (zero beyond n_in or past the last line)
    const gptr<const real> gin = to_global(in);
    const gptr<C> gout = to_global(out);
    auto load = [&](C* v, long line) {
        const bool active = line < nlines;
        const gptr<const real> src = gin + (active ? line : 0) * in_pitch;
        stage_load<PL, R0>(v, t, [&](int m) -> C {
            if (vec2) {
                if (active && 2 * m < n_in) return reinterpret_cast<gptr<const C>>(src)[m];
                return cmake<C>(0, 0);
            }
            real x0 = 0, x1 = 0;
            if (active) {
                if (2 * m < n_in) x0 = src[2 * m];
                if (2 * m + 1 < n_in) x1 = src[2 * m + 1];
            }
            return cmake<C>(x0, x1);
        });
    };
    C cur[E], nxt[E];
    long g = blockIdx.x;
    if (g < ngroups) load(cur, g * LPW + l);
    for (; g < ngroups; g += gridDim.x) {
        const long gn = g + gridDim.x;
        if (gn < ngroups) load(nxt, gn * LPW + l);
        fft_line_regs<PL, false, ZS>(cur, t, tw, [&](int k, C v) { view.set(k, v); }, view);
        line_sync<ZS>();
        const long line = g * LPW + l;
        // bin k of the half spectrum from Z[k] and Z[NH - k] (slot 0: X[0] and X[NH])
        auto bin = [&](int k) -> C {
            const C zk = view.get(k);
            if (k == 0) return cmake<C>(zk.x + zk.y, zk.x - zk.y);
            const C zn = cconj(view.get(NH - k));
            const C A = cadd(zk, zn), B = csub(zk, zn);
            const C wb = ctw<false>(B, w2(k));  // W^k B;  X = (A - i W^k B) / 2
            return cscale(cmake<C>(A.x + wb.y, A.y - wb.x), (real)0.5);
        };
        if (line < nlines) {
            const gptr<C> dst = gout + line * out_pitch;
            if constexpr (Z_PAIR_STORE<real, NH, E>) {
                // FP32, even NH: each thread writes two adjacent bins with one 16-byte store
                // (the launcher checks that out_pitch is even and the buffer 16-byte aligned)
#pragma unroll
                for (int q = 0; q < E / 2; ++q) {
                    const int k = 2 * (t + q * P);
                    const C x0 = bin(k), x1 = bin(k + 1);
                    *reinterpret_cast<gptr<float4>>(dst + k) = make_float4(x0.x, x0.y, x1.x, x1.y);
                }
            } else {
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    const int k = t + q * P;
                    out_store(dst + k, bin(k));
                }
            }
        }
        line_sync<ZS>();
#pragma unroll
        for (int q = 0; q < E; ++q) cur[q] = nxt[q];
    }
}

// P5: NH packed bins -> real line, unscaled inverse of length 2*NH times `scale`,
// first n_out values kept.  Z'[k] = (X[k] + conj X[NH-k]) + i W_L^{-k} (X[k] - conj X[NH-k]),
// then x[2m] + i x[2m+1] = IDFT_NH(Z')[m].
// vec2: n_out and out_pitch even and `out` 2-element aligned (pairs stored at once).
template <typename real, int NH>
__global__ __launch_bounds__((z_lines<real, NH>() * (NH / Plan<NH, z_V<real, NH>()>::E)))
void z_c2r_kernel(const cplx<real>* in, long in_pitch, real* out, long out_pitch, int n_out, long nlines,
                  real scale, const twid<real>* __restrict__ tw, const twid<real>* __restrict__ tw2, int vec2,
                  const GroupArgs* __restrict__ group) {
    using C = cplx<real>;
    if (group) {
        in = (const C*)group[blockIdx.z].in;
        out = (real*)group[blockIdx.z].out;
        scale = (real)group[blockIdx.z].scale;
    }
    using PL = Plan<NH, z_V<real, NH>()>;
    constexpr int E = PL::E, P = NH / E, LPW = z_lines<real, NH>();
    constexpr int PADN = lpad_len<z_pad<NH>()>(NH);
    constexpr Sync ZS = z_sync<real, NH>();
    __shared__ C lds[LPW * PADN];
    constexpr bool TW2L = true;   // the inverse pass keeps the table staged (reading it from
                                  // global memory would need 28 more registers: spills)
    __shared__ twid<real> s_tw[NH], s_tw2[TW2L ? NH : 1];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<PL>());
    if constexpr (TW2L) tw2 = stage_twiddles(s_tw2, tw2, NH);
    const gptr<const twid<real>> gtw2 = to_global(tw2);
    auto w2 = [&](int k) -> twid<real> {
        if constexpr (TW2L) return tw2[k];
        else return gtw2[k];
    };
    if constexpr (ZS == Sync::WAVE) __syncthreads();   // the twiddles, written by every wave
    const int t = threadIdx.x % P, l = threadIdx.x / P;
    LdsLine<C, z_pad<NH>()> view{lds + l * PADN};
    const long ngroups = (nlines + LPW - 1) / LPW;
    // the packed bins of line `line`, element k = t + q P in slot q
    const gptr<const C> gin = to_global(in);
    const gptr<real> gout = to_global(out);
    auto load = [&](C* v, long line) {
        const bool active = line < nlines;
        const gptr<const C> src = gin + (active ? line : 0) * in_pitch;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            if (active) v[q] = src[t + q * P];
            else v[q] = cmake<C>(0, 0);
        }
    };
    C cur[E], nxt[E];
    long g = blockIdx.x;
    if (g < ngroups) load(cur, g * LPW + l);
    for (; g < ngroups; g += gridDim.x) {
        const long gn = g + gridDim.x;
#pragma unroll
        for (int q = 0; q < E; ++q) view.set(t + q * P, cur[q]);
        line_sync<ZS>();
        if (gn < ngroups) load(nxt, gn * LPW + l);
        const long line = g * LPW + l;
        const bool active = line < nlines;
        const gptr<real> dst = gout + (active ? line : 0) * out_pitch;
        fft_line<PL, true, true, ZS>(
            t, tw,
            [&](int k) -> C {
                const C xk = view.get(k);
                if (k == 0) return cmake<C>(xk.x + xk.y, xk.x - xk.y);
                const C xn = cconj(view.get(NH - k));
                const C A = cadd(xk, xn), B = csub(xk, xn);
                const C wb = ctw<true>(B, w2(k));  // W^{-k} B
                return cmake<C>(A.x - wb.y, A.y + wb.x);  // A + i W^{-k} B
            },
            [&](int m, C v) {
                if (!active) return;
                if (vec2) {
                    if (2 * m < n_out) out_store(reinterpret_cast<gptr<C>>(dst) + m, cmake<C>(v.x * scale, v.y * scale));
                    return;
                }
                if (2 * m < n_out) dst[2 * m] = v.x * scale;
                if (2 * m + 1 < n_out) dst[2 * m + 1] = v.y * scale;
            },
            view);
        line_sync<ZS>();
#pragma unroll
        for (int q = 0; q < E; ++q) cur[q] = nxt[q];
    }
}

// P2 / P4 / spectra y and x passes: lines along a strided dimension.
// Block = T contiguous columns x P threads per line x SPW slabs.
template <typename real, int N, int T, bool INV>
__global__ __launch_bounds__(ce_max(1, 256 / ((N / Plan<N, strided_V<real, N>()>::E) * T)) *
                             (N / Plan<N, strided_V<real, N>()>::E) * T)
void strided_kernel(const cplx<real>* in, cplx<real>* out, int n_in, int n_out, long in_es, long out_es,
                    long ncols, long in_ss, long out_ss, long nslabs, const twid<real>* __restrict__ tw,
                    const GroupArgs* __restrict__ group) {
    using C = cplx<real>;
    if (group) {
        in = (const C*)group[blockIdx.z].in;
        out = (C*)group[blockIdx.z].out;
    }
    using PL = Plan<N, strided_V<real, N>()>;
    constexpr int P = N / PL::E, SPW = ce_max(1, 256 / (P * T));
    __shared__ C lds[SPW * N * T];
    __shared__ twid<real> s_tw[N];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<PL>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, s = threadIdx.x / (T * P);
    const long slab = (long)blockIdx.y * SPW + s;
    const long col = (long)blockIdx.x * T + c;
    const bool active = slab < nslabs && col < ncols;
    const gptr<const C> src = to_global(in) + (active ? slab * in_ss + col : 0);
    const gptr<C> dst = to_global(out) + (active ? slab * out_ss + col : 0);
    LdsCol<C, T> view{lds + s * N * T + c};
    fft_line<PL, INV, false>(
        t, tw,
        [&](int e) -> C {
            if (active && e < n_in) return src[e * in_es];
            return cmake<C>(0, 0);
        },
        [&](int e, C v) {
            if (active && e < n_out) out_store(dst + e * out_es, v);
        },
        view);
}

// ---------------------------------------------------------------- launchers

// Persistent grid of the z passes: at most zcap blocks in total (over all
// members of a grouped launch; a plan's schedule sets zcap), each looping over
// its share of line groups.
static unsigned z_grid(long ngroups, int nmembers, int zcap) {
    long cap = (zcap > 0 ? zcap : 2048) / (nmembers > 0 ? nmembers : 1);
    if (cap < 1) cap = 1;
    return (unsigned)(ngroups < cap ? ngroups : cap);
}


template <typename real>
hipError_t launch_z_r2c(int nh, const real* in, long in_pitch, int n_in, void* out, long out_pitch,
                        long nlines, const TwiddleBank& twb, hipStream_t s, const GroupArgs* group, int ngroup,
                        bool aligned, int zcap) {
    using C = cplx<real>;
    const twid<real>* tw2 = twb.get<twid<real>>(2 * nh);
    if (!tw2 || nlines <= 0) return hipErrorInvalidValue;
    const int vec2 = (n_in % 2 == 0) && (in_pitch % 2 == 0) && aligned &&
                     (group || (uintptr_t)in % (2 * sizeof(real)) == 0);
    switch (nh) {
#define X(N_)                                                                                   \
    case N_: {                                                                                  \
        constexpr int V = z_V<real, N_>(), P = N_ / Plan<N_, V>::E, LPW = z_lines<real, N_>();       \
        const twid<real>* tw = twb.stage<twid<real>>(N_, V);                                                      \
        if (!tw) return hipErrorInvalidValue;                                                   \
        /* paired 16-byte stores need an even output pitch and 16-byte aligned lines */        \
        if (Z_PAIR_STORE<real, N_, Plan<N_, V>::E> &&                                           \
            (out_pitch % 2 || (!group && (uintptr_t)out % 16)))                                 \
            return hipErrorInvalidValue;                                                        \
        dim3 grid(z_grid((nlines + LPW - 1) / LPW, ngroup, zcap), 1, (unsigned)ngroup);               \
        hipLaunchKernelGGL((z_r2c_kernel<real, N_>), grid, dim3(LPW * P), 0, s, in, in_pitch,   \
                           n_in, (C*)out, out_pitch, nlines, tw, tw2, vec2, group);             \
        return hipGetLastError();                                                               \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename real>
hipError_t launch_z_c2r(int nh, const void* in, long in_pitch, real* out, long out_pitch, int n_out,
                        long nlines, real scale, const TwiddleBank& twb, hipStream_t s, const GroupArgs* group,
                        int ngroup, bool aligned, int zcap) {
    using C = cplx<real>;
    const twid<real>* tw2 = twb.get<twid<real>>(2 * nh);
    if (!tw2 || nlines <= 0) return hipErrorInvalidValue;
    const int vec2 = (n_out % 2 == 0) && (out_pitch % 2 == 0) && aligned &&
                     (group || (uintptr_t)out % (2 * sizeof(real)) == 0);
    switch (nh) {
#define X(N_)                                                                                   \
    case N_: {                                                                                  \
        constexpr int V = z_V<real, N_>(), P = N_ / Plan<N_, V>::E, LPW = z_lines<real, N_>();       \
        const twid<real>* tw = twb.stage<twid<real>>(N_, V);                                                      \
        if (!tw) return hipErrorInvalidValue;                                                   \
        dim3 grid(z_grid((nlines + LPW - 1) / LPW, ngroup, zcap), 1, (unsigned)ngroup);               \
        hipLaunchKernelGGL((z_c2r_kernel<real, N_>), grid, dim3(LPW * P), 0, s, (const C*)in,   \
                           in_pitch, out, out_pitch, n_out, nlines, scale, tw, tw2, vec2, group); \
        return hipGetLastError();                                                               \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename real>
hipError_t launch_strided(int n, bool inverse, const void* in, void* out, int n_in, int n_out, long in_es,
                          long out_es, long ncols, long in_ss, long out_ss, long nslabs,
                          const TwiddleBank& twb, hipStream_t s, const GroupArgs* group, int ngroup) {
    using C = cplx<real>;
    if (ncols <= 0 || nslabs <= 0) return hipErrorInvalidValue;
    switch (n) {
#define X(N_)                                                                                      \
    case N_: {                                                                                     \
        constexpr int T = strided_T<real, N_>(), V = strided_V<real, N_>();                        \
        constexpr int P = N_ / Plan<N_, V>::E, SPW = ce_max(1, 256 / (P * T));                     \
        const twid<real>* tw = twb.stage<twid<real>>(N_, V);                                                         \
        if (!tw) return hipErrorInvalidValue;                                                      \
        dim3 grid((unsigned)((ncols + T - 1) / T), (unsigned)((nslabs + SPW - 1) / SPW),           \
                  (unsigned)ngroup);                                                               \
        if (inverse)                                                                               \
            hipLaunchKernelGGL((strided_kernel<real, N_, T, true>), grid, dim3(SPW * P * T), 0, s, \
                               (const C*)in, (C*)out, n_in, n_out, in_es, out_es, ncols, in_ss,     \
                               out_ss, nslabs, tw, group);                                         \
        else                                                                                       \
            hipLaunchKernelGGL((strided_kernel<real, N_, T, false>), grid, dim3(SPW * P * T), 0,   \
                               s, (const C*)in, (C*)out, n_in, n_out, in_es, out_es, ncols, in_ss,  \
                               out_ss, nslabs, tw, group);                                         \
        return hipGetLastError();                                                                  \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

#define PIPE_INST(real)                                                                               \
    template hipError_t launch_z_r2c<real>(int, const real*, long, int, void*, long, long,             \
                                           const TwiddleBank&, hipStream_t, const GroupArgs*, int, bool, int); \
    template hipError_t launch_z_c2r<real>(int, const void*, long, real*, long, int, long, real,       \
                                           const TwiddleBank&, hipStream_t, const GroupArgs*, int, bool, int); \
    template hipError_t launch_strided<real>(int, bool, const void*, void*, int, int, long, long, long, \
                                             long, long, long, const TwiddleBank&, hipStream_t,         \
                                             const GroupArgs*, int);
#if PIPE_TU_FP32
PIPE_INST(float)
#endif
#if PIPE_TU_FP64
PIPE_INST(double)
#endif
#undef PIPE_INST

}  // namespace pipe
