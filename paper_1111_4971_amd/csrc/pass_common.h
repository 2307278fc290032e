// pass_common.h -- device helpers shared by the pass kernels (passes.hip, band.hip).
#pragma once
#include "fft_engine.h"
#include "pipe_internal.h"

namespace pipe {

// LDS views ----------------------------------------------------------------

// Column-interleaved: element e of column c at base[e * T] (base = lds + c).
template <typename C, int T> struct LdsCol {
    C* base;
    __device__ __forceinline__ C get(int e) const { return base[e * T]; }
    __device__ __forceinline__ void set(int e, C v) const { base[e * T] = v; }
};

// Contiguous line padded by one slot every 2^SH values (SH = 0: no padding);
// the padding breaks the power-of-two strides of the exchanges.
template <int SH> __device__ __forceinline__ int lpad(int e) {
    if constexpr (SH == 0) return e;
    else return e + (e >> SH);
}
template <int SH> constexpr int lpad_len(int n) { return SH == 0 ? n : n + (n >> SH) + 1; }
template <typename C, int SH = 4> struct LdsLine {
    C* base;
    __device__ __forceinline__ C get(int e) const { return base[lpad<SH>(e)]; }
    __device__ __forceinline__ void set(int e, C v) const { base[lpad<SH>(e)] = v; }
};

constexpr int ce_max(int a, int b) { return a > b ? a : b; }

// Launch-shape constants (overridable at build time for tuning sweeps).
#ifndef PIPE_LDS_CAP
#define PIPE_LDS_CAP 65536   // LDS bytes a y-pass or fused x-pass block may use
#endif
#ifndef PIPE_Z_THREADS
#define PIPE_Z_THREADS 256   // threads per block of the z passes (lines per block = this / P)
#endif
#ifndef PIPE_XPROD_TMAX
#define PIPE_XPROD_TMAX 8    // widest kz tile of the fused x pass
#endif
#ifndef PIPE_STRIDED_TMAX
#define PIPE_STRIDED_TMAX 32 // widest column tile of the y passes
#endif
// lines per block of the z passes: PIPE_Z_THREADS / P, halved until the block's LDS fits PIPE_LDS_CAP
#ifndef PIPE_TW_LDS
#define PIPE_TW_LDS 1        // stage twiddle tables in LDS at block start
#endif

// Every supported FFT length (every 2^p 3^q in [8, 1024]), for the launchers'
// switch statements; must list the same lengths as kFftLengths.
#define PIPE_FOR_EACH_N(X)                                                                               \
    X(8) X(9) X(12) X(16) X(18) X(24) X(27) X(32) X(36) X(48) X(54) X(64) X(72) X(81) X(96) X(108)      \
    X(128) X(144) X(162) X(192) X(216) X(243) X(256) X(288) X(324) X(384) X(432) X(486) X(512) X(576) \
    X(648) X(729) X(768) X(864) X(972) X(1024)
// The lengths the banded x pass takes: its orbit items tile E/4 per thread, so
// N and the plan's E must be multiples of 4; must match kBandLengths.
#define PIPE_FOR_EACH_BAND_N(X)                                                                          \
    X(8) X(12) X(16) X(24) X(32) X(36) X(48) X(64) X(72) X(96) X(108) X(128) X(144) X(192) X(216)       \
    X(256) X(288) X(384) X(432) X(512) X(576) X(768) X(864) X(1024)

// Column tile of the y passes for plan variant V: PIPE_STRIDED_TMAX columns per
// row segment, halved until the block's LDS (slabs x N x T complex) fits in
// PIPE_LDS_CAP and its P x T threads (P = N / E per line) fit in 1024.
template <typename real, int N, int V> constexpr int strided_T_of() {
    constexpr int P = N / Plan<N, V>::E;
    int t = PIPE_STRIDED_TMAX;
    while (t > 1 && (ce_max(1, 256 / (P * t)) * N * t * (int)sizeof(real) * 2 > PIPE_LDS_CAP || P * t > 1024)) t /= 2;
    return t;
}
// Plan of the y passes: the narrow variant where the default plan holds more
// than 8 values per thread in FP64, and in FP32 where it holds more than 16
// and the narrow plan keeps the same column tile.  A block's LDS tile is N x T
// complex values whatever the plan, so fewer values per thread means more
// waves on the same tile (FP32 432: 5 -> 9 waves per block, y passes 0.33 ->
// 0.39 of HBM peak; 324: 0.42 -> 0.52); the 16-value power-of-two plans stay,
// their narrow variants measured 5 % slower.
template <typename real, int N> constexpr int strided_V() {
    if constexpr (sizeof(real) == 8) {
        return narrow_variant<N>(8);
    } else {
        constexpr int v = narrow_variant<N>(16);
        if constexpr (v != 0) {
            if constexpr (strided_T_of<real, N, v>() >= strided_T_of<real, N, 0>()) return v;
        }
        return 0;
    }
}
template <typename real, int N> constexpr int strided_T() { return strided_T_of<real, N, strided_V<real, N>()>(); }

// Pointer into device global memory.  Buffers taken from a grouped launch's
// descriptor array arrive as generic pointers, which compile to flat memory
// instructions; flat accesses also count on the LDS wait counter, so every LDS
// wait would drain the global loads in flight.  The kernels address their
// buffers through global-typed pointers instead.  (The host pass of the
// compiler only parses device code and has no such address space.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T> using gptr = T*;
#endif
template <typename T> __device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)p; }

// Store of a pass's output element; NT: as a non-temporal store (the
// fused x pass can take this as part of its plan's schedule: it keeps the
// written rows from displacing the spectra and rows other blocks still read).
template <bool NT = false, typename C> __device__ __forceinline__ void out_store(gptr<C> p, C v) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (NT) {
        using R = decltype(C::x);
        typedef R V2 __attribute__((ext_vector_type(2)));
        V2 w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, reinterpret_cast<__attribute__((address_space(1))) V2*>(p));
        return;
    }
#endif
    *p = v;
}

// Copy n twiddles into LDS (no barrier: every use follows a later barrier).
template <typename C>
__device__ __forceinline__ const C* stage_twiddles(C* s_tw, const C* __restrict__ tw, int n) {
#if PIPE_TW_LDS
    for (int i = threadIdx.x; i < n; i += blockDim.x) s_tw[i] = tw[i];
    return s_tw;
#else
    return tw;
#endif
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2) in
// order of their linear id.  xcd_remap turns the linear id p < total into a
// logical id such that consecutive logical ids run on the same XCD, one after
// the other: XCD x takes the x-th contiguous share of logical ids.
#ifndef PIPE_NUM_XCD
#define PIPE_NUM_XCD 8
#endif
__device__ __forceinline__ unsigned xcd_remap(unsigned p, unsigned total) {
    const unsigned q = total / PIPE_NUM_XCD, r = total % PIPE_NUM_XCD;
    const unsigned xcd = p % PIPE_NUM_XCD, k = p / PIPE_NUM_XCD;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// Exchange ordering of the z passes: with PIPE_Z_WAVE_SYNC, a length whose
// lines each fit inside one wavefront (P divides 64) orders its LDS exchanges
// per wave, so the waves of a block need not wait for each other.
#ifndef PIPE_Z_WAVE_SYNC
#define PIPE_Z_WAVE_SYNC 1
#endif
// Plan of the z passes: each thread holds two line groups (current and
// prefetched), so plans with more than 12 values per thread (8 in FP64) take
// the narrow variant.
// LDS padding of the z passes' lines: one slot every 16 for power-of-two
// lengths; none where the length has a factor 3 (its exchange strides are not
// powers of two, and the padding itself then adds bank conflicts).
#ifndef PIPE_Z_PAD_POW2
#define PIPE_Z_PAD_POW2 4
#endif
#ifndef PIPE_Z_PAD_SMOOTH
#define PIPE_Z_PAD_SMOOTH 0
#endif
template <int NH> constexpr int z_pad() { return (NH & (NH - 1)) == 0 ? PIPE_Z_PAD_POW2 : PIPE_Z_PAD_SMOOTH; }
// Waves per SIMD the FP32 z forward pass's registers must allow where its plan
// holds 12 values per thread (1: no constraint).  Left alone the compiler takes
// 120-150 registers there (3 waves per SIMD); at 4 waves most lengths fit
// without spills and lengths 288-768 ran 4-7 % faster (432: 33.8 -> 31.4 us at
// 128x128x432), 48-192 unchanged; 972 would spill heavily and keeps 1.  (The z
// inverse pass gained at 768 but lost up to 4 % at the small lengths.)
template <typename real, int NH> constexpr int z_V();
template <typename real, int NH> constexpr int z_waves() {
    return (sizeof(real) == 4 && Plan<NH, z_V<real, NH>()>::E == 12 && NH != 972) ? 4 : 1;
}
// The z forward pass in FP64 at lz/2 >= 1024, where the split table is read
// from global memory (see z_tw2_lds): 3 waves per SIMD, the blocks the LDS allows.
template <typename real, int NH> constexpr bool z_tw2_lds();
template <typename real, int NH> constexpr int z_waves_big() { return z_tw2_lds<real, NH>() ? 1 : 3; }
template <typename real, int NH> constexpr int z_V() { return narrow_variant<NH>(sizeof(real) == 8 ? 8 : 12); }

template <typename real, int NH> constexpr Sync z_sync() {
    constexpr int P = NH / Plan<NH, z_V<real, NH>()>::E;
    return (PIPE_Z_WAVE_SYNC && P <= 64 && 64 % P == 0) ? Sync::WAVE : Sync::BLOCK;
}

template <typename real, int NH> constexpr int z_lines() {
    int l = ce_max(1, PIPE_Z_THREADS / (NH / Plan<NH, z_V<real, NH>()>::E));
    while (l > 1 && l * lpad_len<z_pad<NH>()>(NH) * 2 * (int)sizeof(real) > PIPE_LDS_CAP) l /= 2;
    return l;
}
// Whether a z forward block stages the real/complex split's table W_2N in LDS.
// Each line reads it once, at consecutive entries; in FP64 at lz/2 >= 1024
// the staged table (16 KB) costs a block per CU (2 instead of 3), so there the
// forward pass reads it from global memory and is held to the 168 registers
// of 3 waves per SIMD (no spills).
#ifndef PIPE_Z_TW2_RULE
#define PIPE_Z_TW2_RULE 1
#endif
template <typename real, int NH> constexpr bool z_tw2_lds() {
    return !(PIPE_Z_TW2_RULE && sizeof(real) == 8 && NH >= 1024);
}


// Spectra table (plan precision), 9 values per orbit (kx <= lx/2, ky <= ly/2, kz):
//   0: T_cc (real)   1,2: T_cr   3,4: T_rc   5,6: T_rr(kx,ky)   7,8: T_rr(-kx,ky)
// Symmetries of real Green arrays: T_cc real and even in kx, ky; T_cr even in kx,
// T_cr(kx,-ky) = conj; T_rc even in ky, T_rc(-kx,ky) = conj; T_rr(-kx,-ky) = conj T_rr(kx,ky).
template <typename real> struct Orbit {
    real cc;
    cplx<real> cr, rc, rr, rr2;
};

// Nine values of one orbit, `stride` apart (T in the tiled table, 1 for kz = lz/2).
template <typename real>
__device__ __forceinline__ Orbit<real> load_orbit(gptr<const real> e, int stride) {
    using C = cplx<real>;
    Orbit<real> o;
    o.cc = e[0];
    o.cr = cmake<C>(e[stride], e[2 * stride]);
    o.rc = cmake<C>(e[3 * stride], e[4 * stride]);
    o.rr = cmake<C>(e[5 * stride], e[6 * stride]);
    o.rr2 = cmake<C>(e[7 * stride], e[8 * stride]);
    return o;
}

// The same from LDS.
template <typename real>
__device__ __forceinline__ Orbit<real> load_orbit_lds(const real* e, int stride) {
    using C = cplx<real>;
    Orbit<real> o;
    o.cc = e[0];
    o.cr = cmake<C>(e[stride], e[2 * stride]);
    o.rc = cmake<C>(e[3 * stride], e[4 * stride]);
    o.rr = cmake<C>(e[5 * stride], e[6 * stride]);
    o.rr2 = cmake<C>(e[7 * stride], e[8 * stride]);
    return o;
}

// T_ab at (sx kx, sy ky) from the orbit entry (sx, sy = +1 or -1).
template <typename real> struct OrbitView {
    const Orbit<real>& o;
    __device__ __forceinline__ cplx<real> cc(int, int) const { return cmake<cplx<real>>(o.cc, (real)0); }
    __device__ __forceinline__ cplx<real> cr(int, int sy) const { return sy > 0 ? o.cr : cconj(o.cr); }
    __device__ __forceinline__ cplx<real> rc(int sx, int) const { return sx > 0 ? o.rc : cconj(o.rc); }
    __device__ __forceinline__ cplx<real> rr(int sx, int sy) const {
        if (sx > 0 && sy > 0) return o.rr;
        if (sx < 0 && sy < 0) return cconj(o.rr);
        if (sx < 0) return o.rr2;            // (-kx, ky)
        return cconj(o.rr2);                 // (kx, -ky)
    }
};

// acc += S t x (S = +1 or -1) as four fused multiply-adds.
template <int S, typename C> __device__ __forceinline__ void cfma(C& acc, C t, C x) {
    const auto tx = S > 0 ? t.x : -t.x, ty = S > 0 ? t.y : -t.y;
    acc.x = fma(tx, x.x, acc.x);
    acc.x = fma(-ty, x.y, acc.x);
    acc.y = fma(tx, x.y, acc.y);
    acc.y = fma(ty, x.x, acc.y);
}

// r[q] = rho at point q of the orbit: q = 0 (kx,ky), 1 (-kx,ky), 2 (kx,-ky), 3 (-kx,-ky).
// Forward: Phi(p) = sum_ab sigma_ab T_ab(p) rho(S_ab p).
// Adjoint: Phi(p) = sum_ab sigma_ab conj(T_ab(S_ab p)) g(S_ab p)  (transposed gather).
// Outputs q < NQ only (NQ = 2 where Phi is Hermitian and q = 2, 3 follow by conjugation).
template <bool ADJ, int NQ = 4, typename real>
__device__ __forceinline__ void orbit_product(const Orbit<real>& o, const cplx<real>* r, cplx<real>* out) {
    using C = cplx<real>;
    OrbitView<real> T{o};
    const int SX[4] = {1, -1, 1, -1}, SY[4] = {1, 1, -1, -1};
    auto idx = [](int sx, int sy) { return (sx > 0 ? 0 : 1) + (sy > 0 ? 0 : 2); };
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int sx = SX[q], sy = SY[q];
        const int qcr = idx(sx, -sy), qrc = idx(-sx, sy), qrr = idx(-sx, -sy);
        C tcc, tcr, trc, trr;
        if constexpr (!ADJ) {
            tcc = T.cc(sx, sy);
            tcr = T.cr(sx, sy);
            trc = T.rc(sx, sy);
            trr = T.rr(sx, sy);
        } else {
            tcc = cconj(T.cc(sx, sy));
            tcr = cconj(T.cr(sx, -sy));
            trc = cconj(T.rc(-sx, sy));
            trr = cconj(T.rr(-sx, -sy));
        }
        // T_cc is real: two products; the other three terms as fused multiply-adds
        C acc = cscale(r[q], tcc.x);
        cfma<-1>(acc, tcr, r[qcr]);
        cfma<-1>(acc, trc, r[qrc]);
        cfma<1>(acc, trr, r[qrr]);
        out[q] = acc;
    }
}


}  // namespace pipe
