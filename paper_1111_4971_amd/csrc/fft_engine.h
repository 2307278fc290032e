// fft_engine.h -- register/LDS Stockham FFT building blocks for gfx950.
//
// A length-N line (N = 2^p 3^q, 8 <= N <= 1024) is processed by P = N/E
// threads, each holding E complex values in registers.  Every stage of radix R
// (2, 3, 4, 8, 9 or 16) applies E/R radix-R butterflies per thread (Stockham
// autosort: inputs j + r N/R, twiddles W_{Ns R}^{r (j mod Ns)}, outputs
// (j div Ns) Ns R + (j mod Ns) + r Ns).  Between stages the line is exchanged
// through LDS.  The first stage reads its inputs straight from any source
// (global memory with zero padding, or LDS) and the last stage writes element
// j + r N/R, i.e. natural order, straight to any sink, so a transform costs
// (stages - 1) LDS round trips.
//
// Direction: forward uses W = e^{-2 pi i/N}, inverse W^{-1}; both unscaled.
// Twiddles come from a per-length stage table (stage_tw_offset) whose values
// W_N^m are computed on the host in extended precision and rounded once to the
// working precision.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace pipe {

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename R> using cplx = typename cplx_t<R>::type;

// Twiddles.  FP64 passes take W as one double2.  FP32 passes take W either
// rounded once to float2, or (PIPE_TW_COMPENSATED) as an unevaluated sum
// hi + lo of two float2 (lo = the FP32 rounding of W - hi), applied as
// a hi + a lo, which removes the twiddles' own rounding from the transform.
#ifndef PIPE_TW_COMPENSATED
#define PIPE_TW_COMPENSATED 0
#endif
struct TwPair32 {
    float2 hi, lo;
};
template <typename real> struct twid_t { using type = cplx<real>; };
template <> struct twid_t<float> { using type = std::conditional_t<PIPE_TW_COMPENSATED != 0, TwPair32, float2>; };
template <typename real> using twid = typename twid_t<real>::type;
// the complex type a twiddle type multiplies
template <typename TW> struct tw_complex { using type = TW; };
template <> struct tw_complex<TwPair32> { using type = float2; };


template <typename C> __device__ __forceinline__ C cmake(decltype(C::x) x, decltype(C::x) y) { C c; c.x = x; c.y = y; return c; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
    return cmake<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C cmul_mi(C a) {
    return INV ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}
// twiddle multiply: a * w (forward) or a * conj(w) (inverse)
template <bool INV, typename C> __device__ __forceinline__ C ctw(C a, C w) {
    return INV ? cmulc(a, w) : cmul(a, w);
}
template <bool INV> __device__ __forceinline__ float2 ctw(float2 a, TwPair32 w) {
    // the lo products first, then the hi products fused onto them
    const float sy = INV ? -1.f : 1.f;
    const float lr = a.x * w.lo.x - sy * (a.y * w.lo.y);
    const float li = sy * (a.x * w.lo.y) + a.y * w.lo.x;
    float2 r;
    r.x = fmaf(a.x, w.hi.x, fmaf(-sy * a.y, w.hi.y, lr));
    r.y = fmaf(sy * a.x, w.hi.y, fmaf(a.y, w.hi.x, li));
    return r;
}

// ---------------------------------------------------------------- butterflies
// In-place DFT of R values v[0], v[s], ..., v[(R-1)s] -- always called with s = 1.

template <bool INV, typename C> __device__ __forceinline__ void dft2(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV, typename C> __device__ __forceinline__ void dft3(C* v) {
    using R = decltype(C::x);
    const R s3 = (R)0.86602540378443864676372317075294;  // sqrt(3)/2
    C t1 = cadd(v[1], v[2]);
    C t2 = csub(v[0], cscale(t1, (R)0.5));
    C d = csub(v[1], v[2]);
    // forward: -i s3 d ; inverse: +i s3 d
    C t3 = cmul_mi<INV>(cscale(d, s3));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C* v) {
    C t0 = cadd(v[0], v[2]);
    C t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]);
    C t3 = cmul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft8(C* v) {
    using R = decltype(C::x);
    const R h = (R)0.70710678118654752440084436210485;
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // o[k] *= W8^k : forward W8 = (h, -h), inverse (h, h)
    C o1 = INV ? cmake<C>(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : cmake<C>(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    C o2 = cmul_mi<INV>(o[2]);
    C o3 = INV ? cmake<C>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : cmake<C>(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft16(C* v) {
    using R = decltype(C::x);
    // n = n1 + 4 n2, k = k2 + 4 k1:  four DFT4 over n2, twiddle W16^{n1 k2}, four DFT4 over n1
    C a[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) a[n1][n2] = v[n1 + 4 * n2];
        dft4<INV>(a[n1]);
    }
    const R c1 = (R)0.92387953251128675612818318939679;  // cos(pi/8)
    const R s1 = (R)0.38268343236508977172845998403040;  // sin(pi/8)
    const R h = (R)0.70710678118654752440084436210485;
    // W16^m for m = n1*k2 in {1,2,3,4,6,9}; forward = (cos, -sin)
    const R sg = INV ? (R)1 : (R)-1;
    const C w1 = cmake<C>(c1, sg * s1), w2 = cmake<C>(h, sg * h), w3 = cmake<C>(s1, sg * c1);
    const C w6 = cmake<C>(-h, sg * h), w9 = cmake<C>(-c1, -sg * s1);
    a[1][1] = cmul(a[1][1], w1);
    a[1][2] = cmul(a[1][2], w2);
    a[1][3] = cmul(a[1][3], w3);
    a[2][1] = cmul(a[2][1], w2);
    a[2][2] = cmul_mi<INV>(a[2][2]);
    a[2][3] = cmul(a[2][3], w6);
    a[3][1] = cmul(a[3][1], w3);
    a[3][2] = cmul(a[3][2], w6);
    a[3][3] = cmul(a[3][3], w9);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        C b[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
        dft4<INV>(b);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = b[k1];
    }
}

template <bool INV, typename C> __device__ __forceinline__ void dft9(C* v) {
    using R = decltype(C::x);
    // n = n1 + 3 n2, k = k2 + 3 k1:  three DFT3 over n2, twiddle W9^{n1 k2}, three DFT3 over n1
    C a[3][3];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) a[n1][n2] = v[n1 + 3 * n2];
        dft3<INV>(a[n1]);
    }
    // W9^m = cos(2 pi m/9) -+ i sin(2 pi m/9) for m = n1 k2 in {1, 2, 4}
    const R sg = INV ? (R)1 : (R)-1;
    const C w1 = cmake<C>((R)0.766044443118978035202392650555416674, sg * (R)0.642787609686539326322643409907263433);
    const C w2 = cmake<C>((R)0.173648177666930348851716626769314796, sg * (R)0.984807753012208059366743024589523014);
    const C w4 = cmake<C>((R)-0.93969262078590838405410927732473147, sg * (R)0.342020143325668733044099614682259581);
    a[1][1] = cmul(a[1][1], w1);
    a[1][2] = cmul(a[1][2], w2);
    a[2][1] = cmul(a[2][1], w2);
    a[2][2] = cmul(a[2][2], w4);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
        C b[3] = {a[0][k2], a[1][k2], a[2][k2]};
        dft3<INV>(b);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) v[k2 + 3 * k1] = b[k1];
    }
}

template <int R, bool INV, typename C> __device__ __forceinline__ void dft(C* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 9) dft9<INV>(v);
    else if constexpr (R == 16) dft16<INV>(v);
    else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------- length plans
// E = values per thread, then the radices applied first to last (product N,
// each dividing E).  E stays <= 24 so that a z-pass thread can hold two lines'
// worth of FP64 values (current and prefetched); single-stage plans have
// P = 1, so a line is never shared by threads of one stage (in-place safe).

// Plan<N> is a length's default plan; Plan<N, V> with V >= 1 are variants a
// kernel may choose instead (another E, so another thread count per line).
template <int N, int V = 0> struct Plan;
#define PIPE_PLAN_V(N_, V_, E_, ...)                                                   \
    template <> struct Plan<N_, V_> {                                                  \
        static constexpr int LEN = N_, VAR = V_, E = E_;                               \
        static constexpr int rad[] = {__VA_ARGS__};                                    \
        static constexpr int S = (int)(sizeof(rad) / sizeof(int));                     \
        static constexpr int radix(int s) { return rad[s]; }                           \
    };
#define PIPE_PLAN(N_, E_, ...) PIPE_PLAN_V(N_, 0, E_, __VA_ARGS__)
PIPE_PLAN(8, 8, 8)
PIPE_PLAN(9, 9, 9)
PIPE_PLAN(12, 12, 3, 4)
PIPE_PLAN(16, 16, 16)
PIPE_PLAN(18, 6, 3, 3, 2)
PIPE_PLAN(24, 24, 3, 8)
PIPE_PLAN(27, 9, 9, 3)
PIPE_PLAN(32, 8, 4, 8)
PIPE_PLAN(36, 12, 3, 3, 4)
PIPE_PLAN(48, 12, 3, 4, 4)
PIPE_PLAN(54, 18, 9, 3, 2)
PIPE_PLAN(64, 8, 8, 8)
PIPE_PLAN(72, 24, 3, 3, 8)
PIPE_PLAN(81, 9, 9, 9)
PIPE_PLAN(96, 24, 3, 4, 8)
PIPE_PLAN(108, 12, 3, 3, 3, 4)
PIPE_PLAN(128, 16, 8, 16)
PIPE_PLAN(144, 12, 3, 3, 4, 4)
PIPE_PLAN(162, 18, 9, 9, 2)
PIPE_PLAN(192, 24, 3, 8, 8)
PIPE_PLAN(216, 24, 3, 3, 3, 8)
PIPE_PLAN(243, 9, 9, 9, 3)
PIPE_PLAN(256, 16, 16, 16)
PIPE_PLAN(288, 24, 3, 3, 8, 4)
PIPE_PLAN(324, 18, 9, 9, 2, 2)
PIPE_PLAN(384, 24, 3, 8, 8, 2)
PIPE_PLAN(432, 24, 3, 3, 3, 8, 2)
PIPE_PLAN(486, 18, 9, 9, 3, 2)
PIPE_PLAN(512, 8, 8, 8, 8)
PIPE_PLAN(576, 24, 3, 3, 8, 8)
PIPE_PLAN(648, 18, 9, 9, 2, 2, 2)
PIPE_PLAN(729, 9, 9, 9, 9)
PIPE_PLAN(768, 24, 3, 8, 8, 4)
PIPE_PLAN(864, 24, 3, 3, 3, 8, 4)
PIPE_PLAN(972, 18, 9, 9, 3, 2, 2)
PIPE_PLAN(1024, 16, 16, 16, 4)
// Variant 2: at most 12 values per thread (8 for powers of two), for kernels
// whose registers or LDS would otherwise limit them to one or two waves per
// SIMD (z passes holding two line groups, FP64 passes); more threads per line
// and usually one more stage.
PIPE_PLAN_V(16, 2, 8, 4, 4)
PIPE_PLAN_V(24, 2, 12, 3, 4, 2)
PIPE_PLAN_V(54, 2, 6, 3, 3, 3, 2)
PIPE_PLAN_V(72, 2, 12, 3, 3, 4, 2)
PIPE_PLAN_V(96, 2, 12, 3, 4, 4, 2)
PIPE_PLAN_V(128, 2, 8, 8, 4, 4)
PIPE_PLAN_V(162, 2, 6, 3, 3, 3, 3, 2)
PIPE_PLAN_V(192, 2, 12, 3, 4, 4, 4)
PIPE_PLAN_V(216, 2, 12, 3, 3, 3, 4, 2)
PIPE_PLAN_V(256, 2, 8, 8, 8, 4)
PIPE_PLAN_V(288, 2, 12, 3, 3, 4, 4, 2)
PIPE_PLAN_V(324, 2, 12, 3, 3, 3, 3, 4)
PIPE_PLAN_V(384, 2, 12, 3, 4, 4, 4, 2)
PIPE_PLAN_V(432, 2, 12, 3, 3, 3, 4, 4)
PIPE_PLAN_V(486, 2, 6, 3, 3, 3, 3, 3, 2)
PIPE_PLAN_V(576, 2, 12, 3, 3, 4, 4, 4)
PIPE_PLAN_V(648, 2, 12, 3, 3, 3, 3, 4, 2)
PIPE_PLAN_V(768, 2, 12, 3, 4, 4, 4, 4)
PIPE_PLAN_V(864, 2, 12, 3, 3, 3, 4, 4, 2)
PIPE_PLAN_V(972, 2, 12, 3, 3, 3, 3, 3, 4)
PIPE_PLAN_V(1024, 2, 8, 8, 8, 4, 4)
#undef PIPE_PLAN
#undef PIPE_PLAN_V

// The (length, variant) pairs that exist beyond the defaults; the twiddle bank
// holds a stage table for each.
#define PIPE_FOR_EACH_VARIANT(X)                                                                     \
    X(16, 2) X(24, 2) X(54, 2) X(72, 2) X(96, 2) X(128, 2) X(162, 2) X(192, 2) X(216, 2) X(256, 2)  \
    X(288, 2) X(324, 2) X(384, 2) X(432, 2) X(486, 2) X(576, 2) X(648, 2) X(768, 2) X(864, 2)      \
    X(972, 2) X(1024, 2)

// Whether Plan<N, V> is defined.
template <int N, int V, typename = void> struct plan_exists { static constexpr bool value = false; };
template <int N, int V> struct plan_exists<N, V, decltype((void)Plan<N, V>::E)> {
    static constexpr bool value = true;
};

// The plan a kernel uses for length N: variant 2 when the default plan holds
// more than emax values per thread and the variant exists, else the default.
template <int N> constexpr int narrow_variant(int emax) {
    if constexpr (plan_exists<N, 2>::value) return Plan<N>::E > emax ? 2 : 0;
    return 0;
}

template <class PL> __host__ __device__ constexpr int plan_ns(int s) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= PL::radix(i);
    return ns;
}

template <class PL> constexpr bool plan_ok() {
    constexpr int N = PL::LEN, E = PL::E, S = PL::S;
    if (N % E != 0 || plan_ns<PL>(S) != N) return false;
    for (int s = 0; s < S; ++s)
        if (E % PL::radix(s) != 0) return false;
    return S > 1 || E == N;
}

// Stage twiddle table of plan PL (length N): stage s >= 1 (radix R, span NS)
// owns R - 1 runs of NS values starting at stage_tw_offset<PL>(NS); run r - 1
// holds W_{NS R}^{r k} = W_N^{r k N / (NS R)} for k < NS.  The lanes of a stage
// differ in k, so they read consecutive entries (no LDS bank conflicts), where
// a natural-order table would be read at stride r N / (NS R).
template <class PL> __host__ __device__ constexpr int stage_tw_offset(int ns) {
    int off = 0;
    for (int s = 1; s < PL::S; ++s) {
        if (plan_ns<PL>(s) == ns) return off;
        off += (PL::radix(s) - 1) * plan_ns<PL>(s);
    }
    return off;
}
template <class PL> __host__ __device__ constexpr int stage_tw_size() { return stage_tw_offset<PL>(0); }

// Exchange ordering between the stages of a transform.  BLOCK: a block barrier
// (the threads of a line may sit in several waves).  WAVE: every line lies
// inside one wavefront (P divides 64), so ordering the wave's own LDS accesses
// suffices and the waves of a block run independently.
enum class Sync { BLOCK, WAVE };
template <Sync SY> __device__ __forceinline__ void line_sync() {
    if constexpr (SY == Sync::BLOCK) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---------------------------------------------------------------- stage pieces
// v[b*R + r] holds input r of the thread's b-th butterfly, j = t + b*P.

// Load the inputs of a stage with radix R: element index e = j + r*N/R.
template <class PL, int R, typename C, typename Src>
__device__ __forceinline__ void stage_load(C* v, int t, Src src) {
    constexpr int N = PL::LEN, E = PL::E, P = N / E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[b * R + r] = src(t + b * P + r * (N / R));
}

// Twiddle (for Ns > 1) and butterfly in registers.
template <class PL, int R, int NS, bool INV, typename C, typename TW>
__device__ __forceinline__ void stage_compute(C* v, int t, const TW* __restrict__ tw) {
    constexpr int N = PL::LEN, E = PL::E, P = N / E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if constexpr (NS > 1) {
            const int k = (t + b * P) % NS;
            constexpr int off = stage_tw_offset<PL>(NS);
#pragma unroll
            for (int r = 1; r < R; ++r) v[b * R + r] = ctw<INV>(v[b * R + r], tw[off + (r - 1) * NS + k]);
        }
        dft<R, INV>(&v[b * R]);
    }
}

// Store the outputs of a stage: element (j div NS) NS R + (j mod NS) + r NS.
template <class PL, int R, int NS, typename C, typename Dst>
__device__ __forceinline__ void stage_store(const C* v, int t, Dst dst) {
    constexpr int N = PL::LEN, E = PL::E, P = N / E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * P;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) dst(base + r * NS, v[b * R + r]);
    }
}

// Stage s of the transform from its inputs in registers: twiddle and
// butterflies, then the last stage stores to dst, any other stage exchanges
// through LDS and continues with stage s + 1.
template <class PL, int s, bool INV, Sync SY, typename C, typename TW, typename Dst, typename Lds>
__device__ __forceinline__ void fft_stages(C* v, int t, const TW* __restrict__ tw, Dst dst, Lds lds) {
    constexpr int R = PL::radix(s), NS = plan_ns<PL>(s);
    stage_compute<PL, R, NS, INV>(v, t, tw);
    if constexpr (s == PL::S - 1) {
        stage_store<PL, R, NS>(v, t, dst);
    } else {
        stage_store<PL, R, NS>(v, t, [&](int e, C x) { lds.set(e, x); });
        line_sync<SY>();
        stage_load<PL, PL::radix(s + 1)>(v, t, [&](int e) { return lds.get(e); });
        line_sync<SY>();
        fft_stages<PL, s + 1, INV, SY>(v, t, tw, dst, lds);
    }
}

// Whole transform from stage-0 inputs already in registers (v, loaded by
// stage_load<PL, radix(0)>).  dst is the element accessor of the last store;
// lds.get(e) / lds.set(e, v) address this thread's line in LDS.  Every thread
// of the block (SY = BLOCK) or of the wave (SY = WAVE) must call this.
template <class PL, bool INV, Sync SY = Sync::BLOCK, typename C, typename TW, typename Dst, typename Lds>
__device__ __forceinline__ void fft_line_regs(C* v, int t, const TW* __restrict__ tw, Dst dst, Lds lds) {
    static_assert(plan_ok<PL>(), "inconsistent length plan");
    fft_stages<PL, 0, INV, SY>(v, t, tw, dst, lds);
}

// Whole transform.  src/dst are element accessors for the first load and the
// last store.  SRC_LDS: the first load reads the same LDS line that later
// stages overwrite, so a barrier separates it from the first store.
template <class PL, bool INV, bool SRC_LDS, Sync SY = Sync::BLOCK, typename TW, typename Src, typename Dst,
          typename Lds>
__device__ __forceinline__ void fft_line(int t, const TW* __restrict__ tw, Src src, Dst dst, Lds lds) {
    using C = typename tw_complex<TW>::type;
    C v[PL::E];
    stage_load<PL, PL::radix(0)>(v, t, src);
    if constexpr (SRC_LDS && PL::S > 1) line_sync<SY>();
    fft_line_regs<PL, INV, SY>(v, t, tw, dst, lds);
}

}  // namespace pipe
