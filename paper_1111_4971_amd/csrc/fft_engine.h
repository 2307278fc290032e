// fft_engine.h -- register/LDS Stockham FFT building blocks for gfx950.
//
// A length-N line is processed by P = N/E threads, each holding E complex
// values in registers.  Every stage of radix R applies E/R radix-R butterflies
// per thread (Stockham autosort: inputs j + r N/R, twiddles W_{Ns R}^{r (j mod Ns)},
// outputs (j div Ns) Ns R + (j mod Ns) + r Ns).  Between stages the line is
// exchanged through LDS.  The first stage reads its inputs straight from any
// source (global memory with zero padding, or LDS) and the last stage writes
// element j + r N/R, i.e. natural order, straight to any sink, so a transform
// costs (stages - 1) LDS round trips.
//
// Direction: forward uses W = e^{-2 pi i/N}, inverse W^{-1}; both unscaled.
// Twiddles come from a per-length stage table (stage_tw_offset) whose values
// W_N^m are computed on the host in extended precision and rounded once to the
// working precision.
#pragma once
#include <hip/hip_runtime.h>

namespace pipe {

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename R> using cplx = typename cplx_t<R>::type;

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

template <int R, bool INV, typename C> __device__ __forceinline__ void dft(C* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 16) dft16<INV>(v);
    else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------- length plans
// E = values per thread, radices applied first to last (product = N, each divides E).

template <int N> struct Plan;
#define PIPE_PLAN(N_, E_, S_, R0_, R1_, R2_, R3_)                                  \
    template <> struct Plan<N_> {                                                   \
        static constexpr int E = E_, S = S_;                                        \
        static constexpr int radix(int s) {                                         \
            return s == 0 ? R0_ : s == 1 ? R1_ : s == 2 ? R2_ : R3_;                \
        }                                                                           \
    };
PIPE_PLAN(8, 8, 1, 8, 1, 1, 1)
PIPE_PLAN(12, 12, 2, 3, 4, 1, 1)
PIPE_PLAN(16, 16, 1, 16, 1, 1, 1)
PIPE_PLAN(24, 24, 2, 3, 8, 1, 1)
PIPE_PLAN(32, 8, 2, 4, 8, 1, 1)
PIPE_PLAN(48, 12, 3, 3, 4, 4, 1)
PIPE_PLAN(64, 8, 2, 8, 8, 1, 1)
PIPE_PLAN(96, 24, 3, 3, 4, 8, 1)
PIPE_PLAN(128, 16, 2, 8, 16, 1, 1)
PIPE_PLAN(192, 24, 3, 3, 8, 8, 1)
PIPE_PLAN(256, 16, 2, 16, 16, 1, 1)
PIPE_PLAN(384, 24, 4, 3, 8, 8, 2)
PIPE_PLAN(512, 8, 3, 8, 8, 8, 1)
PIPE_PLAN(768, 24, 4, 3, 8, 8, 4)
PIPE_PLAN(1024, 16, 3, 16, 16, 4, 1)
#undef PIPE_PLAN

template <int N> __host__ __device__ constexpr int plan_ns(int s) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= Plan<N>::radix(i);
    return ns;
}

// Stage twiddle table of length N: stage s >= 1 (radix R, span NS) owns R - 1
// runs of NS values starting at stage_tw_offset<N>(NS); run r - 1 holds
// W_{NS R}^{r k} = W_N^{r k N / (NS R)} for k < NS.  The lanes of a stage
// differ in k, so they read consecutive entries (no LDS bank conflicts), where
// a natural-order table would be read at stride r N / (NS R).
template <int N> __host__ __device__ constexpr int stage_tw_offset(int ns) {
    int off = 0;
    for (int s = 1; s < Plan<N>::S; ++s) {
        if (plan_ns<N>(s) == ns) return off;
        off += (Plan<N>::radix(s) - 1) * plan_ns<N>(s);
    }
    return off;
}
template <int N> __host__ __device__ constexpr int stage_tw_size() { return stage_tw_offset<N>(0); }

// ---------------------------------------------------------------- stage pieces
// v[b*R + r] holds input r of the thread's b-th butterfly, j = t + b*P.

// Load the inputs of a stage with radix R: element index e = j + r*N/R.
template <int N, int R, typename C, typename Src>
__device__ __forceinline__ void stage_load(C* v, int t, Src src) {
    constexpr int E = Plan<N>::E, P = N / E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[b * R + r] = src(t + b * P + r * (N / R));
}

// Twiddle (for Ns > 1) and butterfly in registers.
template <int N, int R, int NS, bool INV, typename C>
__device__ __forceinline__ void stage_compute(C* v, int t, const C* __restrict__ tw) {
    constexpr int E = Plan<N>::E, P = N / E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if constexpr (NS > 1) {
            const int k = (t + b * P) % NS;
            constexpr int off = stage_tw_offset<N>(NS);
#pragma unroll
            for (int r = 1; r < R; ++r) v[b * R + r] = ctw<INV>(v[b * R + r], tw[off + (r - 1) * NS + k]);
        }
        dft<R, INV>(&v[b * R]);
    }
}

// Store the outputs of a stage: element (j div NS) NS R + (j mod NS) + r NS.
template <int N, int R, int NS, typename C, typename Dst>
__device__ __forceinline__ void stage_store(const C* v, int t, Dst dst) {
    constexpr int E = Plan<N>::E, P = N / E, NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * P;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) dst(base + r * NS, v[b * R + r]);
    }
}

// Whole transform from stage-0 inputs already in registers (v, loaded by
// stage_load<N, radix(0)>).  dst is the element accessor of the last store;
// lds.get(e) / lds.set(e, v) address this thread's line in LDS.  Every thread
// of the block must call this (it contains barriers).
template <int N, bool INV, typename C, typename Dst, typename Lds>
__device__ __forceinline__ void fft_line_regs(C* v, int t, const C* __restrict__ tw, Dst dst, Lds lds) {
    constexpr int S = Plan<N>::S;
    constexpr int R0 = Plan<N>::radix(0);
    stage_compute<N, R0, 1, INV>(v, t, tw);
    if constexpr (S == 1) {
        stage_store<N, R0, plan_ns<N>(0)>(v, t, dst);
    } else {
        stage_store<N, R0, 1>(v, t, [&](int e, C x) { lds.set(e, x); });
        __syncthreads();
        constexpr int R1 = Plan<N>::radix(1);
        stage_load<N, R1>(v, t, [&](int e) { return lds.get(e); });
        __syncthreads();
        stage_compute<N, R1, plan_ns<N>(1), INV>(v, t, tw);
        if constexpr (S == 2) {
            stage_store<N, R1, plan_ns<N>(1)>(v, t, dst);
        } else {
            stage_store<N, R1, plan_ns<N>(1)>(v, t, [&](int e, C x) { lds.set(e, x); });
            __syncthreads();
            constexpr int R2 = Plan<N>::radix(2);
            stage_load<N, R2>(v, t, [&](int e) { return lds.get(e); });
            __syncthreads();
            stage_compute<N, R2, plan_ns<N>(2), INV>(v, t, tw);
            if constexpr (S == 3) {
                stage_store<N, R2, plan_ns<N>(2)>(v, t, dst);
            } else {
                stage_store<N, R2, plan_ns<N>(2)>(v, t, [&](int e, C x) { lds.set(e, x); });
                __syncthreads();
                constexpr int R3 = Plan<N>::radix(3);
                stage_load<N, R3>(v, t, [&](int e) { return lds.get(e); });
                __syncthreads();
                stage_compute<N, R3, plan_ns<N>(3), INV>(v, t, tw);
                stage_store<N, R3, plan_ns<N>(3)>(v, t, dst);
            }
        }
    }
}

// Whole transform.  src/dst are element accessors for the first load and the
// last store.  SRC_LDS: the first load reads the same LDS line that later
// stages overwrite, so a barrier separates it from the first store.
template <int N, bool INV, bool SRC_LDS, typename C, typename Src, typename Dst, typename Lds>
__device__ __forceinline__ void fft_line(int t, const C* __restrict__ tw, Src src, Dst dst, Lds lds) {
    C v[Plan<N>::E];
    stage_load<N, Plan<N>::radix(0)>(v, t, src);
    if constexpr (SRC_LDS && Plan<N>::S > 1) __syncthreads();
    fft_line_regs<N, INV>(v, t, tw, dst, lds);
}

}  // namespace pipe
