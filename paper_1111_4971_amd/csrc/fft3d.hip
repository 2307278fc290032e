// fft3d.hip -- batched complex FFTs along contiguous lines, the last axis of
// the public mixed-direction 3-D transform (pipe_fft3d).  Each line of length N
// is handled by P = N/E threads of the Stockham engine, several lines per block,
// each line padded in LDS (one slot every 16) against bank conflicts.
#include "pass_common.h"

namespace pipe {

template <typename real, int N> constexpr int lines_per_block() {
    int l = ce_max(1, 256 / (N / Plan<N>::E));
    while (l > 1 && l * (N + N / 16 + 1) * 2 * (int)sizeof(real) > PIPE_LDS_CAP) l /= 2;
    return l;
}

template <typename real, int N, bool INV>
__global__ __launch_bounds__((lines_per_block<real, N>() * (N / Plan<N>::E)))
void lines_kernel(const cplx<real>* in, cplx<real>* out, long nlines, const twid<real>* __restrict__ tw) {
    using C = cplx<real>;
    constexpr int P = N / Plan<N>::E, LPB = lines_per_block<real, N>(), LS = N + N / 16 + 1;
    __shared__ C lds[LPB * LS];
    __shared__ twid<real> s_tw[N];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<Plan<N>>());
    const int t = threadIdx.x % P, li = threadIdx.x / P;
    const long line = (long)blockIdx.x * LPB + li;
    const bool active = line < nlines;
    const C* src = in + (active ? line * N : 0);
    C* dst = out + (active ? line * N : 0);
    LdsLine<C> view{lds + li * LS};
    // single-stage plans (P = 1) keep a line in one thread, so in == out is safe
    fft_line<Plan<N>, INV, false>(
        t, tw, [&](int e) -> C { return active ? src[e] : cmake<C>(0, 0); },
        [&](int e, C v) {
            if (active) dst[e] = v;
        },
        view);
}

template <typename real>
hipError_t launch_lines(int n, bool inverse, const void* in, void* out, long nlines, const TwiddleBank& twb,
                        hipStream_t s) {
    using C = cplx<real>;
    const twid<real>* tw = twb.stage<twid<real>>(n);
    if (!tw || nlines <= 0) return hipErrorInvalidValue;
    switch (n) {
#define X(N_)                                                                                        \
    case N_: {                                                                                       \
        constexpr int LPB = lines_per_block<real, N_>(), P = N_ / Plan<N_>::E;                       \
        dim3 grid((unsigned)((nlines + LPB - 1) / LPB));                                             \
        if (inverse)                                                                                 \
            hipLaunchKernelGGL((lines_kernel<real, N_, true>), grid, dim3(LPB * P), 0, s,            \
                               (const C*)in, (C*)out, nlines, tw);                                   \
        else                                                                                         \
            hipLaunchKernelGGL((lines_kernel<real, N_, false>), grid, dim3(LPB * P), 0, s,           \
                               (const C*)in, (C*)out, nlines, tw);                                   \
        return hipGetLastError();                                                                    \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

#if !defined(PIPE_TU) || PIPE_TU == 1
template hipError_t launch_lines<float>(int, bool, const void*, void*, long, const TwiddleBank&, hipStream_t);
#endif
#if !defined(PIPE_TU) || PIPE_TU == 2
template hipError_t launch_lines<double>(int, bool, const void*, void*, long, const TwiddleBank&, hipStream_t);
#endif

}  // namespace pipe
