// xprod.hip -- P3 of a solve: x forward transform, the mixed spectral product
// of the four terms of Eq. 10 on each orbit, x inverse transform (the fused
// x pass), and its launcher.  See passes.hip for the pass sequence and the
// data layout.
#include "pass_common.h"

// Compiled as one unit (PIPE_TU undefined) or as two: PIPE_TU = 1 (FP32 and
// the precision-independent functions), PIPE_TU = 2 (FP64).
#if !defined(PIPE_TU) || PIPE_TU == 1
#define PIPE_TU_FP32 1
#endif
#if !defined(PIPE_TU) || PIPE_TU == 2
#define PIPE_TU_FP64 1
#endif

namespace pipe {

template <typename real> using C_of = cplx<real>;

// Length plan of the fused x pass: the narrow variant where the default plan
// holds more than 16 values per thread (8 in FP64): more threads on the same
// LDS tile and fewer registers per thread.
template <typename real, int N> constexpr int xprod_V() { return narrow_variant<N>(sizeof(real) == 8 ? 8 : 16); }

// Waves per SIMD the register allocation must allow (1: no constraint).  The
// FP32 length-512 pass needs 66 registers left alone, which fits one
// 1024-thread block per CU although the LDS holds two; at 64 registers two fit
// (measured: 1049 -> 913 us at 256x256x1024, no spills at T = 8).
template <typename real, int N> constexpr int xprod_waves() { return (sizeof(real) == 4 && N == 512) ? 8 : 1; }

// P3: for one ky pair (ky, ly-ky) and T consecutive kz: forward x transform of
// the nx nonzero rows, the mixed product on each orbit {+-kx} x {+-ky} (see
// orbit_product), inverse x transform, rows i < nx written back in place.  The
// data is the ky-major (ly, nx, lz/2) array, so a line's rows are lz/2 apart.  The
// spectra are stored tile-blocked (see xprod_tile); the kz = lz/2 values sit in
// `nyq`.  NV = 9: the four terms; NV = 1: T_cc alone (free space), where the
// product is a real scaling and its own adjoint.  V selects the length plan
// (Plan<N, V>: the variant with fewer values per thread gives FP64 more
// threads for the same LDS tile).
template <typename real, int N, int V, int T, bool ADJ, int NV, bool NTS>
__global__ __launch_bounds__(2 * (N / Plan<N, V>::E) * T) __attribute__((amdgpu_waves_per_eu(xprod_waves<real, N>())))
void xprod_kernel(cplx<real>* data, int nx, int ly, int nh, long xs, const real* __restrict__ table,
                  const real* __restrict__ nyq, const twid<real>* __restrict__ tw,
                  const GroupArgs* __restrict__ group, int shared_table) {
    using C = cplx<real>;
    using PL = Plan<N, V>;
    // Logical order of the (kz tile, ky) items: neighbouring kz tiles share
    // 128-byte lines when T complex values are narrower, so consecutive items
    // run back to back on one XCD.  When the members of a grouped launch share
    // one spectra table (one plan, many charges), the member index goes
    // fastest, so all members of an item read its spectra tile from L2 after
    // the first; otherwise each member's items stay together.
    const unsigned ntile = gridDim.x, nmem = gridDim.z, nitem = ntile * gridDim.y;
    unsigned member, item;
    if (shared_table) {
        const unsigned lid = xcd_remap(blockIdx.x + ntile * (blockIdx.y + gridDim.y * blockIdx.z), nitem * nmem);
        member = lid % nmem;
        item = lid / nmem;
    } else {
        member = blockIdx.z;
        item = xcd_remap(blockIdx.x + ntile * blockIdx.y, nitem);
    }
    if (group) {
        data = (C*)group[member].out;
        table = (const real*)group[member].table;
        nyq = (const real*)group[member].nyq;
    }
    constexpr int P = N / PL::E, NT = 2 * P * T;
    // Orbits kx = 0 .. NKX - 1 (NKX = N/2 + 1 table entries).  For even N the
    // Nyquist orbit kx = N/2 would add a whole register set of spectra per
    // thread for T items; when the block has at least NV T threads its values
    // are loaded one per thread and staged through LDS instead (NYQ_LDS), and
    // the register loop covers the NO = N/2 other orbits.
    constexpr int NKX = N / 2 + 1;
    constexpr bool NYQ_LDS = (N % 2 == 0) && NT >= NV * T;
    constexpr int NO = NYQ_LDS ? N / 2 : NKX;
    __shared__ C lds[2 * N * T];
    __shared__ twid<real> s_tw[N];
    __shared__ real s_nyo[NYQ_LDS ? NV * T : 1];
    tw = stage_twiddles(s_tw, tw, stage_tw_size<PL>());
    const int c = threadIdx.x % T, t = (threadIdx.x / T) % P, l = threadIdx.x / (T * P);
    const int tile = (int)(item % ntile);
    const int ky = (int)(item / ntile);
    const int kyl = l == 0 ? ky : (ly - ky) % ly;
    const bool self = (ky == 0) || (2 * ky == ly);
    const long kz = (long)tile * T + c;
    const bool active = kz < nh;
    // xs: row (x) stride of the ky-major array
    const gptr<C> line = to_global(data) + (active ? (long)kyl * nx * xs + kz : 0);
    LdsCol<C, T> view{lds + l * N * T + c};

    const int kyo = ky;
    const int ntiles = (nh + T - 1) / T;
    const gptr<const real> tblock = to_global(table) + ((long)kyo * ntiles + tile) * NKX * NV * T;
    auto load = [](gptr<const real> e, int stride) -> Orbit<real> {
        if constexpr (NV == 9) return load_orbit(e, stride);
        Orbit<real> o{};
        o.cc = e[0];
        return o;
    };
    auto product = [](const Orbit<real>& ob, const C* rin, C* pout) {
        if constexpr (NV == 9) {
            orbit_product<ADJ>(ob, rin, pout);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) pout[q] = cscale(rin[q], ob.cc);
        }
    };
    // The spectra of this thread's items w = threadIdx.x + it NT are loaded
    // together with the block's rows, before the forward transform, so all of
    // the block's global reads are in flight at once.  Issue order (measured):
    // rows first in single precision, spectra first in double.
    constexpr int IT = (NO * T + NT - 1) / NT;
    Orbit<real> obs[IT];
    real nyo = 0;
    auto load_spectra = [&] {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int w = threadIdx.x + it * NT;
            if (w < NO * T) obs[it] = load(tblock + (long)(w / T) * NV * T + w % T, T);
        }
        if constexpr (NYQ_LDS) {
            if (threadIdx.x < NV * T) nyo = tblock[(long)(N / 2) * NV * T + threadIdx.x];
        }
    };
    C v0[PL::E];
    auto load_rows = [&] {
        stage_load<PL, PL::radix(0)>(v0, t, [&](int e) -> C {
            if (active && e < nx) return line[e * xs];
            return cmake<C>(0, 0);
        });
    };
    if constexpr (sizeof(real) == 8) {
        load_spectra();
        load_rows();
    } else {
        load_rows();
        load_spectra();
    }
    fft_line_regs<PL, false>(v0, t, tw, [&](int e, C v) { view.set(e, v); }, view);
    if constexpr (NYQ_LDS) {
        if (threadIdx.x < NV * T) s_nyo[threadIdx.x] = nyo;
    }
    __syncthreads();

    // the product of orbit o, kz column cc (in place in the two LDS lines)
    auto orbit_item = [&](int o, int cc, const Orbit<real>& ob) {
        const long kzz = (long)tile * T + cc;
        if (kzz >= nh) return;
        const int on = (N - o) % N;
        C* L0 = lds + cc;
        C* L1 = lds + N * T + cc;
        C r[4] = {L0[o * T], L0[on * T], L1[o * T], L1[on * T]};
        C p[4];
        if (kzz != 0) {
            product(ob, r, p);
        } else {
            // slot 0 carries A + iB, A at kz = 0, B at kz = lz/2 (both Hermitian in (kx,ky)):
            // A(k) = (P(k) + conj P(-k))/2, B(k) = (P(k) - conj P(-k))/(2i); -point of q is 3-q.
            C ra[4], rb[4], pa[4], pb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const C pm = cconj(r[3 - q]);
                const C sm = cadd(r[q], pm), d = csub(r[q], pm);
                ra[q] = cscale(sm, (real)0.5);
                rb[q] = cscale(cmake<C>(d.y, -d.x), (real)0.5);
            }
            const Orbit<real> obn = load(to_global(nyq) + ((long)kyo * NKX + o) * NV, 1);
            product(ob, ra, pa);
            product(obn, rb, pb);
#pragma unroll
            for (int q = 0; q < 4; ++q) p[q] = cmake<C>(pa[q].x - pb[q].y, pa[q].y + pb[q].x);
        }
        L0[o * T] = p[0];
        L0[on * T] = p[1];
        L1[o * T] = p[2];
        L1[on * T] = p[3];
    };
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int w = threadIdx.x + it * NT;
        if (w >= NO * T) break;
        orbit_item(w / T, w % T, obs[it]);
    }
    if constexpr (NYQ_LDS) {
        // the Nyquist orbit: T items, one per thread of the first T
        if (threadIdx.x < T) {
            Orbit<real> ob;
            if constexpr (NV == 9) {
                ob = load_orbit_lds(s_nyo + threadIdx.x, T);
            } else {
                ob = Orbit<real>{};
                ob.cc = s_nyo[threadIdx.x];
            }
            orbit_item(N / 2, threadIdx.x, ob);
        }
    }
    __syncthreads();

    fft_line<PL, true, true>(
        t, tw, [&](int e) -> C { return view.get(e); },
        [&](int e, C v) {
            if (active && e < nx && !(l == 1 && self)) out_store<NTS>(line + e * xs, v);
        },
        view);
}

// kz tile of the fused x pass: 2 lines x lx x T complex values in LDS.
template <typename real, int N> constexpr int xprod_T() {
    constexpr int bytes = sizeof(real) * 2;
    constexpr int P = N / Plan<N, xprod_V<real, N>()>::E;
    int t = PIPE_XPROD_TMAX;
    while (t > 1 && (2 * N * t * bytes > PIPE_LDS_CAP || 2 * P * t > 1024)) t /= 2;
    return t;
}

#if PIPE_TU_FP32
int xprod_tile(int lx, int real_bytes) {
    switch (lx) {
#define X(N_) \
    case N_: return real_bytes == 8 ? xprod_T<double, N_>() : xprod_T<float, N_>();
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return 0;
}
#endif

// The fused pass is compiled for two kz tiles per length: the widest T (above)
// and T/2 (when T > 1); a plan's schedule picks one.
template <typename real, int N, int T, int V, bool NTS>
static hipError_t launch_xprod_nt(bool adjoint, C_of<real>* data, int nx, int ly, int nh, long pitch,
                                  const real* table, const real* nyq, const twid<real>* tw, hipStream_t s,
                                  const GroupArgs* group, int ngroup, bool shared_table, int nval) {
    constexpr int P = N / Plan<N, V>::E;
    dim3 grid((unsigned)((nh + T - 1) / T), (unsigned)(ly / 2 + 1), (unsigned)ngroup);
    if (nval == 1)
        hipLaunchKernelGGL((xprod_kernel<real, N, V, T, false, 1, NTS>), grid, dim3(2 * P * T), 0, s, data, nx, ly,
                           nh, pitch, table, nyq, tw, group, (int)shared_table);
    else if (adjoint)
        hipLaunchKernelGGL((xprod_kernel<real, N, V, T, true, 9, NTS>), grid, dim3(2 * P * T), 0, s, data, nx, ly,
                           nh, pitch, table, nyq, tw, group, (int)shared_table);
    else
        hipLaunchKernelGGL((xprod_kernel<real, N, V, T, false, 9, NTS>), grid, dim3(2 * P * T), 0, s, data, nx, ly,
                           nh, pitch, table, nyq, tw, group, (int)shared_table);
    return hipGetLastError();
}
template <typename real, int N, int T, int V>
static hipError_t launch_xprod_t(bool adjoint, bool nt_store, C_of<real>* data, int nx, int ly, int nh, long pitch,
                                 const real* table, const real* nyq, const twid<real>* tw, hipStream_t s,
                                 const GroupArgs* group, int ngroup, bool shared_table, int nval) {
    // non-temporal row stores are compiled for FP64 only (they slowed every FP32 pass measured)
    if constexpr (sizeof(real) == 8) {
        if (nt_store)
            return launch_xprod_nt<real, N, T, V, true>(adjoint, data, nx, ly, nh, pitch, table, nyq, tw, s, group,
                                                        ngroup, shared_table, nval);
    }
    return launch_xprod_nt<real, N, T, V, false>(adjoint, data, nx, ly, nh, pitch, table, nyq, tw, s, group,
                                                 ngroup, shared_table, nval);
}

template <typename real>
hipError_t launch_xprod(int lx, bool adjoint, void* data, int nx, int ly, int nh, long pitch, int tile,
                        bool nt_store, const real* table, const real* nyq, const TwiddleBank& twb, hipStream_t s,
                        const GroupArgs* group, int ngroup, bool shared_table, int nval) {
    using C = cplx<real>;
    if ((nval != 9 && nval != 1) || pitch < nh) return hipErrorInvalidValue;
    switch (lx) {
#define X(N_)                                                                                          \
    case N_: {                                                                                         \
        constexpr int V = xprod_V<real, N_>(), T = xprod_T<real, N_>();                                \
        const twid<real>* tw = twb.stage<twid<real>>(N_, V);                                                             \
        if (!tw) return hipErrorInvalidValue;                                                          \
        if (tile == T)                                                                                 \
            return launch_xprod_t<real, N_, T, V>(adjoint, nt_store, (C*)data, nx, ly, nh, pitch, table, nyq, tw, s, \
                                                  group, ngroup, shared_table, nval);                  \
        if constexpr (T > 1) {                                                                         \
            if (tile == T / 2)                                                                         \
                return launch_xprod_t<real, N_, (T > 1 ? T / 2 : 1), V>(adjoint, nt_store, (C*)data, nx, ly, nh, pitch, \
                                                                        table, nyq, tw, s, group, ngroup, \
                                                                        shared_table, nval);           \
        }                                                                                              \
        return hipErrorInvalidValue;                                                                   \
    }
        PIPE_FOR_EACH_N(X)
#undef X
    }
    return hipErrorInvalidValue;
}

#if PIPE_TU_FP32
template hipError_t launch_xprod<float>(int, bool, void*, int, int, int, long, int, bool, const float*, const float*,
                                        const TwiddleBank&, hipStream_t, const GroupArgs*, int, bool, int);
#endif
#if PIPE_TU_FP64
template hipError_t launch_xprod<double>(int, bool, void*, int, int, int, long, int, bool, const double*,
                                         const double*, const TwiddleBank&, hipStream_t, const GroupArgs*, int, bool,
                                         int);
#endif

}  // namespace pipe
