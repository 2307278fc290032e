// pipe_internal.h -- declarations shared by the host API and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace pipe {

// Supported complex FFT lengths: every 2^p 3^q in [8, 1024] (the plans are in
// fft_engine.h).  The twiddle bank also holds natural tables of length 2N for
// the real-to-complex post-processing of z lines of length 2N.
constexpr int kFftLengths[] = {8,   9,   12,  16,  18,  24,  27,  32,  36,  48,  54,  64,
                               72,  81,  96,  108, 128, 144, 162, 192, 216, 243, 256, 288,
                               324, 384, 432, 486, 512, 576, 648, 729, 768, 864, 972, 1024};
constexpr int kNumFft = sizeof(kFftLengths) / sizeof(int);
// Lengths the banded x pass supports (N and E multiples of 4).
constexpr int kBandLengths[] = {8,   12,  16,  24,  32,  36,  48,  64,  72,  96,  108, 128,
                                144, 192, 216, 256, 288, 384, 432, 512, 576, 768, 864, 1024};

inline bool fft_length_ok(int n) {
    for (int v : kFftLengths) if (v == n) return true;
    return false;
}
inline bool band_length_ok(int n) {
    for (int v : kBandLengths) if (v == n) return true;
    return false;
}

// Plan variants beyond each length's default plan (fft_engine.h, Plan<N, V>);
// must list the same pairs as PIPE_FOR_EACH_VARIANT.
struct PlanVariant {
    int n, v;
};
constexpr PlanVariant kPlanVariants[] = {{16, 2},  {24, 2},  {54, 2},  {72, 2},  {96, 2},  {128, 2}, {162, 2},
                                         {192, 2}, {216, 2}, {256, 2}, {288, 2}, {324, 2}, {384, 2}, {432, 2},
                                         {486, 2}, {576, 2}, {648, 2}, {768, 2}, {864, 2}, {972, 2}, {1024, 2}};
constexpr int kNumVariants = sizeof(kPlanVariants) / sizeof(PlanVariant);

// Per-device twiddle bank: for every FFT length N the natural tables
// tw[m] = exp(-2 pi i m / L), m < L, for L = N and L = 2N (get), and the stage
// table of every plan of the transform engine (stage; see stage_tw_offset),
// all in one allocation per precision.
struct TwiddleBank {
    void* d64 = nullptr;   // double2
    void* d32 = nullptr;   // float2
    void* d32c = nullptr;  // TwPair32: the same entries as FP32 (hi, lo) pairs
    size_t offset[kNumFft] = {};        // natural table of length N
    size_t offset2[kNumFft] = {};       // natural table of length 2N
    size_t soffset[kNumFft] = {};       // stage table of the default plan of length N
    size_t voffset[kNumVariants] = {};  // stage tables of the variant plans
    size_t total = 0;
    template <typename C> const C* get(int n) const;
    template <typename C> const C* stage(int n, int variant = 0) const;
};

// Stage table of the plan (n, variant): writes the exponent m of each entry
// (the entry is W_n^m) to m_out (at least n slots) and returns the entry
// count, or -1 if there is no such plan.
int fft_stage_exponents(int n, int variant, int* m_out);

// Per-member pointers of a grouped launch: blockIdx.z selects the member and its
// entry replaces the launch's own data pointers (in/out; table/nyq for the x
// pass; scale for the z inverse).  All members share the launch's sizes.
struct GroupArgs {
    const void* in;
    void* out;
    const void* table;
    const void* nyq;
    double scale;
};

// Kernel launchers (passes.hip).  All return hipSuccess or the launch error.
// group (device array of ngroup entries) may be null for a single solve.
template <typename real>
// zcap: at most this many blocks in the persistent grid (over all members).
hipError_t launch_z_r2c(int nh, const real* in, long in_pitch, int n_in, void* out, long out_pitch,
                        long nlines, const TwiddleBank& tw, hipStream_t s,
                        const GroupArgs* group = nullptr, int ngroup = 1, bool aligned = true, int zcap = 2048);
template <typename real>
hipError_t launch_z_c2r(int nh, const void* in, long in_pitch, real* out, long out_pitch, int n_out,
                        long nlines, real scale, const TwiddleBank& tw, hipStream_t s,
                        const GroupArgs* group = nullptr, int ngroup = 1, bool aligned = true, int zcap = 2048);
template <typename real>
hipError_t launch_strided(int n, bool inverse, const void* in, void* out, int n_in, int n_out,
                          long in_es, long out_es, long ncols, long in_ss, long out_ss, long nslabs,
                          const TwiddleBank& tw, hipStream_t s, const GroupArgs* group = nullptr,
                          int ngroup = 1);
template <typename real>
// shared_table (grouped launches whose members all use one plan's spectra):
// members of one (kz tile, ky) item run back to back, so the tile is read once.
// nval: values per orbit in the table, 9 (four terms) or 1 (T_cc only: free space).
// pitch: row stride of the (ly, nx, pitch) array, >= nh; tile: the kz tile,
// xprod_tile(lx, .) or half of it (the table must be laid out for that tile).
// nt_store: write the output rows with non-temporal stores.
hipError_t launch_xprod(int lx, bool adjoint, void* data, int nx, int ly, int nh, long pitch, int tile,
                        bool nt_store, const real* table, const real* nyq, const TwiddleBank& tw, hipStream_t s,
                        const GroupArgs* group = nullptr, int ngroup = 1, bool shared_table = false,
                        int nval = 9);

// Row pitch (complex values) of the y-transformed array A2 = (ly, nx, pitch):
// lz/2 plus pad unused slots per row (a plan's schedule sets pad).
inline long a2_pitch(int nh, int pad) { return (long)nh + pad; }

// kz tile width of the fused x pass for padded length lx (0 if unsupported).
// The Green spectra are stored tile-blocked to match: for orbit row kyo, kz tile
// t, orbit kx = o, plane p < nval (9, or 1 for free space) and column c < T the
// value sits at
//   (((kyo * ntiles + t) * (lx/2 + 1) + o) * nval + p) * T + c,   kz = t * T + c,
// so one block of the fused pass reads one contiguous run.  The kz = lz/2
// values sit at (kyo * (lx/2 + 1) + o) * nval + p.
int xprod_tile(int lx, int real_bytes);

// Green evaluation (green.hip).
hipError_t launch_cos_table(double* out, int nconv, int ncorr, int m, double s, double off, hipStream_t st);
hipError_t launch_modes(double* d, int mx, int my, int rz, double a, double b, double hz, int igf,
                        double norm, hipStream_t st);
hipError_t launch_gemm_f64(const double* A, const double* B, double* C, int M, int N, int K,
                           long lda, long ldb, long ldc, long sA, long sB, long sC, int batch,
                           hipStream_t st);
// Green arrangement of one term (Appendix A.3 / A.9 slots) into xi[lx][ly][lz];
// z_identity (lz == nz): slot s holds plane distance s (banded spectra).
hipError_t launch_arrange(double* xi, const double* rbar, int nx, int ny, int nz, int lx, int ly,
                          int lz, int xcorr, int ycorr, hipStream_t st, bool z_identity = false);
// Free-space (Eq. 5) Green array into xi[lx][ly][lz]: 1/r at the convolution
// slots, g0 at zero distance.
hipError_t launch_free_arrange(double* xi, int nx, int ny, int nz, int lx, int ly, int lz, double hx, double hy,
                              double hz, double g0, hipStream_t st);
hipError_t launch_compress(const void* spec, void* table, void* nyq, int real_bytes, int term,
                           int lx, int ly, int nh, int tile, hipStream_t st, int nval = 9);
hipError_t launch_untile(const void* table, const void* nyq, void* out, int real_bytes, int lx, int ly, int nh,
                         int tile, hipStream_t st, int nval = 9);

// Neighbouring-plane (banded z) path (band.hip).
// y pass between real planes (rho, phi: (slab, e, z) at slab r_ss + e r_es + z,
// z < nz) and packed complex columns p < ceil(nz/2) holding planes 2p + i (2p+1)
// ((slab, e, p) at slab c_ss + e c_es + p).  Forward reads rows e < n_in and
// writes all n rows; inverse reads n rows, writes rows e < n_out times scale.
template <typename real>
hipError_t launch_strided_pair(int n, bool inverse, const void* in, void* out, int n_in, int n_out, long r_es,
                               long c_es, long r_ss, long c_ss, long nslabs, int nz, real scale,
                               const TwiddleBank& tw, hipStream_t s);
// y pass with real input (forward) or real output (inverse, times scale), one
// plane per column; arguments as launch_strided.
template <typename real>
hipError_t launch_strided_real(int n, bool inverse, const void* in, void* out, int n_in, int n_out, long in_es,
                               long out_es, long ncols, long in_ss, long out_ss, long nslabs, real scale,
                               const TwiddleBank& tw, hipStream_t s);
// x forward, split of the packed plane pairs, sum over plane distances
// |d| <= nb of the orbit products, packing, x inverse: in, out (ly, nx,
// ceil(nz/2)) packed complex, ky-major (distinct buffers); table: the banded
// coefficients (launch_band_coefficients).  The output carries a factor 2.
// The coefficient matrices are symmetric, so the adjoint is the same launch.
// For nb >= 1 two x-pass kernels exist: single_window (the whole input window of
// a block is one transform chunk, available when band_small_columns_for > 0) and
// the chunked one; the plan times both and keeps the faster.
template <typename real>
// Row pad of the banded plans' packed arrays, in complex values: rows
// ceil(nz/2) + PIPE_BAND_PAD apart instead of a power-of-two stride (measured
// at 256x256x1024: the y inverse pass 448 -> 336 us in FP64, 180 -> 167 us in
// FP32; the x pass 4 % slower in FP64; neutral at 128x128x256).
#ifndef PIPE_BAND_PAD
#define PIPE_BAND_PAD 16
#endif
// tile0 (nb = 0 only): the N = 0 kernel's packed-column tile, band0_tile(lx, .) or half of it.
// pitch: row (x) stride of the packed arrays in complex values, >= ceil(nz/2).
hipError_t launch_xband(int lx, const void* in, void* out, int nx, int ly, int nz, long pitch, int nb,
                        const real* table, const TwiddleBank& tw, hipStream_t s, bool single_window, int tile0 = 0);
// Widest packed-column tile of the N = 0 banded x pass (0 if lx unsupported).
int band0_tile(int lx, int real_bytes);
// Output columns per block of the single-window banded x pass, 0 if not available.
int band_small_columns_for(int lx, int real_bytes, int nb);
// Packed columns per block of the banded x pass (0 if lx unsupported).
int band_tile(int lx, int real_bytes);
// One term's 2-D spectra S[lx][ly][D] (FP64 complex) into the nine-value
// FP64 staging table tmp ((ly/2+1) D 9 (lx/2+1) values).
hipError_t launch_compress_band(const void* spec, double* tmp, int term, int lx, int ly, int D, hipStream_t st);
// The banded coefficient table (10 values per orbit and distance, plan
// precision) from the staging table once all four terms are in.
hipError_t launch_band_coefficients(const double* tmp, void* table, int real_bytes, int lx, int ly, int D,
                                    hipStream_t st);

// Batched contiguous complex lines (fft3d.hip): nlines lines of length n at
// in + l n, out + l n (in == out allowed), forward (W^{jk}) or inverse (W^{-jk}),
// unscaled.
template <typename real>
hipError_t launch_lines(int n, bool inverse, const void* in, void* out, long nlines, const TwiddleBank& tw,
                        hipStream_t s);

}  // namespace pipe
