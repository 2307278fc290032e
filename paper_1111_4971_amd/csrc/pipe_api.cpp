// pipe_api.cpp -- host side of libpipe: argument validation, plan build
// (Green evaluation, arrangement, spectra), solve orchestration, batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pipe_poisson.h"
#include "pipe_internal.h"

using namespace pipe;

// ---------------------------------------------------------------- errors

namespace {

thread_local std::string g_err;

pipe_status_t fail(pipe_status_t st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

pipe_status_t hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(PIPE_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice)
        return fail(PIPE_ERR_NO_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return fail(PIPE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool fault_inject_alloc() {
    const char* v = getenv("PIPE_FAULT_INJECT");
    return v && strcmp(v, "alloc") == 0;
}

hipError_t dev_alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (fault_inject_alloc()) return hipErrorOutOfMemory;
    if (bytes == 0) bytes = 256;
    return hipMalloc(p, bytes);
}

// ---------------------------------------------------------------- device context

// Fixed device scratch of pipe_poisson_solve_noalloc: the solve's workspace
// for callers that cannot allocate.  One copy per device, alive until the
// process ends.  In host code the name is only a stand-in for the symbol: its
// device address comes from hipGetSymbolAddress (DeviceCtx::scratch).
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceCtx {
    bool ready = false;
    TwiddleBank tw;
    void* scratch = nullptr;   // this device's address of `scratch`
};
std::mutex g_ctx_mu;
DeviceCtx g_ctx[64];

pipe_status_t device_ctx(int dev, DeviceCtx** out) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (dev < 0 || dev >= 64) return fail(PIPE_ERR_NO_DEVICE, "device index %d out of range", dev);
    DeviceCtx& c = g_ctx[dev];
    if (!c.ready) {
        // natural tables of lengths N and 2N (exponent m at offset + m), then
        // the stage tables of the FFT lengths (exponents from fft_stage_exponents)
        std::vector<int> m_of;   // exponent of every entry
        std::vector<int> n_of;   // its table length
        for (int i = 0; i < kNumFft; ++i) {
            for (int twice = 0; twice < 2; ++twice) {
                const int n = kFftLengths[i] << twice;
                (twice ? c.tw.offset2[i] : c.tw.offset[i]) = m_of.size();
                for (int m = 0; m < n; ++m) {
                    m_of.push_back(m);
                    n_of.push_back(n);
                }
            }
        }
        std::vector<int> ms(4096);
        for (int i = 0; i < kNumFft + kNumVariants; ++i) {
            const int n = i < kNumFft ? kFftLengths[i] : kPlanVariants[i - kNumFft].n;
            const int v = i < kNumFft ? 0 : kPlanVariants[i - kNumFft].v;
            (i < kNumFft ? c.tw.soffset[i] : c.tw.voffset[i - kNumFft]) = m_of.size();
            const int cnt = fft_stage_exponents(n, v, ms.data());
            if (cnt < 0) return fail(PIPE_ERR_HIP, "no stage table for plan (%d, %d)", n, v);
            for (int q = 0; q < cnt; ++q) {
                m_of.push_back(ms[q]);
                n_of.push_back(n);
            }
        }
        const size_t off = m_of.size();
        c.tw.total = off;
        std::vector<double> h64(2 * off);
        std::vector<float> h32(2 * off), h32c(4 * off);
        for (size_t k = 0; k < off; ++k) {
            // W_n^m = exp(-2 pi i m / n), evaluated in long double and rounded once;
            // the FP32 pair holds hi = the rounding and lo = the rounding of the rest
            const long double ang =
                -2.0L * 3.141592653589793238462643383279503L * (long double)m_of[k] / (long double)n_of[k];
            const long double cr = cosl(ang), ci = sinl(ang);
            h64[2 * k] = (double)cr;
            h64[2 * k + 1] = (double)ci;
            h32[2 * k] = (float)cr;
            h32[2 * k + 1] = (float)ci;
            h32c[4 * k] = h32[2 * k];
            h32c[4 * k + 1] = h32[2 * k + 1];
            h32c[4 * k + 2] = (float)(cr - (long double)h32[2 * k]);
            h32c[4 * k + 3] = (float)(ci - (long double)h32[2 * k + 1]);
        }
        void* bufs[3] = {nullptr, nullptr, nullptr};
        const std::vector<float>* srcf[2] = {&h32, &h32c};
        hipError_t e = dev_alloc(&bufs[0], h64.size() * sizeof(double));
        if (e == hipSuccess) e = dev_alloc(&bufs[1], h32.size() * sizeof(float));
        if (e == hipSuccess) e = dev_alloc(&bufs[2], h32c.size() * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(bufs[0], h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice);
        for (int i = 0; i < 2 && e == hipSuccess; ++i)
            e = hipMemcpy(bufs[1 + i], srcf[i]->data(), srcf[i]->size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            for (void* b : bufs)
                if (b) (void)hipFree(b);
            return hip_fail(e, "twiddle tables");
        }
        c.tw.d64 = bufs[0];
        c.tw.d32 = bufs[1];
        c.tw.d32c = bufs[2];
        // device address of the fixed scratch (this device is current here)
        HIP_TRY(hipGetSymbolAddress(&c.scratch, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!c.scratch) return fail(PIPE_ERR_HIP, "scratch symbol address: null");
        c.ready = true;
    }
    *out = &c;
    return PIPE_OK;
}

std::mutex g_reg_mu;
std::set<const void*> g_live;

void reg_add(const void* p) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_live.insert(p);
}
bool reg_has(const void* p) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return p && g_live.count(p);
}
bool reg_del(const void* p) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return p && g_live.erase(p) == 1;
}

int pick_length(int need) {
    for (int v : kFftLengths)
        if (v >= need) return v;
    return -1;
}

// Fraction of the HBM peak the passes of one length reached on MI355X, with
// the mesh padded exactly to that length (x and y: n = L/2 rows, nz = 256, the
// y passes and the fused x pass together; z: a 128 x 128 mesh, nz = L, both z
// passes), FP32 and FP64.  Plans with more stages and more values per thread
// (27 * 2^k, 9 * 2^k) run well below their neighbours.
struct LengthEff {
    int n;
    float xy32, xy64, z32, z64;
};
constexpr LengthEff kLengthEff[] = {
    {64, 0.155, 0.256, 0.194, 0.299},
    {72, 0.148, 0.229, 0.163, 0.237},
    {81, 0.200, 0.316, 0.197, 0.303},
    {96, 0.220, 0.340, 0.211, 0.315},
    {108, 0.240, 0.327, 0.197, 0.289},
    {128, 0.368, 0.530, 0.298, 0.393},
    {144, 0.335, 0.481, 0.223, 0.285},
    {162, 0.334, 0.476, 0.255, 0.353},
    {192, 0.460, 0.570, 0.321, 0.399},
    {216, 0.318, 0.396, 0.249, 0.334},
    {243, 0.519, 0.564, 0.312, 0.393},
    {256, 0.624, 0.646, 0.386, 0.519},
    {288, 0.434, 0.508, 0.287, 0.373},
    {324, 0.435, 0.505, 0.292, 0.367},
    {384, 0.488, 0.526, 0.356, 0.439},
    {432, 0.329, 0.409, 0.332, 0.393},
    {486, 0.380, 0.386, 0.345, 0.433},
    {512, 0.594, 0.606, 0.466, 0.541},
    {576, 0.390, 0.469, 0.340, 0.409},
    {648, 0.361, 0.441, 0.305, 0.368},
    {729, 0.434, 0.403, 0.381, 0.400},
    {768, 0.451, 0.484, 0.382, 0.479},
    {864, 0.272, 0.302, 0.310, 0.373},
    {972, 0.303, 0.291, 0.337, 0.401},
    {1024, 0.490, 0.451, 0.464, 0.528},
};

// Default padded length: among the supported lengths >= need and within 20 %
// of the smallest such length, the one with the lowest modelled pass time.
// x, y: time ~ L / eff_xy(L).  z (half = true, lengths are NH = lz/2): every
// pass scales with NH, the z passes carry about a sixth of a solve's bytes, so
// time ~ NH (1/6 / eff_z(NH) + 5/6 / 0.55).  Below length 64 (latency-bound
// meshes, not modelled) the smallest length is taken.
int pick_modelled_length(int need, bool half, bool fp64) {
    const int first = pick_length(need);
    if (first < 64) return first;
    int best = first;
    double best_cost = 0.0;
    for (const LengthEff& e : kLengthEff) {
        if (e.n < first || e.n > first + first / 5) continue;
        const double eff = half ? (fp64 ? e.z64 : e.z32) : (fp64 ? e.xy64 : e.xy32);
        const double cost = half ? e.n * (1.0 / 6.0 / eff + 5.0 / 6.0 / 0.55) : e.n / eff;
        if (best_cost == 0.0 || cost < best_cost) {
            best = e.n;
            best_cost = cost;
        }
    }
    return best;
}

int pick_band_length(int need) {
    for (int v : kBandLengths)
        if (v >= need) return v;
    return -1;
}

}  // namespace

// ---------------------------------------------------------------- plan

struct pipe_plan_s {
    int nx, ny, nz, lx, ly, lz, nh, mx, my, kind, rb;
    double hx, hy, hz, a, b;
    double x0 = 0, y0 = 0;   // mesh offset: node i at x0 + (i+1) hx, node j at y0 + (j+1) hy
    int device;
    DeviceCtx* ctx;
    void* table = nullptr;   // tile-blocked spectra, nval values per orbit (see xprod_tile)
    void* nyq = nullptr;     // kz = lz/2 values, nval per orbit (inside the table allocation)
    size_t table_elems = 0, nyq_elems = 0;
    int tile = 0;            // kz tile of the table layout (and of the fused x pass)
    int apad = 0;            // schedule: unused slots per row of the y-transformed array
    int zcap = 2048;         // schedule: block cap of the persistent z passes
    int xnt = 0;             // schedule: the x pass writes its rows with non-temporal stores
    int nval = 9;            // values per orbit: 9 (four terms), 1 (free space: T_cc only)
    int band = -1;           // banded plan: planes kept each side of the z sum (Eq. 18); -1 = 3-D plan
    double g0 = 0;           // free-space plans: G at zero separation
    bool band_single = false; // banded x pass: single-window kernel (else chunked), chosen by timing
    int band_tile0 = 0;       // banded N = 0 x pass: packed-column tile, chosen by timing
    int band_pad = PIPE_BAND_PAD;   // banded: row pitch of the packed array = ceil(nz/2) + band_pad
    int a1pad = 0;                  // row pitch of A1 = lz/2 + a1pad (set with the launch schedule)
    double band_speedup = 0;  // banded build: measured 3-D solve time / banded solve time
    double* green = nullptr; // optional copy of Rbar
    double build_ms = 0;
    double tune_ms = -1;     // autotuner: best candidate's time per solve, 0 if cached, -1 if not tuned
    size_t ws_bytes = 0;
    // event timing (pipe_plan_timing): 6 events per recorded solve
    std::vector<hipEvent_t> tev;
    int tmax = 0, tn = 0;
    // one event per stream the plan has solved on, recorded after each solve's
    // last kernel: destroy waits on these rather than on the whole device
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

long band_pitch(const pipe_plan_s* p) { return (p->nz + 1) / 2 + p->band_pad; }
long a1_pitch(const pipe_plan_s* p) { return p->nh + p->a1pad; }
// A1's row pad by rule rather than by timing (its effect, about 1 %, is below
// what a few timed solves resolve): 16 slots where lz/2 is a power of two and
// a row spans at least 8 KB, where the power-of-two stride slowed the y passes
// (256x256x1024: y forward 6 % faster padded, solve 1.0 % (FP32) and 1.7 %
// (FP64); 128x128x512 FP32, 4 KB rows: 0-0.7 % slower padded).
int a1_pad_rule(const pipe_plan_s* p) {
    const long row = (long)p->nh * 2 * p->rb;
    return ((p->nh & (p->nh - 1)) == 0 && row >= 8192) ? 16 : 0;
}

size_t plan_ws_bytes(const pipe_plan_s* p) {
    const size_t cb = 2 * (size_t)p->rb;
    if (p->band >= 0) return 2 * align256((size_t)p->nx * p->ly * band_pitch(p) * cb);   // A, B: packed pairs
    const size_t a1 = (size_t)p->nx * p->ny * a1_pitch(p) * cb;
    const size_t a2 = (size_t)p->nx * p->ly * a2_pitch(p->nh, p->apad) * cb;
    return align256(a1) + align256(a2);
}

void plan_pass_bytes(const pipe_plan_s* p, double out[5]) {
    const double rb = p->rb, cb = 2.0 * p->rb;
    const double phys = (double)p->nx * p->ny * p->nz * rb;
    const double a1 = (double)p->nx * p->ny * p->nh * cb;
    const double a2 = (double)p->nx * p->ly * p->nh * cb;
    const double orbits = (double)(p->lx / 2 + 1) * (p->ly / 2 + 1);
    const double tab = p->nval * orbits * (p->nh + 1) * rb;   // values read once per solve
    if (p->band >= 0) {
        // banded: y forward (real in), x + banded product, y inverse (real out)
        const double A = (double)p->nx * p->ly * ((p->nz + 1) / 2) * cb;
        out[0] = phys + A;
        out[1] = 2.0 * A + 10.0 * orbits * (p->band + 1) * rb;   // K0..K9 per orbit and distance
        out[2] = A + phys;
        out[3] = out[4] = 0.0;
        return;
    }
    out[0] = phys + a1;
    out[1] = a1 + a2;
    out[2] = 2.0 * a2 + tab;
    out[3] = a2 + a1;
    out[4] = a1 + phys;
}

// free_space: the Eq. 5 plan (no pipe: a, b, offsets and modes are not used).
pipe_status_t validate(int nx, int ny, int nz, double hx, double hy, double hz, double a, double b, double x0,
                       double y0, int kind, int mx, int my, int* lx, int* ly, int* lz, bool free_space = false) {
    if (nx < 1 || ny < 1 || nz < 1) return fail(PIPE_ERR_INVALID_ARG, "mesh sizes must be >= 1 (got %d,%d,%d)", nx, ny, nz);
    const double v[5] = {hx, hy, hz, free_space ? 1.0 : a, free_space ? 1.0 : b};
    for (double t : v)
        if (!(t > 0.0) || !std::isfinite(t)) return fail(PIPE_ERR_INVALID_ARG, "spacings and pipe sizes must be finite and > 0");
    if (free_space) {
        x0 = y0 = 0.0;
        a = nx * hx;
        b = ny * hy;
        mx = my = 1;
    }
    if (!(x0 >= 0.0) || !(y0 >= 0.0) || !std::isfinite(x0) || !std::isfinite(y0))
        return fail(PIPE_ERR_INVALID_ARG, "mesh offsets must be finite and >= 0");
    if (x0 + nx * hx > a * (1.0 + 1e-12))
        return fail(PIPE_ERR_INVALID_ARG, "x0 + nx*hx = %g exceeds the pipe width a = %g", x0 + nx * hx, a);
    if (y0 + ny * hy > b * (1.0 + 1e-12))
        return fail(PIPE_ERR_INVALID_ARG, "y0 + ny*hy = %g exceeds the pipe height b = %g", y0 + ny * hy, b);
    const int g = kind & 0x0f, pr = kind & ~0x0f;
    if (free_space ? g != PIPE_GREEN_FREE : (g != PIPE_GREEN_POINT && g != PIPE_GREEN_IGF_Z))
        return fail(PIPE_ERR_INVALID_ARG, g == PIPE_GREEN_FREE ? "free-space plans are made by pipe_free_plan"
                                                               : "unknown Green kind %d", g);
    if (pr != PIPE_PREC_FP64 && pr != PIPE_PREC_FP32) return fail(PIPE_ERR_INVALID_ARG, "unknown precision flag 0x%x", pr);
    if (mx < 1 || my < 1 || mx > 8192 || my > 8192) return fail(PIPE_ERR_INVALID_ARG, "mode counts must be in [1, 8192]");
    // padded lengths
    auto choose = [&](int n, int* L, bool half, const char* nm) -> pipe_status_t {
        if (*L == 0) {
            const int h = pick_modelled_length(half ? n : 2 * n, half, pr == PIPE_PREC_FP64);
            if (h < 0) return fail(PIPE_ERR_UNSUPPORTED_SIZE, "%s: no supported padded length for n = %d", nm, n);
            *L = half ? 2 * h : h;
            return PIPE_OK;
        }
        if (*L < 2 * n - 1) return fail(PIPE_ERR_INVALID_ARG, "%s: padded length %d < 2n - 1 = %d", nm, *L, 2 * n - 1);
        // z is transformed real-to-complex as lz/2 packed pairs, so lz must be even
        if (half && *L % 2) return fail(PIPE_ERR_UNSUPPORTED_SIZE, "%s: padded length %d must be even", nm, *L);
        if (!fft_length_ok(half ? *L / 2 : *L))
            return fail(PIPE_ERR_UNSUPPORTED_SIZE, "%s: padded length %d is not of the form 2^p 3^q in [%d, %d]", nm,
                        *L, half ? 16 : 8, half ? 2048 : 1024);
        return PIPE_OK;
    };
    pipe_status_t st;
    if ((st = choose(nx, lx, false, "lx")) != PIPE_OK) return st;
    if ((st = choose(ny, ly, false, "ly")) != PIPE_OK) return st;
    if (lz && (st = choose(nz, lz, true, "lz")) != PIPE_OK) return st;   // lz null: no z transform
    return PIPE_OK;
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    hipError_t get(void** p, size_t bytes) {
        hipError_t e = dev_alloc(p, bytes);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

// Eq. 5: one term, G = 1/r arranged straight into the padded array.
pipe_status_t build_free_spectra(pipe_plan_s* p, hipStream_t st) {
    const int lx = p->lx, ly = p->ly, lz = p->lz, nh = p->nh;
    Scratch s;
    double* buf;
    HIP_TRY(s.get((void**)&buf, sizeof(double) * (size_t)lx * ly * lz), "allocation (spectrum buffer)");
    HIP_TRY(launch_free_arrange(buf, p->nx, p->ny, p->nz, lx, ly, lz, p->hx, p->hy, p->hz, p->g0, st),
            "Green arrangement");
    HIP_TRY(launch_z_r2c<double>(nh, buf, lz, lz, buf, nh, (long)lx * ly, p->ctx->tw, st), "spectra z transform");
    HIP_TRY(launch_strided<double>(ly, false, buf, buf, ly, ly, nh, nh, nh, (long)ly * nh, (long)ly * nh, lx,
                                   p->ctx->tw, st),
            "spectra y transform");
    HIP_TRY(launch_strided<double>(lx, false, buf, buf, lx, lx, (long)ly * nh, (long)ly * nh, (long)ly * nh, 0, 0, 1,
                                   p->ctx->tw, st),
            "spectra x transform");
    // only T_cc, stored alone (one value per orbit)
    HIP_TRY(launch_compress(buf, p->table, p->nyq, p->rb, 0, lx, ly, nh, p->tile, st, p->nval),
            "spectra compression");
    HIP_TRY(hipStreamSynchronize(st), "plan build");
    return PIPE_OK;
}

pipe_status_t build_spectra(pipe_plan_s* p, hipStream_t st, bool keep_green) {
    if ((p->kind & 0x0f) == PIPE_GREEN_FREE) return build_free_spectra(p, st);
    // Rbar rows: nx differences then 2nx - 1 sums along x, likewise along y
    const int px = 3 * p->nx - 1, qy = 3 * p->ny - 1, rz = p->nz;
    const int lx = p->lx, ly = p->ly, lz = p->lz, nh = p->nh;
    Scratch s;
    double *cx, *cy, *d, *u, *rbar, *buf;
    HIP_TRY(s.get((void**)&cx, sizeof(double) * px * p->mx), "allocation (cos table)");
    HIP_TRY(s.get((void**)&cy, sizeof(double) * qy * p->my), "allocation (cos table)");
    HIP_TRY(s.get((void**)&d, sizeof(double) * (size_t)p->mx * p->my * rz), "allocation (mode table)");
    HIP_TRY(s.get((void**)&u, sizeof(double) * (size_t)p->mx * qy * rz), "allocation (partial sums)");
    HIP_TRY(s.get((void**)&rbar, sizeof(double) * (size_t)px * qy * rz), "allocation (Green table)");
    HIP_TRY(s.get((void**)&buf, sizeof(double) * (size_t)lx * ly * lz), "allocation (spectrum buffer)");

    const double norm = 1.0 / (2.0 * M_PI * p->a * p->b);
    HIP_TRY(launch_cos_table(cx, p->nx, 2 * p->nx - 1, p->mx, p->hx / p->a, 2.0 * p->x0 / p->a, st), "cos table");
    HIP_TRY(launch_cos_table(cy, p->ny, 2 * p->ny - 1, p->my, p->hy / p->b, 2.0 * p->y0 / p->b, st), "cos table");
    HIP_TRY(launch_modes(d, p->mx, p->my, rz, p->a, p->b, p->hz, (p->kind & 0x0f) == PIPE_GREEN_IGF_Z, norm, st), "mode table");
    // U[m] (qy x rz) = Cy (qy x my) * D[m] (my x rz)
    HIP_TRY(launch_gemm_f64(cy, d, u, qy, rz, p->my, p->my, rz, rz, 0, (long)p->my * rz, (long)qy * rz, p->mx, st),
            "mode contraction (y)");
    // Rbar (px x qy*rz) = Cx (px x mx) * U (mx x qy*rz)
    HIP_TRY(launch_gemm_f64(cx, u, rbar, px, qy * rz, p->mx, p->mx, (long)qy * rz, (long)qy * rz, 0, 0, 0, 1, st),
            "mode contraction (x)");
    for (int term = 0; term < 4; ++term) {
        const int xcorr = (term == 2 || term == 3), ycorr = (term == 1 || term == 3);
        HIP_TRY(launch_arrange(buf, rbar, p->nx, p->ny, p->nz, lx, ly, lz, xcorr, ycorr, st), "Green arrangement");
        HIP_TRY(launch_z_r2c<double>(nh, buf, lz, lz, buf, nh, (long)lx * ly, p->ctx->tw, st), "spectra z transform");
        HIP_TRY(launch_strided<double>(ly, false, buf, buf, ly, ly, nh, nh, nh, (long)ly * nh, (long)ly * nh, lx,
                                       p->ctx->tw, st),
                "spectra y transform");
        HIP_TRY(launch_strided<double>(lx, false, buf, buf, lx, lx, (long)ly * nh, (long)ly * nh, (long)ly * nh, 0, 0, 1,
                                       p->ctx->tw, st),
                "spectra x transform");
        HIP_TRY(launch_compress(buf, p->table, p->nyq, p->rb, term, lx, ly, nh, p->tile, st), "spectra compression");
    }
    if (keep_green) {
        HIP_TRY(dev_alloc((void**)&p->green, sizeof(double) * (size_t)px * qy * rz), "allocation (kept Green table)");
        HIP_TRY(hipMemcpyAsync(p->green, rbar, sizeof(double) * (size_t)px * qy * rz, hipMemcpyDeviceToDevice, st),
                "Green table copy");
    }
    HIP_TRY(hipStreamSynchronize(st), "plan build");
    return PIPE_OK;
}

// Banded spectra (Eq. 18): the Green table at plane distances 0..N, each
// slice arranged in x and y and transformed in x and y only.  nband < 0: N
// from the decay bound B(d) = sum_mn |D_mn(d)| of the mode table (|R| <= B).
pipe_status_t build_band_spectra(pipe_plan_s* p, hipStream_t st, int nband, double tol, bool keep_green) {
    const int px = 3 * p->nx - 1, qy = 3 * p->ny - 1;
    const int lx = p->lx, ly = p->ly, mx = p->mx, my = p->my;
    const int rfull = nband < 0 ? p->nz : std::min(nband, p->nz - 1) + 1;   // planes of the mode table
    Scratch s;
    double *cx, *cy, *d, *u, *rbar, *buf, *cbuf;
    HIP_TRY(s.get((void**)&cx, sizeof(double) * px * mx), "allocation (cos table)");
    HIP_TRY(s.get((void**)&cy, sizeof(double) * qy * my), "allocation (cos table)");
    HIP_TRY(s.get((void**)&d, sizeof(double) * (size_t)mx * my * rfull), "allocation (mode table)");
    const double norm = 1.0 / (2.0 * M_PI * p->a * p->b);
    HIP_TRY(launch_cos_table(cx, p->nx, 2 * p->nx - 1, mx, p->hx / p->a, 2.0 * p->x0 / p->a, st), "cos table");
    HIP_TRY(launch_cos_table(cy, p->ny, 2 * p->ny - 1, my, p->hy / p->b, 2.0 * p->y0 / p->b, st), "cos table");
    HIP_TRY(launch_modes(d, mx, my, rfull, p->a, p->b, p->hz, (p->kind & 0x0f) == PIPE_GREEN_IGF_Z, norm, st),
            "mode table");
    int nb = rfull - 1;
    if (nband < 0) {
        std::vector<double> h((size_t)mx * my * rfull);
        HIP_TRY(hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, st), "mode table copy");
        HIP_TRY(hipStreamSynchronize(st), "mode table copy");
        std::vector<double> B(rfull, 0.0);
        for (size_t i = 0; i < h.size(); ++i) B[i % rfull] += std::fabs(h[i]);
        // smallest N with B(d) <= tol B(0) for every N < d < nz
        while (nb > 0 && B[nb] <= tol * B[0]) --nb;
    }
    p->band = nb;
    const int D = nb + 1;
    const size_t orbits = (size_t)(lx / 2 + 1) * (ly / 2 + 1);
    p->table_elems = 10 * orbits * D;
    p->nyq_elems = 0;
    HIP_TRY(dev_alloc(&p->table, p->table_elems * p->rb), "allocation (Green spectra)");
    p->nyq = nullptr;
    HIP_TRY(hipMemsetAsync(p->table, 0, p->table_elems * p->rb, st), "spectra clear");
    HIP_TRY(s.get((void**)&u, sizeof(double) * (size_t)mx * qy * D), "allocation (partial sums)");
    HIP_TRY(s.get((void**)&rbar, sizeof(double) * (size_t)px * qy * D), "allocation (Green table)");
    HIP_TRY(s.get((void**)&buf, sizeof(double) * (size_t)lx * ly * D), "allocation (spectrum buffer)");
    HIP_TRY(s.get((void**)&cbuf, 2 * sizeof(double) * (size_t)lx * ly * D), "allocation (spectrum buffer)");
    double* tmp;
    HIP_TRY(s.get((void**)&tmp, sizeof(double) * 9 * orbits * D), "allocation (spectra staging)");
    // U[m] (qy x D) = Cy (qy x my) * D[m] (my x D, rows rfull apart)
    HIP_TRY(launch_gemm_f64(cy, d, u, qy, D, my, my, rfull, D, 0, (long)my * rfull, (long)qy * D, mx, st),
            "mode contraction (y)");
    // Rbar (px x qy*D) = Cx (px x mx) * U (mx x qy*D)
    HIP_TRY(launch_gemm_f64(cx, u, rbar, px, qy * D, mx, mx, (long)qy * D, (long)qy * D, 0, 0, 0, 1, st),
            "mode contraction (x)");
    for (int term = 0; term < 4; ++term) {
        const int xcorr = (term == 2 || term == 3), ycorr = (term == 1 || term == 3);
        HIP_TRY(launch_arrange(buf, rbar, p->nx, p->ny, D, lx, ly, D, xcorr, ycorr, st, true), "Green arrangement");
        HIP_TRY(launch_strided_real<double>(ly, false, buf, cbuf, ly, ly, D, D, D, (long)ly * D, (long)ly * D, lx, 1.0,
                                            p->ctx->tw, st),
                "spectra y transform");
        HIP_TRY(launch_strided<double>(lx, false, cbuf, cbuf, lx, lx, (long)ly * D, (long)ly * D, (long)ly * D, 0, 0, 1,
                                       p->ctx->tw, st),
                "spectra x transform");
        HIP_TRY(launch_compress_band(cbuf, tmp, term, lx, ly, D, st), "spectra compression");
    }
    HIP_TRY(launch_band_coefficients(tmp, p->table, p->rb, lx, ly, D, st), "banded coefficients");
    if (keep_green) {
        HIP_TRY(dev_alloc((void**)&p->green, sizeof(double) * (size_t)px * qy * D), "allocation (kept Green table)");
        HIP_TRY(hipMemcpyAsync(p->green, rbar, sizeof(double) * (size_t)px * qy * D, hipMemcpyDeviceToDevice, st),
                "Green table copy");
    }
    HIP_TRY(hipStreamSynchronize(st), "plan build");
    return PIPE_OK;
}

std::mutex g_use_mu;

// Record that a solve on stream st has just been queued (skipped while the
// stream is being captured into a graph: the caller then owns the ordering).
hipError_t note_use(pipe_plan_s* p, hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess || cs != hipStreamCaptureStatusNone) return e;
    std::lock_guard<std::mutex> lk(g_use_mu);
    for (auto& u : p->uses)
        if (u.first == st) return hipEventRecord(u.second, st);
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    p->uses.push_back({st, ev});
    return hipEventRecord(ev, st);
}

void plan_free(pipe_plan_s* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    // wait for this plan's own queued solves only
    for (auto& u : p->uses) {
        (void)hipEventSynchronize(u.second);
        (void)hipEventDestroy(u.second);
    }
    for (hipEvent_t e : p->tev) (void)hipEventSynchronize(e);
    for (hipEvent_t e : p->tev) (void)hipEventDestroy(e);
    if (p->table) (void)hipFree(p->table);
    if (p->green) (void)hipFree(p->green);
    delete p;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

pipe_status_t check_solve_args(pipe_plan_t plan, const void* rho, void* phi, void* ws) {
    if (!reg_has(plan)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed plan handle");
    if (!rho || !phi || !ws) return fail(PIPE_ERR_INVALID_ARG, "rho, phi and workspace must be non-null");
    if (((uintptr_t)ws) & 255) return fail(PIPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (((uintptr_t)rho) % plan->rb || ((uintptr_t)phi) % plan->rb)
        return fail(PIPE_ERR_INVALID_ARG, "rho and phi must be aligned to the element size");
    const size_t nb = (size_t)plan->nx * plan->ny * plan->nz * plan->rb;
    if (overlaps(rho, nb, phi, nb)) return fail(PIPE_ERR_ALIASING, "rho and phi overlap");
    if (overlaps(rho, nb, ws, plan->ws_bytes) || overlaps(phi, nb, ws, plan->ws_bytes))
        return fail(PIPE_ERR_ALIASING, "workspace overlaps rho or phi");
    return PIPE_OK;
}

enum { EV_NONE = 0 };

template <typename real>
pipe_status_t run_passes(pipe_plan_s* p, const void* rho, void* phi, void* ws, hipStream_t st, bool adjoint,
                         hipEvent_t* ev) {
    const size_t cb = 2 * sizeof(real);
    char* A1 = (char*)ws;
    char* A2 = A1 + align256((size_t)p->nx * p->ny * a1_pitch(p) * cb);
    const int nx = p->nx, ny = p->ny, nz = p->nz, ly = p->ly, nh = p->nh;
    const long p1 = a1_pitch(p);
    const TwiddleBank& tw = p->ctx->tw;
    if (ev) HIP_TRY(hipEventRecord(ev[0], st), "event");
    HIP_TRY(launch_z_r2c<real>(nh, (const real*)rho, nz, nz, A1, p1, (long)nx * ny, tw, st, nullptr, 1, true,
                               p->zcap),
            "z forward pass");
    if (ev) HIP_TRY(hipEventRecord(ev[1], st), "event");
    // A2 is (ly, nx, lz/2): ky-major, see passes.hip
    const long pa = a2_pitch(nh, p->apad);
    HIP_TRY(launch_strided<real>(ly, false, A1, A2, ny, ly, p1, (long)nx * pa, nh, (long)ny * p1, pa, nx, tw, st),
            "y forward pass");
    if (ev) HIP_TRY(hipEventRecord(ev[2], st), "event");
    HIP_TRY(launch_xprod<real>(p->lx, adjoint, A2, nx, ly, nh, pa, p->tile, p->xnt != 0, (const real*)p->table,
                               (const real*)p->nyq, tw, st, nullptr, 1, false, p->nval),
            "x pass with spectral product");
    if (ev) HIP_TRY(hipEventRecord(ev[3], st), "event");
    HIP_TRY(launch_strided<real>(ly, true, A2, A1, ly, ny, (long)nx * pa, p1, nh, pa, (long)ny * p1, nx, tw, st),
            "y inverse pass");
    if (ev) HIP_TRY(hipEventRecord(ev[4], st), "event");
    const real scale = (real)(p->hx * p->hy * p->hz / ((double)p->lx * p->ly * p->lz));
    HIP_TRY(launch_z_c2r<real>(nh, A1, p1, (real*)phi, nz, nz, (long)nx * ny, scale, tw, st, nullptr, 1, true,
                               p->zcap),
            "z inverse pass");
    if (ev) HIP_TRY(hipEventRecord(ev[5], st), "event");
    return PIPE_OK;
}

// Chooses the banded x pass by timing (on zeroed scratch of the workspace's
// size: timing does not depend on the values): for N >= 1 the single-window
// or the chunked kernel (PIPE_BAND_KERNEL=single or =chunked forces one), for
// N = 0 the packed-column tile, the widest or half of it (PIPE_BAND_TILE0=T
// forces one).  Tests exercise every choice.
pipe_status_t choose_band_kernel(pipe_plan_s* p, hipStream_t st) {
    struct Cand {
        bool single;
        int tile0;
    };
    std::vector<Cand> cands;
    const int T0 = band0_tile(p->lx, p->rb);
    if (p->band == 0) {
        if (const char* f = std::getenv("PIPE_BAND_TILE0")) {
            const int t = atoi(f);
            if (t != T0 && !(T0 > 1 && t == T0 / 2))
                return fail(PIPE_ERR_INVALID_ARG, "PIPE_BAND_TILE0 must be %d or %d (got '%s')", T0, T0 / 2, f);
            p->band_tile0 = t;
            return PIPE_OK;
        }
        cands.push_back({false, T0});
        if (T0 > 1) cands.push_back({false, T0 / 2});
    } else {
        p->band_tile0 = T0;
        if (band_small_columns_for(p->lx, p->rb, p->band) <= 0) {
            p->band_single = false;
            return PIPE_OK;
        }
        if (const char* f = std::getenv("PIPE_BAND_KERNEL")) {
            if (!strcmp(f, "single") || !strcmp(f, "chunked")) {
                p->band_single = !strcmp(f, "single");
                return PIPE_OK;
            }
        }
        cands.push_back({false, T0});
        cands.push_back({true, T0});
    }
    if (cands.size() == 1) {
        p->band_single = cands[0].single;
        p->band_tile0 = cands[0].tile0;
        return PIPE_OK;
    }
    void* ws = nullptr;
    HIP_TRY(dev_alloc(&ws, p->ws_bytes), "allocation (band kernel timing)");
    struct Free {
        void* q;
        ~Free() { (void)hipFree(q); }
    } guard{ws};
    HIP_TRY(hipMemsetAsync(ws, 0, p->ws_bytes, st), "band kernel timing");
    const size_t half = p->ws_bytes / 2;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    std::vector<float> best(cands.size(), 0.f);
    pipe_status_t s = PIPE_OK;
    for (size_t v = 0; v < cands.size() && s == PIPE_OK; ++v) {
        auto launch = [&]() -> hipError_t {
            return p->rb == 8 ? launch_xband<double>(p->lx, ws, (char*)ws + half, p->nx, p->ly, p->nz, band_pitch(p),
                                                     p->band, (const double*)p->table, p->ctx->tw, st,
                                                     cands[v].single, cands[v].tile0)
                              : launch_xband<float>(p->lx, ws, (char*)ws + half, p->nx, p->ly, p->nz, band_pitch(p),
                                                    p->band, (const float*)p->table, p->ctx->tw, st, cands[v].single,
                                                    cands[v].tile0);
        };
        hipError_t e = launch();   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < 5 && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&best[v], e0, e1);
        if (e != hipSuccess) s = hip_fail(e, "band kernel timing");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == PIPE_OK) {
        const size_t bi = std::min_element(best.begin(), best.end()) - best.begin();
        p->band_single = cands[bi].single;
        p->band_tile0 = cands[bi].tile0;
    }
    return s;
}

// Banded solve (Eq. 18): three kernels; the timing events of the two absent
// passes are recorded back to back.
template <typename real>
pipe_status_t run_band_passes(pipe_plan_s* p, const void* rho, void* phi, void* ws, hipStream_t st, bool adjoint,
                              hipEvent_t* ev) {
    const size_t cb = 2 * sizeof(real);
    char* A = (char*)ws;
    const int nx = p->nx, ny = p->ny, nz = p->nz, ly = p->ly;
    const long pitch = band_pitch(p);
    char* B = A + align256((size_t)nx * ly * pitch * cb);
    const TwiddleBank& tw = p->ctx->tw;
    if (ev) HIP_TRY(hipEventRecord(ev[0], st), "event");
    HIP_TRY(launch_strided_pair<real>(ly, false, rho, A, ny, ly, nz, (long)nx * pitch, (long)ny * nz, pitch, nx, nz,
                                      (real)1, tw, st),
            "y forward pass");
    if (ev) HIP_TRY(hipEventRecord(ev[1], st), "event");
    (void)adjoint;   // the banded coefficient matrices are symmetric: same kernel both ways
    HIP_TRY(launch_xband<real>(p->lx, A, B, nx, ly, nz, pitch, p->band, (const real*)p->table, tw, st,
                               p->band_single, p->band_tile0),
            "x pass with banded product");
    if (ev) HIP_TRY(hipEventRecord(ev[2], st), "event");
    // 1/2 undoes the factor 2 of the split in the x pass
    const real scale = (real)(0.5 * p->hx * p->hy * p->hz / ((double)p->lx * p->ly));
    HIP_TRY(launch_strided_pair<real>(ly, true, B, phi, ly, ny, nz, (long)nx * pitch, (long)ny * nz, pitch, nx, nz,
                                      scale, tw, st),
            "y inverse pass");
    if (ev)
        for (int i = 3; i < 6; ++i) HIP_TRY(hipEventRecord(ev[i], st), "event");
    return PIPE_OK;
}

// record_use: note the stream for pipe_plan_destroy (creates one event the
// first time a stream is seen; the allocation-free entry point skips it).
pipe_status_t solve_impl(pipe_plan_t plan, const void* rho, void* phi, void* ws, void* stream, bool adjoint,
                         hipEvent_t* ev, bool record_use = true) {
    pipe_status_t s = check_solve_args(plan, rho, phi, ws);
    if (s != PIPE_OK) return s;
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != plan->device) HIP_TRY(hipSetDevice(plan->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    if (!ev && plan->tn < plan->tmax) ev = &plan->tev[6 * (size_t)plan->tn++];
    if (plan->band >= 0)
        s = plan->rb == 8 ? run_band_passes<double>(plan, rho, phi, ws, st, adjoint, ev)
                          : run_band_passes<float>(plan, rho, phi, ws, st, adjoint, ev);
    else
        s = plan->rb == 8 ? run_passes<double>(plan, rho, phi, ws, st, adjoint, ev)
                          : run_passes<float>(plan, rho, phi, ws, st, adjoint, ev);
    if (s == PIPE_OK && record_use) {
        const hipError_t e = note_use(plan, st);
        if (e != hipSuccess) s = hip_fail(e, "solve completion event");
    }
    if (cur != plan->device) (void)hipSetDevice(cur);
    return s;
}

}  // namespace

// ---------------------------------------------------------------- autotuner
//
// For a mesh with default padded lengths, the plan can time the five passes
// for each candidate factorisation of the padded lengths (smallest supported
// 2^p 3^q length >= 2n, smallest power of two, smallest 3 * 2^k) and keep the
// fastest.  Pass timing does not depend on the values, so candidates run on
// scratch buffers with a zero table.  Results are cached per (mesh,
// precision) for the process and, if PIPE_TUNE_CACHE names a file, on disk.
namespace {

struct TuneKey {
    std::string arch;   // device architecture (gcnArchName): timings do not carry across chips
    int nx, ny, nz, rb, nval, members;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, nx, ny, nz, rb, nval, members) <
               std::tie(o.arch, o.nx, o.ny, o.nz, o.rb, o.nval, o.members);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, 3>> g_tune;
std::string g_tune_loaded;   // the cache file read last (re-read when PIPE_TUNE_CACHE names another)

// Padded lengths a cached entry may hold for this mesh: the same rules as
// explicit lengths in validate() (even, >= 2n - 1, a supported transform).
bool tuned_lengths_ok(const TuneKey& k, const std::array<int, 3>& v) {
    const int n[3] = {k.nx, k.ny, k.nz};
    for (int d = 0; d < 3; ++d) {
        const int L = v[d];
        if (L < 2 * n[d] - 1 || (d == 2 && L % 2)) return false;
        if (!fft_length_ok(d == 2 ? L / 2 : L)) return false;
    }
    return true;
}

// Cache file: one entry per line, "pipe-tune-v2 arch nx ny nz real_bytes nval
// members lx ly lz"; other lines are skipped.
void tune_cache_load() {
    const char* path = getenv("PIPE_TUNE_CACHE");
    if (!path || g_tune_loaded == path) return;
    g_tune_loaded = path;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512], arch[128];
    while (fgets(line, sizeof line, f)) {
        TuneKey k;
        std::array<int, 3> v;
        if (sscanf(line, "pipe-tune-v2 %127s %d %d %d %d %d %d %d %d %d", arch, &k.nx, &k.ny, &k.nz, &k.rb, &k.nval,
                   &k.members, &v[0], &v[1], &v[2]) != 10)
            continue;
        k.arch = arch;
        if (tuned_lengths_ok(k, v)) g_tune[k] = v;
    }
    fclose(f);
}

void tune_cache_store(const TuneKey& k, const std::array<int, 3>& v) {
    const char* path = getenv("PIPE_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "pipe-tune-v2 %s %d %d %d %d %d %d %d %d %d\n", k.arch.c_str(), k.nx, k.ny, k.nz, k.rb, k.nval,
            k.members, v[0], v[1], v[2]);
    fclose(f);
}

std::string device_arch(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    for (char& c : a)
        if (c == ' ') c = '_';
    return a.empty() ? "unknown" : a;
}

// supported lengths >= need: the smallest, the smallest even one, the smallest
// power of two, the smallest 3 * 2^k (each a different radix plan) and the
// modelled default
std::vector<int> length_candidates(int need, bool half, bool fp64) {
    std::vector<int> out{pick_modelled_length(need, half, fp64)};
    int best = -1, even = -1, pow2 = -1, three = -1;
    for (int v : kFftLengths) {
        if (v < need) continue;
        if (best < 0) best = v;
        if (even < 0 && v % 2 == 0) even = v;
        if (pow2 < 0 && (v & (v - 1)) == 0) pow2 = v;
        if (three < 0 && v % 3 == 0 && ((v / 3) & (v / 3 - 1)) == 0) three = v;
    }
    for (int v : {best, even, pow2, three})
        if (v > 0 && std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
    return out;
}

template <typename real>
pipe_status_t run_passes(pipe_plan_s* p, const void* rho, void* phi, void* ws, hipStream_t st, bool adjoint,
                         hipEvent_t* ev);
template <typename real>
pipe_status_t launch_group(pipe_plan_s* p, const GroupArgs* args, int n, bool al_in, bool al_out, hipStream_t st,
                           bool shared_table = false);

// Times candidate configurations of one mesh (lengths and schedule differ,
// everything else equal) on scratch buffers with a zero table: pass timing
// does not depend on the values.  members = 1: one solve at a time
// (latency); members > 1: one grouped launch of that many solves
// (throughput, as in a batch).  ms_out[i] = ms per solve of candidate i.
pipe_status_t time_candidates(std::vector<pipe_plan_s>& cands, int members, hipStream_t st, std::vector<double>& ms_out) {
    size_t ws_max = 0, tab_max = 0;
    for (pipe_plan_s& q : cands) {
        q.nh = q.lz / 2;
        const size_t orbits = (size_t)(q.lx / 2 + 1) * (q.ly / 2 + 1);
        q.table_elems = q.nval * orbits * ((q.nh + q.tile - 1) / q.tile) * q.tile;
        q.nyq_elems = q.nval * orbits;
        q.ws_bytes = plan_ws_bytes(&q);
        ws_max = std::max(ws_max, q.ws_bytes);
        tab_max = std::max(tab_max, (q.table_elems + q.nyq_elems) * q.rb);
    }
    const pipe_plan_s& t0 = cands[0];
    const size_t field = align256((size_t)t0.nx * t0.ny * t0.nz * t0.rb);
    ws_max = align256(ws_max);
    Scratch s;
    void *ws, *tab, *rho, *phi;
    GroupArgs* dargs = nullptr;
    HIP_TRY(s.get(&ws, ws_max * members), "tuning allocation");
    HIP_TRY(s.get(&tab, tab_max), "tuning allocation");
    HIP_TRY(s.get(&rho, field), "tuning allocation");
    HIP_TRY(s.get(&phi, field * members), "tuning allocation");
    if (members > 1) HIP_TRY(s.get((void**)&dargs, sizeof(GroupArgs) * 5 * members), "tuning allocation");
    HIP_TRY(hipMemsetAsync(tab, 0, tab_max, st), "tuning fill");
    HIP_TRY(hipMemsetAsync(rho, 0, field, st), "tuning fill");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    ms_out.assign(cands.size(), 1e30);
    pipe_status_t rs = PIPE_OK;
    for (pipe_plan_s& q : cands) {
        q.table = tab;
        q.nyq = (char*)tab + q.table_elems * q.rb;
        q.tev.clear(); q.tmax = 0; q.tn = 0;
    }
    // Rounds over all candidates, each candidate's best round kept, so that
    // drift during the timing does not favour whichever candidate ran first.
    const int rounds = cands.size() > 1 ? 3 : 1, reps = 3;
    for (int round = 0; round < rounds && rs == PIPE_OK; ++round) {
        for (size_t i = 0; i < cands.size() && rs == PIPE_OK; ++i) {
            pipe_plan_s& q = cands[i];
            if (members > 1) {
                std::vector<GroupArgs> a(5 * members);
                for (int k = 0; k < members; ++k) {
                    char* A1 = (char*)ws + ws_max * k;
                    char* A2 = A1 + align256((size_t)q.nx * q.ny * a1_pitch(&q) * 2 * q.rb);
                    char* ph = (char*)phi + field * k;
                    a[0 * members + k] = {rho, A1, nullptr, nullptr, 0.0};
                    a[1 * members + k] = {A1, A2, nullptr, nullptr, 0.0};
                    a[2 * members + k] = {A2, A2, q.table, q.nyq, 0.0};
                    a[3 * members + k] = {A2, A1, nullptr, nullptr, 0.0};
                    a[4 * members + k] = {A1, ph, nullptr, nullptr, 1.0};
                }
                he = hipMemcpyAsync(dargs, a.data(), a.size() * sizeof(GroupArgs), hipMemcpyHostToDevice, st);
                if (he == hipSuccess) he = hipStreamSynchronize(st);
                if (he != hipSuccess) {
                    rs = hip_fail(he, "tuning descriptors");
                    break;
                }
            }
            for (int r = 0; r < 1 + reps && rs == PIPE_OK; ++r) {   // one warm-up solve, then reps timed
                if (r == 1) {
                    he = hipEventRecord(e0, st);
                    if (he != hipSuccess) rs = hip_fail(he, "tuning timing");
                }
                if (rs != PIPE_OK) break;
                if (members > 1)
                    rs = q.rb == 8 ? launch_group<double>(&q, dargs, members, true, true, st)
                                   : launch_group<float>(&q, dargs, members, true, true, st);
                else
                    rs = q.rb == 8 ? run_passes<double>(&q, rho, phi, ws, st, false, nullptr)
                                   : run_passes<float>(&q, rho, phi, ws, st, false, nullptr);
            }
            if (rs != PIPE_OK) break;
            float ms = 0.f;
            he = hipEventRecord(e1, st);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) rs = hip_fail(he, "tuning timing");
            else ms_out[i] = std::min(ms_out[i], (double)ms / (reps * members));
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rs;
}

pipe_status_t autotune_lengths(pipe_plan_s* tmpl, int members, hipStream_t st, int* lx, int* ly, int* lz,
                               double* ms_out) {
    const TuneKey key{device_arch(tmpl->device), tmpl->nx, tmpl->ny, tmpl->nz, tmpl->rb, tmpl->nval, members};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto it = g_tune.find(key);
        if (it != g_tune.end() && !tuned_lengths_ok(key, it->second)) {
            g_tune.erase(it);   // unusable entry: tune again
            it = g_tune.end();
        }
        if (it != g_tune.end()) {
            *lx = it->second[0];
            *ly = it->second[1];
            *lz = it->second[2];
            *ms_out = 0.0;
            return PIPE_OK;
        }
    }
    const bool f64 = tmpl->rb == 8;
    const std::vector<int> cx = length_candidates(2 * tmpl->nx, false, f64),
                           cy = length_candidates(2 * tmpl->ny, false, f64), cz = length_candidates(tmpl->nz, true, f64);
    std::vector<pipe_plan_s> cands;
    for (int a : cx)
        for (int b : cy)
            for (int c : cz) {
                pipe_plan_s q = *tmpl;
                q.lx = a; q.ly = b; q.lz = 2 * c;
                q.tile = xprod_tile(q.lx, q.rb);   // default schedule
                q.apad = 0; q.zcap = 2048;
                cands.push_back(q);
            }
    if (cands.size() == 1) {
        *lx = cands[0].lx; *ly = cands[0].ly; *lz = cands[0].lz;
        *ms_out = 0.0;
        return PIPE_OK;
    }
    std::vector<double> ms;
    pipe_status_t rs = time_candidates(cands, members, st, ms);
    if (rs != PIPE_OK) return rs;
    const size_t bi = std::min_element(ms.begin(), ms.end()) - ms.begin();
    *lx = cands[bi].lx; *ly = cands[bi].ly; *lz = cands[bi].lz;
    *ms_out = ms[bi];
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const std::array<int, 3> v{*lx, *ly, *lz};
        g_tune[key] = v;
        tune_cache_store(key, v);
    }
    return PIPE_OK;
}

// ---------------------------------------------------------------- schedule
//
// With the padded lengths fixed, three launch parameters change no result
// (each output value is computed by the same arithmetic) but move the time a
// lot depending on the mesh, the precision and the chip's memory interleave:
// the kz tile of the fused x pass (its widest T or T/2), the row pitch of the
// y-transformed array (lz/2 plus 0, 16 or 32 unused slots: its rows are read
// and written at a stride of pitch values by the fused and y passes), and the
// block cap of the persistent z passes (1024, 2048 or 4096), and whether the
// fused x pass writes its rows with non-temporal stores.  Each plan times the
// (tile, pitch) pairs, then the caps and the stores, on scratch buffers, and keeps the
// fastest; the choice is cached like the lengths.  PIPE_SCHEDULE=fixed uses
// (widest T, no pad, 2048, plain stores); PIPE_SCHEDULE=T,pad,cap[,nt] forces one.

struct SchedKey {
    std::string arch;
    int nx, ny, nz, lx, ly, lz, rb, nval, members;
    bool operator<(const SchedKey& o) const {
        return std::tie(arch, nx, ny, nz, lx, ly, lz, rb, nval, members) <
               std::tie(o.arch, o.nx, o.ny, o.nz, o.lx, o.ly, o.lz, o.rb, o.nval, o.members);
    }
};
std::map<SchedKey, std::array<int, 5>> g_sched;
std::string g_sched_loaded;

bool schedule_ok(int lx, int rb, const std::array<int, 5>& v) {
    const int T = xprod_tile(lx, rb);
    // non-temporal x-pass stores exist in FP64 only; the A1 pad keeps rows 16-byte aligned (even)
    return (v[0] == T || (T > 1 && v[0] == T / 2)) && v[1] >= 0 && v[1] <= 256 && v[2] >= 1 && v[2] <= 65536 &&
           (v[3] == 0 || (v[3] == 1 && rb == 8)) && v[4] >= 0 && v[4] <= 256 && v[4] % 2 == 0;
}

void sched_cache_load() {
    const char* path = getenv("PIPE_TUNE_CACHE");
    if (!path || g_sched_loaded == path) return;
    g_sched_loaded = path;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512], arch[128];
    while (fgets(line, sizeof line, f)) {
        SchedKey k;
        std::array<int, 5> v;
        if (sscanf(line, "pipe-sched-v3 %127s %d %d %d %d %d %d %d %d %d %d %d %d %d %d", arch, &k.nx, &k.ny, &k.nz,
                   &k.lx, &k.ly, &k.lz, &k.rb, &k.nval, &k.members, &v[0], &v[1], &v[2], &v[3], &v[4]) != 15)
            continue;
        k.arch = arch;
        if (schedule_ok(k.lx, k.rb, v)) g_sched[k] = v;
    }
    fclose(f);
}

void sched_cache_store(const SchedKey& k, const std::array<int, 5>& v) {
    const char* path = getenv("PIPE_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "pipe-sched-v3 %s %d %d %d %d %d %d %d %d %d %d %d %d %d %d\n", k.arch.c_str(), k.nx, k.ny, k.nz,
            k.lx, k.ly, k.lz, k.rb, k.nval, k.members, v[0], v[1], v[2], v[3], v[4]);
    fclose(f);
}

// Sets p->tile, p->apad, p->zcap, p->xnt, p->a1pad (p's lengths and sizes already set).
pipe_status_t tune_schedule(pipe_plan_s* p, int members, hipStream_t st) {
    const int T = xprod_tile(p->lx, p->rb);
    std::array<int, 5> v{T, 0, 2048, 0, a1_pad_rule(p)};
    auto apply = [&] {
        p->tile = v[0]; p->apad = v[1]; p->zcap = v[2]; p->xnt = v[3]; p->a1pad = v[4];
    };
    if (const char* f = getenv("PIPE_SCHEDULE")) {
        if (!strcmp(f, "fixed")) {
            apply();
            return PIPE_OK;
        }
        const int got = sscanf(f, "%d,%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3], &v[4]);
        if (got < 3 || !schedule_ok(p->lx, p->rb, v))
            return fail(PIPE_ERR_INVALID_ARG, "PIPE_SCHEDULE must be 'fixed' or 'T,pad,cap[,nt[,a1pad]]' with T %d or "
                        "%d, 0 <= pad <= 256, cap >= 1, nt 0 or 1 (1 in FP64 only), a1pad even in [0, 256] (got '%s')",
                        T, T / 2, f);
        apply();
        return PIPE_OK;
    }
    const SchedKey key{device_arch(p->device), p->nx, p->ny, p->nz, p->lx, p->ly, p->lz, p->rb, p->nval, members};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        sched_cache_load();
        auto it = g_sched.find(key);
        if (it != g_sched.end()) {
            v = it->second;
            apply();
            return PIPE_OK;
        }
    }
    // (tile, pad) pairs first, then the z cap and the x-pass stores with the best pair
    std::vector<pipe_plan_s> cands;
    for (int t : {T, T / 2}) {
        if (t < 1 || (t == T / 2 && T == 1)) continue;
        for (int pad : {0, 16, 32}) {
            pipe_plan_s q = *p;
            q.tile = t; q.apad = pad; q.zcap = 2048; q.xnt = 0; q.a1pad = a1_pad_rule(p);
            cands.push_back(q);
        }
    }
    std::vector<double> ms;
    pipe_status_t rs = time_candidates(cands, members, st, ms);
    if (rs != PIPE_OK) return rs;
    size_t bi = std::min_element(ms.begin(), ms.end()) - ms.begin();
    v = {cands[bi].tile, cands[bi].apad, 2048, 0, a1_pad_rule(p)};
    double best = ms[bi];
    std::vector<pipe_plan_s> more(p->rb == 8 ? 3 : 2, cands[bi]);
    more[0].zcap = 1024;
    more[1].zcap = 4096;
    if (p->rb == 8) more[2].xnt = 1;
    std::vector<double> ms2;
    if ((rs = time_candidates(more, members, st, ms2)) != PIPE_OK) return rs;
    for (int i = 0; i < 2; ++i)
        if (ms2[i] < best) {
            best = ms2[i];
            v[2] = more[i].zcap;
        }
    if (p->rb == 8 && ms2[2] < ms[bi]) v[3] = 1;   // compared at the same z cap
    apply();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_sched[key] = v;
    sched_cache_store(key, v);
    return PIPE_OK;
}

}  // namespace

extern "C" {

const char* pipe_status_string(pipe_status_t s) {
    switch (s) {
        case PIPE_OK: return "PIPE_OK";
        case PIPE_ERR_INVALID_ARG: return "PIPE_ERR_INVALID_ARG";
        case PIPE_ERR_UNSUPPORTED_SIZE: return "PIPE_ERR_UNSUPPORTED_SIZE";
        case PIPE_ERR_OUT_OF_MEMORY: return "PIPE_ERR_OUT_OF_MEMORY";
        case PIPE_ERR_NO_DEVICE: return "PIPE_ERR_NO_DEVICE";
        case PIPE_ERR_HIP: return "PIPE_ERR_HIP";
        case PIPE_ERR_ALIASING: return "PIPE_ERR_ALIASING";
    }
    return "PIPE_ERR_UNKNOWN";
}

const char* pipe_last_error(void) { return g_err.c_str(); }

namespace {

pipe_status_t create_plan(int nx, int ny, int nz, double hx, double hy, double hz, double a, double b, double x0,
                          double y0, int kind, int mx, int my, int lx, int ly, int lz, bool free_space, double g0,
                          void* hip_stream, pipe_plan_t* out) {
    if (!out) return fail(PIPE_ERR_INVALID_ARG, "out must be non-null");
    *out = nullptr;
    const bool keep = (kind & PIPE_KEEP_GREEN) != 0;
    const bool tune = (kind & (PIPE_AUTOTUNE | PIPE_AUTOTUNE_BATCH)) != 0 && lx == 0 && ly == 0 && lz == 0;
    const int tune_members = (kind & PIPE_AUTOTUNE_BATCH) ? 16 : 1;
    kind &= 0xff;
    pipe_status_t s = validate(nx, ny, nz, hx, hy, hz, a, b, x0, y0, kind, mx, my, &lx, &ly, &lz, free_space);
    if (s != PIPE_OK) return s;
    if (free_space && !std::isfinite(g0)) return fail(PIPE_ERR_INVALID_ARG, "g0 must be finite");
    if (free_space && keep) return fail(PIPE_ERR_INVALID_ARG, "free-space plans keep no Green table");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(PIPE_ERR_NO_DEVICE, "no HIP device available");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DeviceCtx* ctx = nullptr;
    if ((s = device_ctx(dev, &ctx)) != PIPE_OK) return s;

    auto t0 = std::chrono::steady_clock::now();
    double tune_ms = -1.0;
    if (tune) {
        pipe_plan_s tmpl;
        tmpl.nx = nx; tmpl.ny = ny; tmpl.nz = nz; tmpl.kind = kind; tmpl.rb = (kind & PIPE_PREC_FP32) ? 4 : 8;
        tmpl.hx = hx; tmpl.hy = hy; tmpl.hz = hz; tmpl.a = a; tmpl.b = b; tmpl.mx = mx; tmpl.my = my;
        tmpl.device = dev; tmpl.ctx = ctx; tmpl.nval = free_space ? 1 : 9;
        if ((s = autotune_lengths(&tmpl, tune_members, (hipStream_t)hip_stream, &lx, &ly, &lz, &tune_ms)) != PIPE_OK)
            return s;
    }
    pipe_plan_s* p = new pipe_plan_s();
    p->nx = nx; p->ny = ny; p->nz = nz; p->lx = lx; p->ly = ly; p->lz = lz; p->nh = lz / 2;
    p->mx = mx; p->my = my; p->kind = kind; p->rb = (kind & PIPE_PREC_FP32) ? 4 : 8;
    p->hx = hx; p->hy = hy; p->hz = hz; p->a = a; p->b = b;
    p->x0 = x0; p->y0 = y0; p->g0 = g0;
    p->device = dev; p->ctx = ctx;
    p->nval = free_space ? 1 : 9;
    const size_t orbits = (size_t)(lx / 2 + 1) * (ly / 2 + 1);
    // launch schedule (kz tile, row pitch, z block cap); the table layout follows the tile
    s = tune_schedule(p, tune_members, (hipStream_t)hip_stream);
    if (s != PIPE_OK) {
        plan_free(p);
        return s;
    }
    const size_t ntiles = (p->nh + p->tile - 1) / p->tile;
    p->table_elems = p->nval * orbits * ntiles * p->tile;
    p->nyq_elems = p->nval * orbits;
    e = dev_alloc(&p->table, (p->table_elems + p->nyq_elems) * p->rb);
    if (e == hipSuccess) e = hipMemset(p->table, 0, (p->table_elems + p->nyq_elems) * p->rb);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "allocation (Green spectra)");
    }
    p->nyq = (char*)p->table + p->table_elems * p->rb;
    s = build_spectra(p, (hipStream_t)hip_stream, keep);
    if (s != PIPE_OK) {
        plan_free(p);
        return s;
    }
    p->ws_bytes = plan_ws_bytes(p);
    p->tune_ms = tune_ms;
    p->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    reg_add(p);
    *out = p;
    return PIPE_OK;
}

}  // namespace

pipe_status_t pipe_green_plan_region(int nx, int ny, int nz, double hx, double hy, double hz, double a, double b,
                                     double x0, double y0, int kind, int mx, int my, int lx, int ly, int lz,
                                     void* hip_stream, pipe_plan_t* out) {
    return create_plan(nx, ny, nz, hx, hy, hz, a, b, x0, y0, kind, mx, my, lx, ly, lz, false, 0.0, hip_stream, out);
}

pipe_status_t pipe_free_plan(int nx, int ny, int nz, double hx, double hy, double hz, double g0, int kind, int lx,
                             int ly, int lz, void* hip_stream, pipe_plan_t* out) {
    if ((kind & 0x0f) != 0) return fail(PIPE_ERR_INVALID_ARG, "pipe_free_plan takes precision and autotune flags only");
    return create_plan(nx, ny, nz, hx, hy, hz, 0.0, 0.0, 0.0, 0.0, kind | PIPE_GREEN_FREE, 0, 0, lx, ly, lz, true, g0,
                       hip_stream, out);
}

pipe_status_t pipe_green_plan_ex(int nx, int ny, int nz, double hx, double hy, double hz, double a, double b,
                                 int kind, int mx, int my, int lx, int ly, int lz, void* hip_stream,
                                 pipe_plan_t* out) {
    return pipe_green_plan_region(nx, ny, nz, hx, hy, hz, a, b, 0.0, 0.0, kind, mx, my, lx, ly, lz, hip_stream, out);
}

namespace {
// ms per banded solve of p, on scratch buffers (timing does not depend on values).
pipe_status_t time_banded(pipe_plan_s* p, hipStream_t st, double* ms_out) {
    Scratch s;
    void *ws, *rho, *phi;
    const size_t field = align256((size_t)p->nx * p->ny * p->nz * p->rb);
    HIP_TRY(s.get(&ws, p->ws_bytes), "band timing allocation");
    HIP_TRY(s.get(&rho, field), "band timing allocation");
    HIP_TRY(s.get(&phi, field), "band timing allocation");
    HIP_TRY(hipMemsetAsync(rho, 0, field, st), "band timing fill");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    pipe_status_t rs = PIPE_OK;
    const int reps = 5;
    for (int r = 0; r < 2 + reps && rs == PIPE_OK; ++r) {
        if (r == 2 && (he = hipEventRecord(e0, st)) != hipSuccess) rs = hip_fail(he, "band timing");
        if (rs == PIPE_OK)
            rs = p->rb == 8 ? run_band_passes<double>(p, rho, phi, ws, st, false, nullptr)
                            : run_band_passes<float>(p, rho, phi, ws, st, false, nullptr);
    }
    float ms = 0.f;
    if (rs == PIPE_OK) {
        he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) rs = hip_fail(he, "band timing");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / reps;
    return rs;
}

// ms per solve of the 3-D plan the same mesh would get by default (default
// lengths and schedule), on scratch buffers.
pipe_status_t time_full_for(const pipe_plan_s* b, hipStream_t st, double* ms_out) {
    int lx = 0, ly = 0, lz = 0;
    pipe_status_t s = validate(b->nx, b->ny, b->nz, b->hx, b->hy, b->hz, b->a, b->b, b->x0, b->y0, b->kind, b->mx,
                               b->my, &lx, &ly, &lz);
    if (s != PIPE_OK) return s;
    std::vector<pipe_plan_s> c(1);
    pipe_plan_s& q = c[0];
    q.nx = b->nx; q.ny = b->ny; q.nz = b->nz; q.lx = lx; q.ly = ly; q.lz = lz; q.nh = lz / 2;
    q.mx = b->mx; q.my = b->my; q.kind = b->kind; q.rb = b->rb;
    q.hx = b->hx; q.hy = b->hy; q.hz = b->hz; q.a = b->a; q.b = b->b; q.x0 = b->x0; q.y0 = b->y0;
    q.device = b->device; q.ctx = b->ctx; q.nval = 9;
    q.tile = xprod_tile(lx, q.rb); q.apad = 0; q.zcap = 2048;
    std::vector<double> ms;
    if ((s = time_candidates(c, 1, st, ms)) != PIPE_OK) return s;
    *ms_out = ms[0];
    return PIPE_OK;
}
}  // namespace

pipe_status_t pipe_green_plan_banded(int nx, int ny, int nz, double hx, double hy, double hz, double a, double b,
                                     double x0, double y0, int kind, int mx, int my, int lx, int ly, int nband,
                                     double tol, void* hip_stream, pipe_plan_t* out) {
    if (!out) return fail(PIPE_ERR_INVALID_ARG, "out must be non-null");
    *out = nullptr;
    const bool keep = (kind & PIPE_KEEP_GREEN) != 0;
    const bool fastest = (kind & PIPE_BAND_FASTEST) != 0;
    kind &= 0xff;
    // the banded x pass takes a subset of the transform lengths
    if (lx == 0 && nx >= 1 && nx <= 512) {
        lx = pick_band_length(2 * nx);
        if (lx < 0) return fail(PIPE_ERR_UNSUPPORTED_SIZE, "lx: no banded padded length for nx = %d", nx);
    }
    pipe_status_t s = validate(nx, ny, nz, hx, hy, hz, a, b, x0, y0, kind, mx, my, &lx, &ly, nullptr);
    if (s != PIPE_OK) return s;
    if (!band_length_ok(lx))
        return fail(PIPE_ERR_UNSUPPORTED_SIZE,
                    "lx: banded plans take padded lengths divisible by 4 with a plan of 4k values per thread "
                    "(8, 12, 16, 24, 32, 36, 48, 64, 72, 96, 108, 128, 144, 192, 216, 256, 288, 384, 432, 512, "
                    "576, 768, 864, 1024); got %d", lx);
    if (nband < 0 && !(tol > 0.0 && tol < 1.0))
        return fail(PIPE_ERR_INVALID_ARG, "automatic band selection needs 0 < tol < 1 (got %g)", tol);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(PIPE_ERR_NO_DEVICE, "no HIP device available");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DeviceCtx* ctx = nullptr;
    if ((s = device_ctx(dev, &ctx)) != PIPE_OK) return s;
    auto t0 = std::chrono::steady_clock::now();
    pipe_plan_s* p = new pipe_plan_s();
    p->nx = nx; p->ny = ny; p->nz = nz; p->lx = lx; p->ly = ly; p->lz = 0; p->nh = 0;
    p->mx = mx; p->my = my; p->kind = kind; p->rb = (kind & PIPE_PREC_FP32) ? 4 : 8;
    p->hx = hx; p->hy = hy; p->hz = hz; p->a = a; p->b = b;
    p->x0 = x0; p->y0 = y0;
    p->device = dev; p->ctx = ctx;
    p->tile = band_tile(lx, p->rb);
    s = build_band_spectra(p, (hipStream_t)hip_stream, nband, tol, keep);
    if (s != PIPE_OK) {
        plan_free(p);
        return s;
    }
    p->ws_bytes = plan_ws_bytes(p);
    s = choose_band_kernel(p, (hipStream_t)hip_stream);
    if (s != PIPE_OK) {
        plan_free(p);
        return s;
    }
    // time the banded solve against the 3-D solve of the same mesh
    double t_band = 0, t_full = 0;
    s = time_banded(p, (hipStream_t)hip_stream, &t_band);
    if (s == PIPE_OK) s = time_full_for(p, (hipStream_t)hip_stream, &t_full);
    if (s != PIPE_OK) {
        plan_free(p);
        return s;
    }
    p->band_speedup = t_band > 0 ? t_full / t_band : 0;
    if (fastest && t_full < t_band) {
        // the full z sum is exact and faster here: return the 3-D plan instead
        pipe_plan_t full = nullptr;
        s = create_plan(nx, ny, nz, hx, hy, hz, a, b, x0, y0, kind | (keep ? PIPE_KEEP_GREEN : 0), mx, my, 0, 0, 0,
                        false, 0.0, hip_stream, &full);
        const double sp = p->band_speedup;
        plan_free(p);
        if (s != PIPE_OK) return s;
        full->band_speedup = sp;
        *out = full;
        return PIPE_OK;
    }
    p->tune_ms = -1.0;
    p->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    reg_add(p);
    *out = p;
    return PIPE_OK;
}

pipe_status_t pipe_green_plan(int nx, int ny, int nz, double hx, double hy, double hz, double a, double b, int kind,
                              pipe_plan_t* out) {
    return pipe_green_plan_ex(nx, ny, nz, hx, hy, hz, a, b, kind, 2 * nx, 2 * ny, 0, 0, 0, nullptr, out);
}

pipe_status_t pipe_default_lengths(int nx, int ny, int nz, int kind, int* lx, int* ly, int* lz) {
    if (!lx || !ly || !lz) return fail(PIPE_ERR_INVALID_ARG, "lx, ly and lz must be non-null");
    if (nx < 1 || ny < 1 || nz < 1) return fail(PIPE_ERR_INVALID_ARG, "nx, ny, nz must be >= 1");
    const int g = kind & 0x0f, pr = kind & ~0x0f;
    if (g != PIPE_GREEN_POINT && g != PIPE_GREEN_IGF_Z && g != PIPE_GREEN_FREE)
        return fail(PIPE_ERR_INVALID_ARG, "unknown Green kind %d", g);
    if (pr != PIPE_PREC_FP64 && pr != PIPE_PREC_FP32)
        return fail(PIPE_ERR_INVALID_ARG, "kind may hold only a Green kind and a precision flag (got 0x%x)", kind);
    const bool f64 = pr == PIPE_PREC_FP64;
    const int x = pick_modelled_length(2 * nx, false, f64), y = pick_modelled_length(2 * ny, false, f64),
              h = pick_modelled_length(nz, true, f64);
    if (x < 0 || y < 0 || h < 0)
        return fail(PIPE_ERR_UNSUPPORTED_SIZE, "no supported padded length for %s", x < 0 ? "nx" : y < 0 ? "ny" : "nz");
    *lx = x;
    *ly = y;
    *lz = 2 * h;
    return PIPE_OK;
}

pipe_status_t pipe_plan_info(pipe_plan_t p, pipe_plan_info_t* out) {
    if (!reg_has(p)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed plan handle");
    if (!out) return fail(PIPE_ERR_INVALID_ARG, "out must be non-null");
    memset(out, 0, sizeof *out);
    out->nx = p->nx; out->ny = p->ny; out->nz = p->nz;
    out->lx = p->lx; out->ly = p->ly; out->lz = p->lz;
    out->mx = p->mx; out->my = p->my; out->kind = p->kind; out->real_bytes = p->rb;
    out->hx = p->hx; out->hy = p->hy; out->hz = p->hz; out->a = p->a; out->b = p->b;
    out->x0 = p->x0; out->y0 = p->y0;
    out->norm = (p->kind & 0x0f) == PIPE_GREEN_FREE ? 1.0 : 1.0 / (2.0 * M_PI * p->a * p->b);
    out->workspace_bytes = p->ws_bytes;
    out->spectra_bytes = (p->table_elems + p->nyq_elems) * p->rb;
    plan_pass_bytes(p, out->pass_bytes);
    out->model_bytes = 0;
    for (double v : out->pass_bytes) out->model_bytes += v;
    out->build_ms = p->build_ms;
    out->tune_ms = p->tune_ms;
    out->band = p->band;
    out->band_speedup = p->band_speedup;
    out->xtile = p->band >= 0 ? (p->band == 0 ? p->band_tile0 : 0) : p->tile;
    out->apad = p->band >= 0 ? 0 : p->apad;
    out->zblocks = p->band >= 0 ? 0 : p->zcap;
    out->xnt = p->band >= 0 ? 0 : p->xnt;
    out->a1pad = p->band >= 0 ? 0 : p->a1pad;
    return PIPE_OK;
}

pipe_status_t pipe_poisson_solve(pipe_plan_t plan, const void* rho, void* phi, void* ws, void* stream) {
    return solve_impl(plan, rho, phi, ws, stream, false, nullptr);
}

pipe_status_t pipe_poisson_adjoint(pipe_plan_t plan, const void* dphi, void* drho, void* ws, void* stream) {
    return solve_impl(plan, dphi, drho, ws, stream, true, nullptr);
}

pipe_status_t pipe_poisson_solve_noalloc(pipe_plan_t plan, const void* rho, void* phi, void* stream) {
    if (!reg_has(plan)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed plan handle");
    if (plan->ws_bytes > kScratchBytes)
        return fail(PIPE_ERR_UNSUPPORTED_SIZE,
                    "the plan needs %zu bytes of workspace; the fixed scratch holds %zu (use pipe_poisson_solve "
                    "with a workspace of info.workspace_bytes)",
                    plan->ws_bytes, kScratchBytes);
    void* ws = plan->ctx->scratch;   // the plan's device's copy, set up with the device context
    if (!ws) return fail(PIPE_ERR_HIP, "fixed scratch not set up on device %d", plan->device);
    return solve_impl(plan, rho, phi, ws, stream, false, nullptr, false);
}

pipe_status_t pipe_poisson_solve_timed(pipe_plan_t plan, const void* rho, void* phi, void* ws, void* stream,
                                       float* pass_ms) {
    if (!pass_ms) return fail(PIPE_ERR_INVALID_ARG, "pass_ms must be non-null");
    pipe_status_t s = check_solve_args(plan, rho, phi, ws);
    if (s != PIPE_OK) return s;
    hipEvent_t ev[6];
    for (int i = 0; i < 6; ++i) HIP_TRY(hipEventCreate(&ev[i]), "hipEventCreate");
    s = solve_impl(plan, rho, phi, ws, stream, false, ev);
    if (s == PIPE_OK) {
        hipError_t e = hipEventSynchronize(ev[5]);
        if (e != hipSuccess) s = hip_fail(e, "hipEventSynchronize");
        for (int i = 0; i < 5 && s == PIPE_OK; ++i) {
            e = hipEventElapsedTime(&pass_ms[i], ev[i], ev[i + 1]);
            if (e != hipSuccess) s = hip_fail(e, "hipEventElapsedTime");
        }
    }
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
    return s;
}

pipe_status_t pipe_plan_timing(pipe_plan_t p, int max_solves, float* pass_ms_mean, int* count) {
    if (!reg_has(p)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed plan handle");
    if (max_solves < 0) return fail(PIPE_ERR_INVALID_ARG, "max_solves must be >= 0");
    if (max_solves > 0) {
        const size_t need = 6 * (size_t)max_solves;
        while (p->tev.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e), "hipEventCreate");
            p->tev.push_back(e);
        }
        p->tmax = max_solves;
        p->tn = 0;
        return PIPE_OK;
    }
    const int n = p->tn;
    p->tmax = 0;
    p->tn = 0;
    if (count) *count = n;
    if (pass_ms_mean) {
        for (int i = 0; i < 5; ++i) pass_ms_mean[i] = 0.f;
        if (n > 0) {
            HIP_TRY(hipEventSynchronize(p->tev[6 * (size_t)(n - 1) + 5]), "hipEventSynchronize");
            double acc[5] = {0, 0, 0, 0, 0};
            for (int s = 0; s < n; ++s)
                for (int i = 0; i < 5; ++i) {
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, p->tev[6 * (size_t)s + i], p->tev[6 * (size_t)s + i + 1]),
                            "hipEventElapsedTime");
                    acc[i] += ms;
                }
            for (int i = 0; i < 5; ++i) pass_ms_mean[i] = (float)(acc[i] / n);
        }
    }
    return PIPE_OK;
}

pipe_status_t pipe_plan_destroy(pipe_plan_t p) {
    if (!reg_del(p)) return fail(PIPE_ERR_INVALID_ARG, "invalid or already destroyed plan handle");
    plan_free(p);
    return PIPE_OK;
}

pipe_status_t pipe_plan_green_table(pipe_plan_t p, void* out, void* stream) {
    if (!reg_has(p)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed plan handle");
    if (!out) return fail(PIPE_ERR_INVALID_ARG, "out must be non-null");
    if (!p->green) return fail(PIPE_ERR_INVALID_ARG, "plan was built without keeping its Green table");
    const size_t n = (size_t)(3 * p->nx - 1) * (3 * p->ny - 1) * (p->band >= 0 ? p->band + 1 : p->nz);
    HIP_TRY(hipMemcpyAsync(out, p->green, n * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream), "copy");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "copy");
    return PIPE_OK;
}

pipe_status_t pipe_plan_spectra(pipe_plan_t p, void* out, void* stream) {
    if (!reg_has(p)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed plan handle");
    if (!out) return fail(PIPE_ERR_INVALID_ARG, "out must be non-null");
    hipStream_t st = (hipStream_t)stream;
    if (p->band >= 0)
        HIP_TRY(hipMemcpyAsync(out, p->table, p->table_elems * p->rb, hipMemcpyDeviceToDevice, st), "spectra copy");
    else
        HIP_TRY(launch_untile(p->table, p->nyq, out, p->rb, p->lx, p->ly, p->nh, p->tile, st, p->nval),
                "spectra copy");
    HIP_TRY(hipStreamSynchronize(st), "spectra copy");
    return PIPE_OK;
}

pipe_status_t pipe_fft3d(int real_bytes, int n0, int n1, int n2, const char* dirs, const void* in, void* out,
                         void* stream) {
    if (real_bytes != 4 && real_bytes != 8) return fail(PIPE_ERR_INVALID_ARG, "real_bytes must be 4 or 8");
    if (!dirs || strlen(dirs) != 3) return fail(PIPE_ERR_INVALID_ARG, "dirs must be three characters");
    for (int i = 0; i < 3; ++i)
        if (dirs[i] != 'f' && dirs[i] != 'b') return fail(PIPE_ERR_INVALID_ARG, "dirs[%d] must be 'f' or 'b'", i);
    if (n0 < 1 || n1 < 1 || n2 < 1) return fail(PIPE_ERR_INVALID_ARG, "sizes must be >= 1");
    const int n[3] = {n0, n1, n2};
    for (int i = 0; i < 3; ++i)
        if (!fft_length_ok(n[i])) return fail(PIPE_ERR_UNSUPPORTED_SIZE, "length %d not supported", n[i]);
    if (!in || !out) return fail(PIPE_ERR_INVALID_ARG, "null pointer");
    const size_t bytes = (size_t)n0 * n1 * n2 * 2 * real_bytes;
    if (in != out && overlaps(in, bytes, out, bytes)) return fail(PIPE_ERR_ALIASING, "in and out overlap");
    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PIPE_ERR_NO_DEVICE, "no HIP device available");
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DeviceCtx* ctx = nullptr;
    pipe_status_t s = device_ctx(dev, &ctx);
    if (s != PIPE_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const long plane = (long)n1 * n2;
    // last dimension: contiguous lines (in -> out); then the other two in place on out
    auto run = [&](auto zero) -> pipe_status_t {
        using real = decltype(zero);
        HIP_TRY(launch_lines<real>(n2, dirs[2] == 'b', in, out, (long)n0 * n1, ctx->tw, st), "fft3d dimension 2");
        HIP_TRY(launch_strided<real>(n1, dirs[1] == 'b', out, out, n1, n1, n2, n2, n2, plane, plane, n0, ctx->tw, st),
                "fft3d dimension 1");
        HIP_TRY(launch_strided<real>(n0, dirs[0] == 'b', out, out, n0, n0, plane, plane, plane, 0, 0, 1, ctx->tw, st),
                "fft3d dimension 0");
        return PIPE_OK;
    };
    return real_bytes == 8 ? run(0.0) : run(0.0f);
}

pipe_status_t pipe_fft_lines(int real_bytes, int len, int n_in, int howmany, int dir, const void* in, void* out,
                             void* stream) {
    if (real_bytes != 4 && real_bytes != 8) return fail(PIPE_ERR_INVALID_ARG, "real_bytes must be 4 or 8");
    if (!fft_length_ok(len)) return fail(PIPE_ERR_UNSUPPORTED_SIZE, "length %d not supported", len);
    if (n_in < 1 || n_in > len || howmany < 1) return fail(PIPE_ERR_INVALID_ARG, "bad n_in or howmany");
    if (dir != -1 && dir != 1) return fail(PIPE_ERR_INVALID_ARG, "dir must be -1 or +1");
    if (!in || !out) return fail(PIPE_ERR_INVALID_ARG, "null pointer");
    int dev = 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PIPE_ERR_NO_DEVICE, "no HIP device available");
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DeviceCtx* ctx = nullptr;
    pipe_status_t s = device_ctx(dev, &ctx);
    if (s != PIPE_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (real_bytes == 8)
        HIP_TRY(launch_strided<double>(len, dir > 0, in, out, n_in, len, 1, 1, 1, n_in, len, howmany, ctx->tw, st),
                "fft lines");
    else
        HIP_TRY(launch_strided<float>(len, dir > 0, in, out, n_in, len, 1, 1, 1, n_in, len, howmany, ctx->tw, st),
                "fft lines");
    return PIPE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
//
// Members with the same mesh (sizes and padded lengths) form a shape group;
// each of the five passes runs once per group as a grouped launch
// (blockIdx.z = member, per-member pointers from a device array of GroupArgs).
// The groups are independent branches of one captured HIP graph, so the
// passes of different shapes run concurrently.  Every member has its own
// slice of the workspace.

struct pipe_batch_s {
    struct Group {
        std::vector<int> members;
        pipe_plan_t rep;   // representative plan (sizes, lengths, precision)
        bool banded = false;   // one banded plan: its own three passes, not grouped launches
    };
    std::vector<pipe_plan_t> plans;
    std::vector<Group> groups;
    std::vector<size_t> ws_off;
    int device = 0, rb = 8;
    size_t ws_bytes = 0;
    GroupArgs* dargs = nullptr;          // device: per group, 5 passes x members
    std::vector<size_t> args_off;        // entry offset of each group's first pass
    std::vector<hipStream_t> streams;    // one per group (fork/join branches of the capture)
    std::vector<hipEvent_t> events;      // fork + one join event per group
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // descriptors: staged in pinned host memory and copied on the caller's
    // stream, so new pointers need no new graph (only the banded members and
    // the vector-access flags are captured as launch arguments)
    GroupArgs* hargs = nullptr;
    size_t nargs = 0;
    hipEvent_t uploaded = nullptr;        // after the last descriptor copy
    hipEvent_t launched = nullptr;        // after the last graph launch
    bool any_upload = false, any_launch = false;
    std::vector<const void*> last_rho;
    std::vector<void*> last_phi;
    void* last_ws = nullptr;
    std::vector<char> cap_flags;          // per group: aligned input, aligned output (as captured)
};

namespace {
void batch_drop_graph(pipe_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void batch_free(pipe_batch_s* b) {
    (void)hipSetDevice(b->device);
    // wait for this batch's own work only (its last replay and descriptor copy)
    if (b->any_launch) (void)hipEventSynchronize(b->launched);
    if (b->any_upload) (void)hipEventSynchronize(b->uploaded);
    batch_drop_graph(b);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->launched) (void)hipEventDestroy(b->launched);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->dargs) (void)hipFree(b->dargs);
    if (b->hargs) (void)hipHostFree(b->hargs);
    delete b;
}

template <typename real>
// shared_table: every member solves on the same plan (many charges, one spectra table).
pipe_status_t launch_group(pipe_plan_s* p, const GroupArgs* args, int n, bool al_in, bool al_out, hipStream_t st,
                           bool shared_table) {
    const int nx = p->nx, ny = p->ny, nz = p->nz, ly = p->ly, nh = p->nh;
    const TwiddleBank& tw = p->ctx->tw;
    const real scale = (real)0;  // taken from each member's GroupArgs
    const long p1 = a1_pitch(p);
    HIP_TRY(launch_z_r2c<real>(nh, nullptr, nz, nz, nullptr, p1, (long)nx * ny, tw, st, args, n, al_in, p->zcap),
            "grouped z forward pass");
    const long pa = a2_pitch(nh, p->apad);
    HIP_TRY(launch_strided<real>(ly, false, nullptr, nullptr, ny, ly, p1, (long)nx * pa, nh, (long)ny * p1, pa, nx,
                                 tw, st, args + n, n),
            "grouped y forward pass");
    HIP_TRY(launch_xprod<real>(p->lx, false, nullptr, nx, ly, nh, pa, p->tile, p->xnt != 0, nullptr, nullptr, tw,
                               st, args + 2 * n, n, shared_table, p->nval),
            "grouped x pass with spectral product");
    HIP_TRY(launch_strided<real>(ly, true, nullptr, nullptr, ly, ny, (long)nx * pa, p1, nh, pa, (long)ny * p1, nx,
                                 tw, st, args + 3 * n, n),
            "grouped y inverse pass");
    HIP_TRY(launch_z_c2r<real>(nh, nullptr, p1, nullptr, nz, nz, (long)nx * ny, scale, tw, st, args + 4 * n, n,
                               al_out, p->zcap),
            "grouped z inverse pass");
    return PIPE_OK;
}
}  // namespace

extern "C" {

pipe_status_t pipe_batch_create(const pipe_plan_t* plans, int count, pipe_batch_t* out) {
    if (!out) return fail(PIPE_ERR_INVALID_ARG, "out must be non-null");
    *out = nullptr;
    if (!plans || count < 1) return fail(PIPE_ERR_INVALID_ARG, "need at least one plan");
    for (int i = 0; i < count; ++i)
        if (!reg_has(plans[i])) return fail(PIPE_ERR_INVALID_ARG, "plan %d is not a live plan", i);
    for (int i = 1; i < count; ++i)
        if (plans[i]->rb != plans[0]->rb || plans[i]->device != plans[0]->device)
            return fail(PIPE_ERR_INVALID_ARG, "batch members must share precision and device");
    pipe_batch_s* b = new pipe_batch_s();
    b->plans.assign(plans, plans + count);
    b->device = plans[0]->device;
    b->rb = plans[0]->rb;
    for (int i = 0; i < count; ++i) {
        pipe_plan_s* p = plans[i];
        int g = -1;
        for (size_t k = 0; p->band < 0 && k < b->groups.size(); ++k) {
            pipe_plan_s* r = b->groups[k].rep;
            if (!b->groups[k].banded && r->nx == p->nx && r->ny == p->ny && r->nz == p->nz && r->lx == p->lx &&
                r->ly == p->ly && r->lz == p->lz && r->nval == p->nval && r->tile == p->tile &&
                r->apad == p->apad && r->zcap == p->zcap && r->xnt == p->xnt && r->a1pad == p->a1pad)
                g = (int)k;
        }
        if (g < 0) {
            b->groups.push_back({{}, p, p->band >= 0});
            g = (int)b->groups.size() - 1;
        }
        b->groups[g].members.push_back(i);
        b->ws_off.push_back(b->ws_bytes);
        b->ws_bytes += align256(p->ws_bytes);
    }
    size_t entries = 0;
    for (auto& g : b->groups) {
        b->args_off.push_back(entries);
        entries += 5 * g.members.size();
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != b->device) e = hipSetDevice(b->device);
    b->nargs = entries;
    if (e == hipSuccess) e = dev_alloc((void**)&b->dargs, entries * sizeof(GroupArgs));
    if (e == hipSuccess && fault_inject_alloc()) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->hargs, entries * sizeof(GroupArgs), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->launched, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (size_t k = 0; e == hipSuccess && k < b->groups.size(); ++k) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) b->streams.push_back(st);
    }
    for (size_t k = 0; e == hipSuccess && k < b->groups.size() + 1; ++k) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->events.push_back(ev);
    }
    if (cur >= 0 && cur != b->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch setup");
    }
    reg_add(b);
    *out = b;
    return PIPE_OK;
}

pipe_status_t pipe_batch_workspace(pipe_batch_t b, size_t* bytes) {
    if (!reg_has(b)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed batch handle");
    if (!bytes) return fail(PIPE_ERR_INVALID_ARG, "bytes must be non-null");
    *bytes = b->ws_bytes;
    return PIPE_OK;
}

pipe_status_t pipe_batch_solve(pipe_batch_t b, const void* const* rho, void* const* phi, void* ws, void* stream) {
    if (!reg_has(b)) return fail(PIPE_ERR_INVALID_ARG, "invalid or destroyed batch handle");
    if (!rho || !phi || !ws) return fail(PIPE_ERR_INVALID_ARG, "null array");
    if (((uintptr_t)ws) & 255) return fail(PIPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const size_t n = b->plans.size();
    for (size_t i = 0; i < n; ++i) {
        pipe_plan_s* p = b->plans[i];
        if (!reg_has(p)) return fail(PIPE_ERR_INVALID_ARG, "member plan %zu was destroyed", i);
        if (!rho[i] || !phi[i]) return fail(PIPE_ERR_INVALID_ARG, "member %zu: null rho or phi", i);
        if (((uintptr_t)rho[i]) % p->rb || ((uintptr_t)phi[i]) % p->rb)
            return fail(PIPE_ERR_INVALID_ARG, "member %zu: rho and phi must be aligned to the element size", i);
        const size_t nb = (size_t)p->nx * p->ny * p->nz * p->rb;
        if (overlaps(rho[i], nb, phi[i], nb)) return fail(PIPE_ERR_ALIASING, "member %zu: rho and phi overlap", i);
        if (overlaps(rho[i], nb, ws, b->ws_bytes) || overlaps(phi[i], nb, ws, b->ws_bytes))
            return fail(PIPE_ERR_ALIASING, "member %zu: workspace overlaps rho or phi", i);
    }
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != b->device) HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    hipStream_t caller = (hipStream_t)stream;
    bool same = b->exec && b->last_ws == ws;
    for (size_t i = 0; same && i < n; ++i) same = b->last_rho[i] == rho[i] && b->last_phi[i] == phi[i];
    pipe_status_t s = PIPE_OK;
    if (!same) {
        // per-member pointers of the five grouped passes
        std::vector<GroupArgs> host;
        std::vector<char> flags;
        bool banded_moved = false;
        for (auto& g : b->groups) {
            const size_t m = g.members.size();
            bool al_in = true, al_out = true;
            for (int i : g.members) {
                al_in = al_in && ((uintptr_t)rho[i] % (2 * b->rb) == 0);
                al_out = al_out && ((uintptr_t)phi[i] % (2 * b->rb) == 0);
            }
            flags.push_back((char)(al_in | (al_out << 1)));
            if (g.banded) {   // launched directly with its own pointers
                const int i = g.members[0];
                if (!b->exec || b->last_ws != ws || b->last_rho[i] != rho[i] || b->last_phi[i] != phi[i])
                    banded_moved = true;
                host.insert(host.end(), 5 * m, GroupArgs{nullptr, nullptr, nullptr, nullptr, 0.0});
                continue;
            }
            std::vector<GroupArgs> a(5 * m);
            for (size_t k = 0; k < m; ++k) {
                const int i = g.members[k];
                pipe_plan_s* p = b->plans[i];
                char* A1 = (char*)ws + b->ws_off[i];
                char* A2 = A1 + align256((size_t)p->nx * p->ny * a1_pitch(p) * 2 * p->rb);
                const double scale = p->hx * p->hy * p->hz / ((double)p->lx * p->ly * p->lz);
                a[0 * m + k] = {rho[i], A1, nullptr, nullptr, 0.0};
                a[1 * m + k] = {A1, A2, nullptr, nullptr, 0.0};
                a[2 * m + k] = {A2, A2, p->table, p->nyq, 0.0};
                a[3 * m + k] = {A2, A1, nullptr, nullptr, 0.0};
                a[4 * m + k] = {A1, phi[i], nullptr, nullptr, scale};
            }
            host.insert(host.end(), a.begin(), a.end());
        }
        const bool recapture = !b->exec || banded_moved || flags != b->cap_flags;
        hipError_t e = hipSuccess;
        // The staging buffer may still feed the previous copy; the device array may
        // still be read by the previous replay (possibly on another stream).
        if (b->any_upload) e = hipEventSynchronize(b->uploaded);
        if (e == hipSuccess && b->any_launch) e = hipStreamWaitEvent(caller, b->launched, 0);
        if (e == hipSuccess) {
            memcpy(b->hargs, host.data(), host.size() * sizeof(GroupArgs));
            e = hipMemcpyAsync(b->dargs, b->hargs, host.size() * sizeof(GroupArgs), hipMemcpyHostToDevice, caller);
        }
        if (e == hipSuccess) e = hipEventRecord(b->uploaded, caller);
        if (e == hipSuccess) b->any_upload = true;
        if (e != hipSuccess) s = hip_fail(e, "batch descriptor upload");
        if (s == PIPE_OK && recapture) {
            // an earlier replay of the old graph may still run
            if (b->any_launch) e = hipEventSynchronize(b->launched);
            if (e != hipSuccess) s = hip_fail(e, "batch graph wait");
            if (s == PIPE_OK) batch_drop_graph(b);
            if (s == PIPE_OK) {
                e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
                if (e != hipSuccess) s = hip_fail(e, "graph capture");
            }
        }
        if (s == PIPE_OK && recapture) {
            hipError_t ce = hipEventRecord(b->events[0], b->cap);
            for (size_t k = 0; ce == hipSuccess && s == PIPE_OK && k < b->groups.size(); ++k) {
                auto& g = b->groups[k];
                hipStream_t st = b->streams[k];
                ce = hipStreamWaitEvent(st, b->events[0], 0);
                if (ce != hipSuccess) break;
                bool shared = true;
                for (int i : g.members) shared = shared && b->plans[i] == b->plans[g.members[0]];
                const bool al_in = flags[k] & 1, al_out = (flags[k] >> 1) & 1;
                const GroupArgs* args = b->dargs + b->args_off[k];
                const int m = (int)g.members.size();
                if (g.banded) {
                    const int i = g.members[0];
                    void* mws = (char*)ws + b->ws_off[i];
                    s = b->rb == 8 ? run_band_passes<double>(g.rep, rho[i], phi[i], mws, st, false, nullptr)
                                   : run_band_passes<float>(g.rep, rho[i], phi[i], mws, st, false, nullptr);
                } else {
                    s = b->rb == 8 ? launch_group<double>(g.rep, args, m, al_in, al_out, st, shared && m > 1)
                                   : launch_group<float>(g.rep, args, m, al_in, al_out, st, shared && m > 1);
                }
                if (s != PIPE_OK) break;
                ce = hipEventRecord(b->events[k + 1], st);
                if (ce == hipSuccess) ce = hipStreamWaitEvent(b->cap, b->events[k + 1], 0);
            }
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(b->cap, &g);
            if (s == PIPE_OK && ce != hipSuccess) s = hip_fail(ce, "graph capture (fork/join)");
            if (s == PIPE_OK && ee != hipSuccess) s = hip_fail(ee, "graph capture");
            if (s != PIPE_OK) {
                if (g) (void)hipGraphDestroy(g);
            } else {
                b->graph = g;
                e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    batch_drop_graph(b);
                    s = hip_fail(e, "graph instantiate");
                }
            }
            if (s == PIPE_OK) b->cap_flags = flags;
        }
        if (s == PIPE_OK) {
            b->last_rho.assign(rho, rho + n);
            b->last_phi.assign(phi, phi + n);
            b->last_ws = ws;
        } else {
            b->last_rho.clear();   // force a fresh upload (and capture, if needed) next time
            b->last_phi.clear();
            b->last_ws = nullptr;
        }
    }
    if (s == PIPE_OK) {
        // the descriptors may have been copied on another stream
        hipError_t e = b->any_upload ? hipStreamWaitEvent(caller, b->uploaded, 0) : hipSuccess;
        if (e == hipSuccess) e = hipGraphLaunch(b->exec, caller);
        if (e == hipSuccess) e = hipEventRecord(b->launched, caller);
        if (e == hipSuccess) b->any_launch = true;
        if (e != hipSuccess) s = hip_fail(e, "graph launch");
    }
    if (cur != b->device) (void)hipSetDevice(cur);
    return s;
}

pipe_status_t pipe_batch_destroy(pipe_batch_t b) {
    if (!reg_del(b)) return fail(PIPE_ERR_INVALID_ARG, "invalid or already destroyed batch handle");
    batch_free(b);
    return PIPE_OK;
}

}  // extern "C"
