// The extern "C" entry points of liblaph: argument checks, context state
// layout, and the call sequences of laph_solve / laph_perambulator.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "laph_mg.h"
#include "laph_reduce.h"
#include "laph_solver.h"

namespace laph {

// The last failure message of the calling thread: a fixed buffer, so that
// reporting an out-of-memory failure does not itself allocate.
static thread_local char g_err[1024];
constexpr int kIdentMax = 4096;   // identity tile table in the state buffer (standalone calls)

laph_status set_error(laph_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

laph_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LAPH_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return LAPH_OK;
}

static void compute_layout(Ctx &c) {
    const size_t vh = (size_t)c.g.vh;
    c.sz_g64_pm = round256(144 * vh);
    c.sz_g32_pm = round256(48 * vh);
    c.sz_g16a_pm = round256(16 * vh);
    c.sz_g16b_pm = round256(8 * vh);
    c.sz_cl64_par = round256(576 * vh);
    c.sz_cl32_par = round256(288 * vh);
    size_t off = 0;
    c.off_g64 = off;
    off += 8 * c.sz_g64_pm;
    c.off_g32 = off;
    off += 8 * c.sz_g32_pm;
    c.off_g16a = off;
    off += 8 * c.sz_g16a_pm;
    c.off_g16b = off;
    off += 8 * c.sz_g16b_pm;
    c.off_clov = off;
    off += 2 * c.sz_cl64_par;
    c.off_misc = off;
    off += round256(8 * (size_t)c.n_mass_max) + 256 + round256(3 * kIdentMax * sizeof(int) + 16);
    c.off_inv64 = off;
    off += (size_t)c.n_mass_max * 2 * c.sz_cl64_par;
    c.off_inv32 = off;
    off += (size_t)c.n_mass_max * 2 * c.sz_cl32_par;
    c.state_size = off;
}

// identity tables: slots[i] = i, mass[i] = 0, counts[i] = i
static int *ident_base(const Ctx &c) {
    return reinterpret_cast<int *>(c.state + c.off_misc + round256(8 * (size_t)c.n_mass_max) + 256);
}
static Tiles ident_tiles(const Ctx &c, int n) {
    Tiles t;
    int *b = ident_base(c);
    t.slots = b;
    t.mass = b + kIdentMax;
    t.ntiles = b + 2 * kIdentMax + n;
    t.ntiles_max = n;
    t.nr = 1;
    return t;
}

// Tile table of a standalone stage call, written on the device: slots
// [0, ntiles * nr) = RHS index or -1 past nrhs, then ntiles mass indices, then
// the live tile count.
__global__ void fill_stage_tiles_kernel(int *ints, int nrhs, int nr, int ntiles, int mass_idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ns = ntiles * nr;
    if (i < ns)
        ints[i] = i < nrhs ? i : -1;
    else if (i < ns + ntiles)
        ints[i] = mass_idx;
    else if (i == ns + ntiles)
        ints[i] = ntiles;
}

static laph_status fill_stage_tiles(const Ctx &c, int *d_ints, int nrhs, int nr, int ntiles, int mass_idx) {
    const int n = ntiles * nr + ntiles + 1;
    hipLaunchKernelGGL(fill_stage_tiles_kernel, dim3((n + 255) / 256), dim3(256), 0, c.stream, d_ints, nrhs, nr, ntiles,
                       mass_idx);
    return check_launch("fill_stage_tiles_kernel");
}

// Device scratch of laph_apply_stage_noalloc, for callers that cannot allocate
// device memory: one fixed array per device, alive until the process ends.  Its
// name is a host-side stand-in in host code; the device address of each GPU's
// copy is taken once per device (laph_create, with that device current) and
// only that address is handed to kernels.
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static laph_status scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return set_error(LAPH_ERR_INVALID, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev]) return LAPH_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(LAPH_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_dev[dev] = p;
    return LAPH_OK;
}

}  // namespace laph

using namespace laph;

// Exception barrier of the C ABI: every extern "C" body below is a
// function-try-block whose handlers turn a C++ exception (std::bad_alloc from a
// host container, anything else thrown inside the library) into LAPH_ERR_HOST;
// size queries return 0.  Nothing throws across the boundary.
#define LAPH_CATCH_STATUS                                                                          \
    catch (const std::bad_alloc &) {                                                               \
        return ::laph::set_error(LAPH_ERR_HOST, "out of host memory");                             \
    }                                                                                              \
    catch (const std::exception &e_) {                                                             \
        return ::laph::set_error(LAPH_ERR_HOST, "internal error: %s", e_.what());                  \
    }                                                                                              \
    catch (...) {                                                                                  \
        return ::laph::set_error(LAPH_ERR_HOST, "internal error (unknown exception)");             \
    }
#define LAPH_CATCH_SIZE                                                                            \
    catch (...) {                                                                                  \
        ::laph::set_error(LAPH_ERR_HOST, "host-side failure in a size query");                     \
        return 0;                                                                                  \
    }

static laph_status check_ctx(laph_ctx h, bool need_gauge = false, bool need_clover = false) {
    if (!h) return set_error(LAPH_ERR_INVALID, "null context");
    Ctx *c = reinterpret_cast<Ctx *>(h);
    if (!c->state) return set_error(LAPH_ERR_WORKSPACE, "no state buffer attached (laph_attach_state)");
    if (need_gauge && !c->gauge_loaded) return set_error(LAPH_ERR_INVALID, "no gauge field loaded");
    if (need_clover && c->n_mass <= 0) return set_error(LAPH_ERR_INVALID, "no clover term set (laph_set_clover)");
    return LAPH_OK;
}
static inline Ctx &C(laph_ctx h) { return *reinterpret_cast<Ctx *>(h); }
static bool valid_prec(int p) { return p == LAPH_F64 || p == LAPH_F32 || p == LAPH_F16N; }

extern "C" {

void laph_default_params(laph_solve_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->inner_prec = LAPH_F32;
    p->batched = 1;
    p->delta = 0;
    p->maxiter = 10000;
    p->graph_iters = 8;
    p->use_graph = 1;
    p->rhs_tile = 0;
    p->chunk = 0;
    p->stencil = 0;
    p->traversal = 0;
    p->stencil64 = 0;
    p->rhs_tile64 = 0;
}

const char *laph_last_error(void) { return g_err; }

laph_status laph_create(laph_ctx *out, const int dims[4], int t_antiperiodic, int n_mass_max, void *hip_stream) try {
    if (!out || !dims) return set_error(LAPH_ERR_INVALID, "null argument");
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 4 || dims[i] % 2) return set_error(LAPH_ERR_INVALID, "extent %d = %d must be even and >= 4", i, dims[i]);
    const double vol = (double)dims[0] * dims[1] * dims[2] * dims[3];
    if (vol * 12 >= 2147483647.0) return set_error(LAPH_ERR_INVALID, "lattice too large for 32-bit site indices");
    if (n_mass_max < 1 || n_mass_max > 64) return set_error(LAPH_ERR_INVALID, "n_mass_max must be in 1..64");
    std::unique_ptr<Ctx> c(new Ctx());
    for (int i = 0; i < 4; ++i) c->dims[i] = dims[i];
    c->g.lx = dims[0];
    c->g.ly = dims[1];
    c->g.lz = dims[2];
    c->g.lt = dims[3];
    c->g.lxh = dims[0] / 2;
    c->g.vh = (int)(vol / 2);
    c->g.vs_h = dims[0] * dims[1] * dims[2] / 2;
    c->g.antiperiodic = t_antiperiodic ? 1 : 0;
    c->n_mass_max = n_mass_max;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    compute_layout(*c);
    {
        int d = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&d) == hipSuccess && hipGetDeviceProperties(&prop, d) == hipSuccess) {
            c->device = d;
            LAPH_TRY(scratch_setup(d));   // the no-allocation entry point's device scratch
            size_t k = 0;
            while (k + 1 < sizeof(c->arch) && prop.gcnArchName[k] && prop.gcnArchName[k] != ':') {
                c->arch[k] = prop.gcnArchName[k];
                ++k;
            }
            c->arch[k] = 0;
        } else {
            (void)hipGetLastError();
        }
    }
    load_tune_cache(*c);
    for (int i = 0; i < 4; ++i) {
        hipError_t e = hipEventCreate(&c->ev[i]);
        if (e != hipSuccess) return set_error(LAPH_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    *out = reinterpret_cast<laph_ctx>(c.release());
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_destroy(laph_ctx h) try {
    if (!h) return LAPH_OK;
    Ctx *c = reinterpret_cast<Ctx *>(h);
    for (int i = 0; i < 4; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    delete c;
    return LAPH_OK;
} LAPH_CATCH_STATUS

size_t laph_state_bytes(laph_ctx h) { return h ? C(h).state_size : 0; }

laph_status laph_attach_state(laph_ctx h, void *dev, size_t bytes) try {
    if (!h || !dev) return set_error(LAPH_ERR_INVALID, "null argument");
    Ctx &c = C(h);
    if (bytes < c.state_size) return set_error(LAPH_ERR_WORKSPACE, "state buffer too small: %zu < %zu", bytes, c.state_size);
    if (reinterpret_cast<uintptr_t>(dev) % 256) return set_error(LAPH_ERR_INVALID, "state buffer must be 256-byte aligned");
    c.state = reinterpret_cast<char *>(dev);
    for (int p = 0; p < 2; ++p)
        for (int mu = 0; mu < 4; ++mu) {
            const int i = p * 4 + mu;
            c.gp.f64[p][mu] = c.state + c.off_g64 + i * c.sz_g64_pm;
            c.gp.f32[p][mu] = c.state + c.off_g32 + i * c.sz_g32_pm;
            c.gp.f16a[p][mu] = c.state + c.off_g16a + i * c.sz_g16a_pm;
            c.gp.f16b[p][mu] = c.state + c.off_g16b + i * c.sz_g16b_pm;
        }
    std::vector<int> ident(3 * kIdentMax);
    for (int i = 0; i < kIdentMax; ++i) {
        ident[i] = i;
        ident[kIdentMax + i] = 0;
        ident[2 * kIdentMax + i] = i;
    }
    LAPH_HIP(hipMemcpyAsync(ident_base(c), ident.data(), ident.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    c.gauge_loaded = false;
    c.n_mass = 0;
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_load_gauge(laph_ctx h, const double *U) try {
    LAPH_TRY(check_ctx(h));
    if (!U) return set_error(LAPH_ERR_INVALID, "null gauge pointer");
    C(h).mgs.ready = false;   // an attached multigrid was built on the previous field
    return load_gauge(C(h), U);
} LAPH_CATCH_STATUS

laph_status laph_set_clover(laph_ctx h, double csw, int n_mass, const double *m0_host) try {
    LAPH_TRY(check_ctx(h, true));
    Ctx &c = C(h);
    if (n_mass < 1 || n_mass > c.n_mass_max || !m0_host)
        return set_error(LAPH_ERR_INVALID, "n_mass must be in 1..%d", c.n_mass_max);
    for (int i = 0; i < n_mass; ++i)
        if (!std::isfinite(m0_host[i]) || 4.0 + m0_host[i] <= 0)
            return set_error(LAPH_ERR_INVALID, "mass %d: 4 + m0 must be positive", i);
    if (!std::isfinite(csw)) return set_error(LAPH_ERR_INVALID, "c_sw not finite");
    c.mgs.ready = false;   // an attached multigrid was built on the previous clover term
    return build_clover(c, csw, n_mass, m0_host);
} LAPH_CATCH_STATUS

size_t laph_field_bytes(laph_ctx h, int prec, int nrhs, int parity_only) try {
    if (!h || !valid_prec(prec) || nrhs < 0) return 0;
    return (size_t)nrhs * (parity_only ? 1 : 2) * C(h).hv(prec);
} LAPH_CATCH_SIZE

static laph_status pack_common(laph_ctx h, int prec, int nrhs, int parity) {
    LAPH_TRY(check_ctx(h));
    if (!valid_prec(prec)) return set_error(LAPH_ERR_INVALID, "bad precision %d", prec);
    if (nrhs < 0 || nrhs > 65535) return set_error(LAPH_ERR_INVALID, "nrhs out of range");
    if (parity < -1 || parity > 1) return set_error(LAPH_ERR_INVALID, "parity must be -1, 0 or 1");
    return LAPH_OK;
}

laph_status laph_pack_spinor(laph_ctx h, void *out, const double *in, int prec, int nrhs, int parity) try {
    LAPH_TRY(pack_common(h, prec, nrhs, parity));
    if (nrhs && (!out || !in)) return set_error(LAPH_ERR_INVALID, "null field pointer");
    Ctx &c = C(h);
    Operand o;
    o.base = reinterpret_cast<char *>(out);
    o.stride = (parity < 0 ? 2 : 1) * c.hv(prec);
    return pack_spinor(c, o, in, prec, nrhs, parity);
} LAPH_CATCH_STATUS

laph_status laph_unpack_spinor(laph_ctx h, double *out, const void *in, int prec, int nrhs, int parity) try {
    LAPH_TRY(pack_common(h, prec, nrhs, parity));
    if (nrhs && (!out || !in)) return set_error(LAPH_ERR_INVALID, "null field pointer");
    Ctx &c = C(h);
    Operand i;
    i.base = reinterpret_cast<char *>(const_cast<void *>(in));
    i.stride = (parity < 0 ? 2 : 1) * c.hv(prec);
    return unpack_spinor(c, out, i, prec, nrhs, parity);
} LAPH_CATCH_STATUS

laph_status laph_apply_dslash(laph_ctx h, void *out, const void *in, int out_parity, int prec, int nrhs, int dagger) try {
    LAPH_TRY(check_ctx(h, true));
    if (!valid_prec(prec) || (out_parity != 0 && out_parity != 1) || nrhs < 0)
        return set_error(LAPH_ERR_INVALID, "bad precision, parity or nrhs");
    if (nrhs && (!out || !in)) return set_error(LAPH_ERR_INVALID, "null field pointer");
    if (out == in && nrhs) return set_error(LAPH_ERR_INVALID, "apply_dslash cannot run in place");
    Ctx &c = C(h);
    const size_t hv = c.hv(prec);
    for (int r0 = 0; r0 < nrhs; r0 += kIdentMax) {
        const int n = std::min(kIdentMax, nrhs - r0);
        StageSpec s;
        s.prec = prec;
        s.out_parity = out_parity;
        s.dagger = dagger ? 1 : 0;
        s.in.base = reinterpret_cast<char *>(const_cast<void *>(in)) + r0 * hv;
        s.in.stride = hv;
        s.out.base = reinterpret_cast<char *>(out) + r0 * hv;
        s.out.stride = hv;
        s.tiles = ident_tiles(c, n);
        LAPH_TRY(launch_stage(c, s));
    }
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_apply_clover(laph_ctx h, void *out, const void *in, int parity, int mass_idx, int inverse, int prec,
                              int nrhs) try {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    if (!valid_prec(prec) || (parity != 0 && parity != 1) || nrhs < 0 || mass_idx < 0 || mass_idx >= c.n_mass)
        return set_error(LAPH_ERR_INVALID, "bad precision, parity, mass index or nrhs");
    if (nrhs && (!out || !in)) return set_error(LAPH_ERR_INVALID, "null field pointer");
    if (nrhs > 65535) return set_error(LAPH_ERR_INVALID, "nrhs out of range");
    CloverSpec s;
    s.prec = prec;
    s.parity = parity;
    s.inverse = inverse ? 1 : 0;
    s.in.base = reinterpret_cast<char *>(const_cast<void *>(in));
    s.in.stride = c.hv(prec);
    s.out.base = reinterpret_cast<char *>(out);
    s.out.stride = c.hv(prec);
    s.mass_idx = mass_idx;
    s.n = nrhs;
    return launch_clover(c, s);
} LAPH_CATCH_STATUS

laph_status laph_apply_D(laph_ctx h, double *out, const double *in, int mass_idx, int nrhs, int dagger, void *work,
                         size_t work_bytes) {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    if (nrhs < 0 || mass_idx < 0 || mass_idx >= c.n_mass) return set_error(LAPH_ERR_INVALID, "bad mass index or nrhs");
    if (nrhs && (!out || !in)) return set_error(LAPH_ERR_INVALID, "null field pointer");
    const size_t hv = c.hv(LAPH_F64);
    if (!work || work_bytes < 4 * hv) return set_error(LAPH_ERR_WORKSPACE, "apply_D workspace too small");
    char *w = reinterpret_cast<char *>(work);
    Operand ie{w, 0}, io{w + hv, 0}, oe{w + 2 * hv, 0}, oo{w + 3 * hv, 0};
    const size_t full = (size_t)2 * c.g.vh * 12 * 2;   // doubles per canonical RHS
    for (int r = 0; r < nrhs; ++r) {
        const double *src = in + r * full;
        double *dst = out + r * full;
        LAPH_TRY(pack_spinor(c, ie, src, LAPH_F64, 1, 0));
        LAPH_TRY(pack_spinor(c, io, src, LAPH_F64, 1, 1));
        for (int p = 0; p < 2; ++p) {
            const Operand &xin = p == 0 ? ie : io, &xother = p == 0 ? io : ie, &o = p == 0 ? oe : oo;
            CloverSpec cs;
            cs.prec = LAPH_F64;
            cs.parity = p;
            cs.inverse = 0;
            cs.in = xin;
            cs.out = o;
            cs.mass_idx = mass_idx;
            cs.n = 1;
            LAPH_TRY(launch_clover(c, cs));
            StageSpec s;
            s.prec = LAPH_F64;
            s.out_parity = p;
            s.dagger = dagger ? 1 : 0;
            s.post = 1;
            s.in = xother;
            s.out = o;
            s.y = o;
            s.a = 1.0;
            s.b = -0.5;
            s.tiles = ident_tiles(c, 1);
            LAPH_TRY(launch_stage(c, s));
        }
        LAPH_TRY(unpack_spinor(c, dst, oe, LAPH_F64, 1, 0));
        LAPH_TRY(unpack_spinor(c, dst, oo, LAPH_F64, 1, 1));
    }
    return LAPH_OK;
}

static laph_status check_params(const laph_solve_params *p, double tol) {
    if (!p) return set_error(LAPH_ERR_INVALID, "null params");
    if (!valid_prec(p->inner_prec)) return set_error(LAPH_ERR_INVALID, "bad inner precision");
    if (!(tol > 0) || !std::isfinite(tol)) return set_error(LAPH_ERR_INVALID, "tol must be positive");
    if (p->rhs_tile > 0 && p->rhs_tile != 1 && p->rhs_tile != 2 && p->rhs_tile != 4 && p->rhs_tile != 8 &&
        p->rhs_tile != 16)
        return set_error(LAPH_ERR_INVALID, "rhs_tile must be 1, 2, 4 (register tiles) or 4, 8, 16 (LDS links)");
    if (p->rhs_tile64 > 0 && p->rhs_tile64 != 1 && p->rhs_tile64 != 2 && p->rhs_tile64 != 4 &&
        p->rhs_tile64 != 8 && p->rhs_tile64 != 16)
        return set_error(LAPH_ERR_INVALID, "rhs_tile64 must be 1, 2, 4 (register tiles) or 4, 8, 16 (LDS links)");
    if (p->stencil < 0 || p->stencil > 2 || p->traversal < 0 || p->traversal > 2 || p->stencil64 < 0 ||
        p->stencil64 > 2)
        return set_error(LAPH_ERR_INVALID, "stencil, stencil64 and traversal must be 0, 1 or 2");
    return LAPH_OK;
}

size_t laph_solve_workspace_bytes(laph_ctx h, int nrhs, const laph_solve_params *p) try {
    if (!h || !p || nrhs <= 0) return 0;
    return solver_workspace_bytes(C(h), p->batched ? nrhs : 1, *p);
} LAPH_CATCH_SIZE

laph_status laph_solve(laph_ctx h, double *X, const double *B, int nrhs, const int *mass_idx_host, double tol,
                       const laph_solve_params *p, laph_rhs_stats *stats_host, void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h, true, true));
    LAPH_TRY(check_params(p, tol));
    Ctx &c = C(h);
    if (nrhs <= 0 || nrhs > 65535) return set_error(LAPH_ERR_INVALID, "nrhs out of range");
    if (!X || !B) return set_error(LAPH_ERR_INVALID, "null X or B");
    std::vector<int> mass(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) {
        mass[r] = mass_idx_host ? mass_idx_host[r] : 0;
        if (mass[r] < 0 || mass[r] >= c.n_mass) return set_error(LAPH_ERR_INVALID, "mass index %d out of range", mass[r]);
    }
    const int ns = p->batched ? nrhs : 1;
    Solver solver;
    LAPH_TRY(solver.init(c, ns, *p, reinterpret_cast<char *>(work), work_bytes, mass[0]));
    const size_t full = (size_t)2 * c.g.vh * 12;   // complex elements per RHS
    LAPH_HIP(hipEventRecord(c.ev[0], c.stream));
    int worst = LAPH_OK;
    for (int r0 = 0; r0 < nrhs; r0 += ns) {
        const int n = std::min(ns, nrhs - r0);
        SourceSpec src;
        src.B = B + r0 * full * 2;
        src.B_stride = full;
        src.n = n;
        std::vector<int> m(mass.begin() + r0, mass.begin() + r0 + n);
        LAPH_TRY(solver.solve(src, m, tol, p->use_x0 ? X + r0 * full * 2 : nullptr, full));
        const auto &ws = solver.workspace();
        LAPH_TRY(unpack_spinor(c, X + r0 * full * 2, ws.E1, LAPH_F64, n, 0, full));
        LAPH_TRY(unpack_spinor(c, X + r0 * full * 2, ws.O0, LAPH_F64, n, 1, full));
        int w = LAPH_OK;
        LAPH_TRY(solver.collect(stats_host ? stats_host + r0 : nullptr, n, tol, &w));
        if (w != LAPH_OK && (worst == LAPH_OK || w == LAPH_ERR_NONFINITE)) worst = w;
    }
    LAPH_HIP(hipEventRecord(c.ev[1], c.stream));
    LAPH_HIP(hipEventSynchronize(c.ev[1]));
    float ms = 0;
    LAPH_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
    c.last_ms[0] = c.last_ms[1] = ms;
    c.last_ms[2] = 0;
    if (worst != LAPH_OK) return set_error((laph_status)worst, "some right-hand sides did not converge (see stats)");
    return LAPH_OK;
} LAPH_CATCH_STATUS

static int peramb_chunk(int nev, const laph_solve_params *p) {
    const int nrhs = 4 * nev;
    int chunk = p->chunk > 0 ? p->chunk : std::min(nrhs, 128);
    if (!p->batched) chunk = 1;
    return std::min(chunk, nrhs);
}

size_t laph_perambulator_workspace_bytes(laph_ctx h, int nev, const laph_solve_params *p) try {
    if (!h || !p || nev <= 0) return 0;
    Ctx &c = C(h);
    const int chunk = peramb_chunk(nev, p);
    return packed_v_bytes(c, nev) + project_scratch_bytes(c, nev, chunk) + solver_workspace_bytes(c, chunk, *p);
} LAPH_CATCH_SIZE

// sources -> batched solves -> projection, streamed in RHS chunks: the perambulator's
// 4 nev sources (rho null) or 4 n_dil diluted noise sources
static laph_status peramb_run(laph_ctx h, double *tau, const double *V, int nev, int t0, int mass_idx,
                              const double *rho, int n_dil, double tol, const laph_solve_params *p,
                              laph_rhs_stats *stats_host, void *work, size_t work_bytes) {
    LAPH_TRY(check_ctx(h, true, true));
    LAPH_TRY(check_params(p, tol));
    Ctx &c = C(h);
    if (!tau || !V) return set_error(LAPH_ERR_INVALID, "null tau or V");
    if (nev <= 0 || nev > 64) return set_error(LAPH_ERR_INVALID, "nev must be in 1..64");
    if (t0 < 0 || t0 >= c.g.lt) return set_error(LAPH_ERR_INVALID, "t0 out of range");
    if (mass_idx < 0 || mass_idx >= c.n_mass) return set_error(LAPH_ERR_INVALID, "mass index out of range");
    if (p->use_x0) return set_error(LAPH_ERR_INVALID, "use_x0 is not available for laph_perambulator");
    const int nsrc = rho ? n_dil : nev;
    const int chunk = peramb_chunk(nsrc, p);
    const size_t need = laph_perambulator_workspace_bytes(h, nev, p);
    if (!work || work_bytes < need) return set_error(LAPH_ERR_WORKSPACE, "perambulator workspace too small: %zu < %zu", work_bytes, need);
    char *w = reinterpret_cast<char *>(work);
    double *Vp = reinterpret_cast<double *>(w);
    double *scratch = reinterpret_cast<double *>(w + packed_v_bytes(c, nev));
    char *swork = w + packed_v_bytes(c, nev) + project_scratch_bytes(c, nev, chunk);
    Solver solver;
    LAPH_TRY(solver.init(c, chunk, *p, swork, need - (swork - w), mass_idx));
    const int nrhs = 4 * nsrc;
    double ms_solve = 0, ms_proj = 0;
    LAPH_HIP(hipEventRecord(c.ev[0], c.stream));
    LAPH_TRY(pack_laph_vectors(c, Vp, V, nev));
    int worst = LAPH_OK;
    for (int r0 = 0; r0 < nrhs; r0 += chunk) {
        const int n = std::min(chunk, nrhs - r0);
        SourceSpec src;
        src.V = V;
        src.nev = nev;
        src.t0 = t0;
        src.r_begin = r0;
        src.n = n;
        src.rho = rho;
        src.n_dil = n_dil;
        LAPH_HIP(hipEventRecord(c.ev[2], c.stream));
        LAPH_TRY(solver.solve(src, std::vector<int>(n, mass_idx), tol, nullptr, 0));
        LAPH_HIP(hipEventRecord(c.ev[3], c.stream));
        ProjectSpec ps;
        ps.xe = solver.workspace().E1;
        ps.xo = solver.workspace().O0;
        ps.n = n;
        ps.r_begin = r0;
        ps.Vp = Vp;
        ps.nev = nev;
        ps.nev_src = nsrc;
        ps.tau = tau;
        ps.scratch = scratch;
        LAPH_TRY(project(c, ps));
        LAPH_HIP(hipEventRecord(c.ev[1], c.stream));
        int wst = LAPH_OK;
        LAPH_TRY(solver.collect(stats_host ? stats_host + r0 : nullptr, n, tol, &wst));
        if (wst != LAPH_OK && (worst == LAPH_OK || wst == LAPH_ERR_NONFINITE)) worst = wst;
        float a = 0, b = 0;
        LAPH_HIP(hipEventElapsedTime(&a, c.ev[2], c.ev[3]));
        LAPH_HIP(hipEventElapsedTime(&b, c.ev[3], c.ev[1]));
        ms_solve += a;
        ms_proj += b;
    }
    LAPH_HIP(hipEventRecord(c.ev[1], c.stream));
    LAPH_HIP(hipEventSynchronize(c.ev[1]));
    float ms = 0;
    LAPH_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
    c.last_ms[0] = ms;
    c.last_ms[1] = ms_solve;
    c.last_ms[2] = ms_proj;
    if (worst != LAPH_OK) return set_error((laph_status)worst, "some right-hand sides did not converge (see stats)");
    return LAPH_OK;
}

laph_status laph_perambulator(laph_ctx h, double *tau, const double *V, int nev, int t0, int mass_idx, double tol,
                              const laph_solve_params *p, laph_rhs_stats *stats_host, void *work, size_t work_bytes) try {
    return peramb_run(h, tau, V, nev, t0, mass_idx, nullptr, 0, tol, p, stats_host, work, work_bytes);
} LAPH_CATCH_STATUS

laph_status laph_stochastic_perambulator(laph_ctx h, double *phi, const double *V, int nev, int t0, int mass_idx,
                                         const double *rho, int n_dil, double tol, const laph_solve_params *p,
                                         laph_rhs_stats *stats_host, void *work, size_t work_bytes) try {
    if (!rho) return set_error(LAPH_ERR_INVALID, "null noise");
    if (n_dil < 1 || n_dil > nev) return set_error(LAPH_ERR_INVALID, "n_dil must be in 1..nev");
    return peramb_run(h, phi, V, nev, t0, mass_idx, rho, n_dil, tol, p, stats_host, work, work_bytes);
} LAPH_CATCH_STATUS

size_t laph_laplacian_workspace_bytes(laph_ctx h, int nev) try {
    if (!h || nev < 1 || nev > 64) return 0;
    return laplacian_eig_workspace_bytes(C(h), nev);
} LAPH_CATCH_SIZE

laph_status laph_apply_laplacian(laph_ctx h, double *out, const double *in, int nvec) try {
    LAPH_TRY(check_ctx(h, true, false));
    if (!out || !in || nvec <= 0 || nvec > 65535 || out == in) return set_error(LAPH_ERR_INVALID, "bad arguments");
    return apply_neg_laplacian(C(h), out, in, nvec);
} LAPH_CATCH_STATUS

laph_status laph_laplacian_eigvecs(laph_ctx h, double *V, double *lambda_host, int nev, double tol, int max_iter,
                                   int degree, void *work, size_t work_bytes, int *iters_host,
                                   double *residual_host) try {
    LAPH_TRY(check_ctx(h, true, false));
    if (!V || !lambda_host) return set_error(LAPH_ERR_INVALID, "null V or lambda");
    return laplacian_eigvecs(C(h), V, lambda_host, nev, tol, max_iter, degree, reinterpret_cast<char *>(work),
                             work_bytes, iters_host, residual_host);
} LAPH_CATCH_STATUS

size_t laph_contract_workspace_bytes(laph_ctx h, int kind, int nev, int n_mom) try {
    if (!h) return 0;
    return contract_workspace_bytes(C(h), kind, nev, n_mom);
} LAPH_CATCH_SIZE

static laph_status contract_entry(laph_ctx h, int kind, double *out, const double *V, int nev, int n_mom,
                                  const int *mom_host, void *work, size_t work_bytes) {
    if (!h) return set_error(LAPH_ERR_INVALID, "null context");
    if (!out || !V) return set_error(LAPH_ERR_INVALID, "null output or V");
    return contract(C(h), kind, out, V, nev, n_mom, mom_host, reinterpret_cast<char *>(work), work_bytes);
}

laph_status laph_meson_doublets(laph_ctx h, double *phi, const double *V, int nev, int n_mom, const int *mom_host,
                                void *work, size_t work_bytes) try {
    return contract_entry(h, 0, phi, V, nev, n_mom, mom_host, work, work_bytes);
} LAPH_CATCH_STATUS

laph_status laph_baryon_triplets(laph_ctx h, double *B, const double *V, int nev, int n_mom, const int *mom_host,
                                 void *work, size_t work_bytes) try {
    return contract_entry(h, 1, B, V, nev, n_mom, mom_host, work, work_bytes);
} LAPH_CATCH_STATUS

laph_status laph_make_sources(laph_ctx h, double *B, const double *V, int nev, int t0) try {
    LAPH_TRY(check_ctx(h));
    Ctx &c = C(h);
    if (!B || !V || nev <= 0 || nev > 16383 || t0 < 0 || t0 >= c.g.lt) return set_error(LAPH_ERR_INVALID, "bad arguments");
    return make_sources_canonical(c, B, V, nev, t0);
} LAPH_CATCH_STATUS

laph_status laph_make_noise_sources(laph_ctx h, double *B, const double *V, int nev, int t0, const double *rho,
                                    int n_dil) try {
    LAPH_TRY(check_ctx(h));
    Ctx &c = C(h);
    if (!B || !V || !rho || nev <= 0 || nev > 16383 || t0 < 0 || t0 >= c.g.lt || n_dil < 1 || n_dil > nev)
        return set_error(LAPH_ERR_INVALID, "bad arguments");
    return make_sources_canonical(c, B, V, nev, t0, rho, n_dil);
} LAPH_CATCH_STATUS

size_t laph_project_workspace_bytes(laph_ctx h, int nev, int nev_src) try {
    if (!h || nev <= 0 || nev_src <= 0) return 0;
    Ctx &c = C(h);
    const int n = std::min(4 * nev_src, 128);
    return packed_v_bytes(c, nev) + project_scratch_bytes(c, nev, n) + 2 * (size_t)n * c.hv(LAPH_F64);
} LAPH_CATCH_SIZE

laph_status laph_project(laph_ctx h, double *tau, const double *X, const double *V, int nev, int nev_src, void *work,
                         size_t work_bytes) try {
    LAPH_TRY(check_ctx(h));
    Ctx &c = C(h);
    if (!tau || !X || !V || nev <= 0 || nev > 64 || nev_src <= 0) return set_error(LAPH_ERR_INVALID, "bad arguments");
    const size_t need = laph_project_workspace_bytes(h, nev, nev_src);
    if (!work || work_bytes < need) return set_error(LAPH_ERR_WORKSPACE, "project workspace too small");
    const int chunk = std::min(4 * nev_src, 128);
    char *w = reinterpret_cast<char *>(work);
    double *Vp = reinterpret_cast<double *>(w);
    double *scratch = reinterpret_cast<double *>(w + packed_v_bytes(c, nev));
    char *xw = w + packed_v_bytes(c, nev) + project_scratch_bytes(c, nev, chunk);
    const size_t hv = c.hv(LAPH_F64);
    Operand xe{xw, hv}, xo{xw + (size_t)chunk * hv, hv};
    LAPH_TRY(pack_laph_vectors(c, Vp, V, nev));
    const size_t full = (size_t)2 * c.g.vh * 12;
    for (int r0 = 0; r0 < 4 * nev_src; r0 += chunk) {
        const int n = std::min(chunk, 4 * nev_src - r0);
        LAPH_TRY(pack_spinor(c, xe, X + r0 * full * 2, LAPH_F64, n, 0, full));
        LAPH_TRY(pack_spinor(c, xo, X + r0 * full * 2, LAPH_F64, n, 1, full));
        ProjectSpec ps;
        ps.xe = xe;
        ps.xo = xo;
        ps.n = n;
        ps.r_begin = r0;
        ps.Vp = Vp;
        ps.nev = nev;
        ps.nev_src = nev_src;
        ps.tau = tau;
        ps.scratch = scratch;
        LAPH_TRY(project(c, ps));
    }
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_spin_rotate(laph_ctx h, double *out, const double *tau, long n_blocks, const double *S_host) try {
    if (!h) return set_error(LAPH_ERR_INVALID, "null context");
    if (!out || !tau || !S_host || n_blocks < 0) return set_error(LAPH_ERR_INVALID, "bad arguments");
    return spin_rotate(C(h), out, tau, n_blocks, S_host);
} LAPH_CATCH_STATUS

laph_status laph_project_adjoint(laph_ctx h, double *GX, const double *Gtau, const double *V, int nev, int nev_src) try {
    LAPH_TRY(check_ctx(h));
    if (!GX || !Gtau || !V || nev <= 0 || nev_src <= 0 || nev_src > 16383) return set_error(LAPH_ERR_INVALID, "bad arguments");
    return project_adjoint(C(h), GX, Gtau, V, nev, nev_src);
} LAPH_CATCH_STATUS

static size_t time_stages_layout(const Ctx &c, int prec, int nrhs, size_t *off_ints, size_t *off_part) {
    const size_t hv = c.hv(prec);
    size_t off = 4 * (size_t)nrhs * hv;   // p (even), t (odd), v (even), r^ (even)
    *off_part = off;
    off += round256((size_t)nrhs * 3 * partial_stride(c) * sizeof(double));
    *off_ints = off;
    off += round256(tune_ints(nrhs) * sizeof(int));
    return off;
}

size_t laph_time_stages_workspace_bytes(laph_ctx h, int prec, int nrhs, int rhs_tile) try {
    (void)rhs_tile;
    if (!h || !valid_prec(prec) || nrhs <= 0) return 0;
    size_t a, b;
    return time_stages_layout(C(h), prec, nrhs, &a, &b);
} LAPH_CATCH_SIZE

laph_status laph_time_stages(laph_ctx h, int prec, int nrhs, int stencil, int rhs_tile, int traversal, int mass_idx,
                             int reps, void *work, size_t work_bytes, double *ms_host2) try {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    const int form = stencil == 2 ? kFormLds : kFormRegister;
    const bool tile_ok = form == kFormLds ? (rhs_tile == 4 || rhs_tile == 8 || rhs_tile == 16)
                                          : (rhs_tile == 1 || rhs_tile == 2 || rhs_tile == 4);
    if (!valid_prec(prec) || nrhs <= 0 || nrhs > 65535 || reps <= 0 || !ms_host2 || !tile_ok || mass_idx < 0 ||
        mass_idx >= c.n_mass || (stencil != 1 && stencil != 2) || (traversal != 1 && traversal != 2))
        return set_error(LAPH_ERR_INVALID, "bad arguments");
    size_t off_ints, off_part;
    const size_t need = time_stages_layout(c, prec, nrhs, &off_ints, &off_part);
    if (!work || work_bytes < need) return set_error(LAPH_ERR_WORKSPACE, "workspace too small");
    char *w = reinterpret_cast<char *>(work);
    return time_stage_pair(c, prec, nrhs, form, rhs_tile, traversal == 2 ? 1 : 0, mass_idx, reps, w,
                           reinterpret_cast<double *>(w + off_part), reinterpret_cast<int *>(w + off_ints), ms_host2);
} LAPH_CATCH_STATUS

laph_status laph_autotune(laph_ctx h, int prec, int nrhs, int mass_idx, void *work, size_t work_bytes,
                          int *stencil_out, int *rhs_tile_out, int *traversal_out, double *ms_out) try {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    if (!valid_prec(prec) || nrhs <= 0 || nrhs > 65535 || mass_idx < 0 || mass_idx >= c.n_mass)
        return set_error(LAPH_ERR_INVALID, "bad arguments");
    size_t off_ints, off_part;
    const size_t need = time_stages_layout(c, prec, nrhs, &off_ints, &off_part);
    if (!work || work_bytes < need) return set_error(LAPH_ERR_WORKSPACE, "workspace too small");
    char *w = reinterpret_cast<char *>(work);
    Ctx::Shape sh{};
    LAPH_TRY(autotune_stencil(c, prec, nrhs, mass_idx, w, reinterpret_cast<double *>(w + off_part),
                              reinterpret_cast<int *>(w + off_ints), &sh, ms_out));
    if (stencil_out) *stencil_out = sh.form == kFormLds ? 2 : 1;
    if (rhs_tile_out) *rhs_tile_out = sh.tile;
    if (traversal_out) *traversal_out = sh.site_major ? 2 : 1;
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_last_timings(laph_ctx h, double *ms_host3) try {
    if (!h || !ms_host3) return set_error(LAPH_ERR_INVALID, "null argument");
    for (int i = 0; i < 3; ++i) ms_host3[i] = C(h).last_ms[i];
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_tuned_choice(laph_ctx h, int prec, int nrhs, int *found, int *stencil_out, int *rhs_tile_out,
                              int *traversal_out) try {
    if (!h || !found) return set_error(LAPH_ERR_INVALID, "null argument");
    Ctx &c = C(h);
    auto it = c.tuned.find({prec, nrhs});
    *found = it != c.tuned.end() ? 1 : 0;
    if (*found) {
        if (stencil_out) *stencil_out = it->second.form == kFormLds ? 2 : 1;
        if (rhs_tile_out) *rhs_tile_out = it->second.tile;
        if (traversal_out) *traversal_out = it->second.site_major ? 2 : 1;
    }
    return LAPH_OK;
} LAPH_CATCH_STATUS

static size_t stage_ws_layout(const Ctx &c, int nrhs, size_t *off_part, size_t *off_dots) {
    size_t off = round256(tune_ints(nrhs) * sizeof(int));
    if (off_part) *off_part = off;
    off += round256((size_t)nrhs * 3 * partial_stride(c) * sizeof(double));
    if (off_dots) *off_dots = off;
    off += round256((size_t)nrhs * 3 * sizeof(double));
    return off;
}

static laph_status stage_check(const Ctx &c, int which, void *out, const void *in, const void *y, const void *w,
                               int prec, int nrhs, int mass_idx, int stencil, int rhs_tile, int traversal,
                               const double *dots_host) {
    const int form = stencil == 2 ? kFormLds : kFormRegister;
    const bool tile_ok = form == kFormLds ? (rhs_tile == 4 || rhs_tile == 8 || rhs_tile == 16)
                                          : (rhs_tile == 1 || rhs_tile == 2 || rhs_tile == 4);
    if (which < 1 || which > 3 || !valid_prec(prec) || nrhs <= 0 || nrhs > 65535 || mass_idx < 0 ||
        mass_idx >= c.n_mass || (stencil != 1 && stencil != 2) || (traversal != 1 && traversal != 2) || !tile_ok)
        return set_error(LAPH_ERR_INVALID, "bad stage, precision, nrhs, mass index or launch shape");
    if (!out || !in || (which >= 2 && !y) || (which == 2 && !w) || (which >= 2 && !dots_host))
        return set_error(LAPH_ERR_INVALID, "null field or dots pointer");
    if (out == in || (which >= 2 && (out == y || (which == 2 && out == w))))
        return set_error(LAPH_ERR_INVALID, "out must not alias in, y or w");
    return LAPH_OK;
}

// One fused stage on checked arguments; wk: stage_ws_layout(c, nrhs) bytes of
// device memory (tile table, per-block partials, per-RHS sums).  Nothing here
// allocates: the tile table is written on the device.
static laph_status stage_run(const Ctx &c, int which, void *out, const void *in, const void *y, const void *w,
                             int prec, int nrhs, int mass_idx, int dagger, int stencil, int rhs_tile, int traversal,
                             double *dots_host, char *wk) {
    const int form = stencil == 2 ? kFormLds : kFormRegister;
    size_t off_part, off_dots;
    stage_ws_layout(c, nrhs, &off_part, &off_dots);
    int *d_ints = reinterpret_cast<int *>(wk);
    double *partials = reinterpret_cast<double *>(wk + off_part);
    double *dots = reinterpret_cast<double *>(wk + off_dots);
    // tile table: tile j holds RHS j * rhs_tile .. (ragged last tile padded with -1), all of mass_idx
    const int ntiles = (nrhs + rhs_tile - 1) / rhs_tile;
    LAPH_TRY(fill_stage_tiles(c, d_ints, nrhs, rhs_tile, ntiles, mass_idx));
    Tiles t;
    t.slots = d_ints;
    t.mass = d_ints + (size_t)ntiles * rhs_tile;
    t.ntiles = d_ints + (size_t)ntiles * rhs_tile + ntiles;
    t.ntiles_max = ntiles;
    t.nr = rhs_tile;
    const size_t hv = c.hv(prec);
    auto op = [&](const void *p) { return Operand{reinterpret_cast<char *>(const_cast<void *>(p)), hv}; };
    StageSpec s;
    s.prec = prec;
    s.form = form;
    s.site_major = traversal == 2 ? 1 : 0;
    s.dagger = dagger ? 1 : 0;
    s.clover = 1;
    s.in = op(in);
    s.out = op(out);
    s.tiles = t;
    s.partials = partials;
    s.pstride = partial_stride(c);
    if (which == 1) {
        s.out_parity = 1;
    } else {
        s.out_parity = 0;
        s.post = 1;
        s.y = op(y);
        s.a = 1.0;
        s.b = -0.25;
        s.red = which == 2 ? 1 : 2;
        if (which == 2) s.w = op(w);
    }
    LAPH_TRY(launch_stage(c, s));
    if (which >= 2) {
        const int nq = which == 2 ? 2 : 3;
        LAPH_TRY(sum_stage_partials(c, partials, s.pstride, stage_nsb(c, form), nrhs, nq, dots));
        LAPH_HIP(hipMemcpyAsync(dots_host, dots, (size_t)nrhs * 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        LAPH_HIP(hipStreamSynchronize(c.stream));
        if (which == 2)
            for (int r = 0; r < nrhs; ++r) dots_host[3 * r + 2] = 0.0;
    }
    return LAPH_OK;
}

size_t laph_apply_stage_workspace_bytes(laph_ctx h, int nrhs) try {
    if (!h || nrhs <= 0 || nrhs > 65535) return 0;
    return stage_ws_layout(C(h), nrhs, nullptr, nullptr);
} LAPH_CATCH_SIZE

laph_status laph_apply_stage(laph_ctx h, int which, void *out, const void *in, const void *y, const void *w,
                             int prec, int nrhs, int mass_idx, int dagger, int stencil, int rhs_tile, int traversal,
                             double *dots_host, void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h, true, true));
    LAPH_TRY(stage_check(C(h), which, out, in, y, w, prec, nrhs, mass_idx, stencil, rhs_tile, traversal, dots_host));
    const size_t need = stage_ws_layout(C(h), nrhs, nullptr, nullptr);
    if (!work || work_bytes < need) return set_error(LAPH_ERR_WORKSPACE, "apply_stage workspace too small: %zu < %zu", work_bytes, need);
    return stage_run(C(h), which, out, in, y, w, prec, nrhs, mass_idx, dagger, stencil, rhs_tile, traversal, dots_host,
                     reinterpret_cast<char *>(work));
} LAPH_CATCH_STATUS

laph_status laph_apply_stage_noalloc(laph_ctx h, int which, void *out, const void *in, const void *y, const void *w,
                                     int prec, int nrhs, int mass_idx, int dagger, int stencil, int rhs_tile,
                                     int traversal, double *dots_host) try {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    LAPH_TRY(stage_check(c, which, out, in, y, w, prec, nrhs, mass_idx, stencil, rhs_tile, traversal, dots_host));
    const size_t need = stage_ws_layout(c, nrhs, nullptr, nullptr);
    if (need > kNoallocScratchBytes)
        return set_error(LAPH_ERR_WORKSPACE,
                         "apply_stage_noalloc: %d RHS need %zu bytes of device scratch, above the library's fixed "
                         "%zu bytes (use laph_apply_stage with a workspace, or fewer RHS per call)",
                         nrhs, need, (size_t)kNoallocScratchBytes);
    if (c.device < 0 || c.device >= kMaxDevices || !g_scratch_dev[c.device])
        return set_error(LAPH_ERR_HIP, "apply_stage_noalloc: no device scratch address for device %d", c.device);
    return stage_run(c, which, out, in, y, w, prec, nrhs, mass_idx, dagger, stencil, rhs_tile, traversal, dots_host,
                     reinterpret_cast<char *>(g_scratch_dev[c.device]));
} LAPH_CATCH_STATUS

size_t laph_mass_gradient_workspace_bytes(laph_ctx h) try {
    if (!h) return 0;
    return round256(kGradScratchDoubles * sizeof(double));
} LAPH_CATCH_SIZE

laph_status laph_mass_gradient(laph_ctx h, double *g_host, const double *Z, const double *X, int nrhs, void *work,
                               size_t work_bytes) try {
    if (!h) return set_error(LAPH_ERR_INVALID, "null context");
    Ctx &c = C(h);
    if (!g_host || !Z || !X || nrhs <= 0 || nrhs > 65535) return set_error(LAPH_ERR_INVALID, "bad arguments");
    if (!work || work_bytes < kGradScratchDoubles * sizeof(double))
        return set_error(LAPH_ERR_WORKSPACE, "mass_gradient workspace too small");
    const size_t n = (size_t)nrhs * 2 * c.g.vh * 12;
    return mass_gradient(c, g_host, Z, X, n, reinterpret_cast<double *>(work));
} LAPH_CATCH_STATUS

laph_status laph_stream_copy(laph_ctx h, void *dst, const void *src, size_t bytes, int reps, double *ms_host) try {
    if (!h) return set_error(LAPH_ERR_INVALID, "null context");
    if (!dst || !src || !ms_host || bytes == 0 || bytes % 16 || reps <= 0)
        return set_error(LAPH_ERR_INVALID, "bad arguments (bytes must be a positive multiple of 16)");
    const char *d = reinterpret_cast<const char *>(dst), *sp = reinterpret_cast<const char *>(src);
    if (d < sp + bytes && sp < d + bytes) return set_error(LAPH_ERR_INVALID, "dst and src overlap");
    return stream_copy(C(h), dst, src, bytes, reps, ms_host);
} LAPH_CATCH_STATUS

// ---- two-level aggregation multigrid ----------------------------------------------

void laph_mg_default_params(laph_mg_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nvec = 12;
    for (int i = 0; i < 4; ++i) p->block[i] = 4;
    p->null_passes = 4;
    p->null_tol = 1e-2;
    p->smooth_iters = 4;
    p->coarse_iters = 16;
    p->coarse_tol = 0.1;
    p->restart = 8;
    p->maxiter = 500;
}

static laph_status mg_params_geo(const Ctx &c, const laph_mg_params *p, MgGeom &g) {
    if (!p) return set_error(LAPH_ERR_INVALID, "null multigrid parameters");
    if (p->null_passes < 0 || (p->null_passes > 0 && !(p->null_tol > 0 && p->null_tol < 1)) || p->smooth_iters < 1 ||
        p->coarse_iters < 1 || !(p->coarse_tol > 0 && p->coarse_tol < 1) || p->restart < 1 ||
        p->restart > kMgMaxRestart || p->maxiter < 1)
        return set_error(LAPH_ERR_INVALID, "bad multigrid parameters");
    return mg_geometry(c, p->nvec, p->block, g);
}

size_t laph_mg_state_bytes(laph_ctx h, const laph_mg_params *p) try {
    if (!h) return 0;
    MgGeom g;
    if (mg_params_geo(C(h), p, g) != LAPH_OK) return 0;
    return mg_state_bytes(C(h), g);
} LAPH_CATCH_SIZE

size_t laph_mg_setup_workspace_bytes(laph_ctx h, const laph_mg_params *p) try {
    if (!h) return 0;
    MgGeom g;
    if (mg_params_geo(C(h), p, g) != LAPH_OK) return 0;
    return mg_setup_workspace_bytes(C(h), g, p->null_passes);
} LAPH_CATCH_SIZE

laph_status laph_mg_setup(laph_ctx h, int mass_idx, const laph_mg_params *p, const double *V0, void *state,
                          size_t state_bytes, void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    c.mgs.ready = false;   // whatever was attached is gone, also when this call fails
    MgGeom g;
    LAPH_TRY(mg_params_geo(c, p, g));
    if (!V0 || !state) return set_error(LAPH_ERR_INVALID, "null start vectors or multigrid buffer");
    if (!work) return set_error(LAPH_ERR_WORKSPACE, "multigrid setup needs a workspace");
    LAPH_TRY(mg_setup(c, mass_idx, g, V0, p->null_passes, p->null_tol, reinterpret_cast<char *>(state), state_bytes,
                      reinterpret_cast<char *>(work), work ? work_bytes : 0));
    c.mgs.smooth_iters = p->smooth_iters;
    c.mgs.coarse_iters = p->coarse_iters;
    c.mgs.coarse_tol = p->coarse_tol;
    c.mgs.restart = p->restart;
    c.mgs.maxiter = p->maxiter;
    return LAPH_OK;
} LAPH_CATCH_STATUS

laph_status laph_mg_basis(laph_ctx h, double *out) try {
    LAPH_TRY(check_ctx(h));
    if (!out) return set_error(LAPH_ERR_INVALID, "null output");
    return mg_basis_canonical(C(h), out);
} LAPH_CATCH_STATUS

laph_status laph_mg_coarse_matrix(laph_ctx h, double *out) try {
    LAPH_TRY(check_ctx(h));
    Ctx &c = C(h);
    if (!out) return set_error(LAPH_ERR_INVALID, "null output");
    if (!c.mgs.ready) return set_error(LAPH_ERR_INVALID, "no multigrid set up (laph_mg_setup)");
    const MgGeom &g = c.mgs.geo;
    LAPH_HIP(hipMemcpyAsync(out, c.mgs.coarse, (size_t)g.nc * 9 * g.ncv * g.ncv * 16, hipMemcpyDeviceToDevice,
                            c.stream));
    return LAPH_OK;
} LAPH_CATCH_STATUS

size_t laph_mg_field_workspace_bytes(laph_ctx h, int n) try {
    if (!h || n <= 0) return 0;
    return (size_t)n * 2 * C(h).hv(LAPH_F64);
} LAPH_CATCH_SIZE

laph_status laph_mg_restrict(laph_ctx h, double *cvec, const double *f, int n, void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h));
    Ctx &c = C(h);
    if (!cvec || !f || n <= 0 || n > 65535) return set_error(LAPH_ERR_INVALID, "bad arguments");
    if (!work || work_bytes < (size_t)n * 2 * c.hv(LAPH_F64)) return set_error(LAPH_ERR_WORKSPACE, "workspace too small");
    return mg_restrict_canonical(c, cvec, f, n, reinterpret_cast<char *>(work));
} LAPH_CATCH_STATUS

laph_status laph_mg_prolong(laph_ctx h, double *f, const double *cvec, int n, void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h));
    Ctx &c = C(h);
    if (!cvec || !f || n <= 0 || n > 65535) return set_error(LAPH_ERR_INVALID, "bad arguments");
    if (!work || work_bytes < (size_t)n * 2 * c.hv(LAPH_F64)) return set_error(LAPH_ERR_WORKSPACE, "workspace too small");
    return mg_prolong_canonical(c, f, cvec, n, reinterpret_cast<char *>(work));
} LAPH_CATCH_STATUS

laph_status laph_mg_coarse_apply(laph_ctx h, double *out, const double *in, int n) try {
    LAPH_TRY(check_ctx(h));
    if (!out || !in || n <= 0 || n > 65535 || out == in) return set_error(LAPH_ERR_INVALID, "bad arguments");
    return mg_coarse_apply(C(h), out, in, n);
} LAPH_CATCH_STATUS

// the attached multigrid with the cycle parameters of p (NULL: those of the setup)
static laph_status mg_run_params(const Ctx &c, const laph_mg_params *p, MgState &run) {
    run = c.mgs;
    if (!p) return LAPH_OK;
    if (p->smooth_iters < 1 || p->coarse_iters < 1 || !(p->coarse_tol > 0 && p->coarse_tol < 1) || p->restart < 1 ||
        p->restart > kMgMaxRestart || p->maxiter < 1)
        return set_error(LAPH_ERR_INVALID, "bad multigrid cycle parameters");
    run.smooth_iters = p->smooth_iters;
    run.coarse_iters = p->coarse_iters;
    run.coarse_tol = p->coarse_tol;
    run.restart = p->restart;
    run.maxiter = p->maxiter;
    return LAPH_OK;
}

laph_status laph_mg_component(laph_ctx h, int what, double *out, const double *in, int n, const laph_mg_params *p,
                              void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h, true, true));
    if (!out || !in || n <= 0 || n > 65535 || out == in) return set_error(LAPH_ERR_INVALID, "bad arguments");
    if (!C(h).mgs.ready) return set_error(LAPH_ERR_INVALID, "no multigrid set up (laph_mg_setup)");
    if (!work) return set_error(LAPH_ERR_WORKSPACE, "null workspace");
    MgState run;
    LAPH_TRY(mg_run_params(C(h), p, run));
    return mg_component(C(h), run, what, out, in, n, reinterpret_cast<char *>(work), work_bytes);
} LAPH_CATCH_STATUS

size_t laph_mg_solve_workspace_bytes(laph_ctx h, int nrhs, const laph_mg_params *p) try {
    if (!h || nrhs <= 0 || !C(h).mgs.ready) return 0;
    MgState run;
    if (mg_run_params(C(h), p, run) != LAPH_OK) return 0;
    return mg_solve_workspace_bytes(C(h), nrhs, run.restart);
} LAPH_CATCH_SIZE

laph_status laph_mg_solve(laph_ctx h, double *X, const double *B, int nrhs, double tol, const laph_mg_params *p,
                          laph_rhs_stats *stats_host, void *work, size_t work_bytes) try {
    LAPH_TRY(check_ctx(h, true, true));
    Ctx &c = C(h);
    if (!X || !B || nrhs <= 0 || nrhs > 65535 || !(tol > 0 && tol < 1))
        return set_error(LAPH_ERR_INVALID, "bad arguments");
    if (!c.mgs.ready) return set_error(LAPH_ERR_INVALID, "no multigrid set up (laph_mg_setup)");
    if (!work) return set_error(LAPH_ERR_WORKSPACE, "null workspace");
    MgState run;
    LAPH_TRY(mg_run_params(c, p, run));
    return mg_solve(c, run, X, B, nrhs, tol, stats_host, reinterpret_cast<char *>(work), work_bytes);
} LAPH_CATCH_STATUS

}  // extern "C"
