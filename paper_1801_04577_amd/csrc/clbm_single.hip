// clbm_single.hip -- single-lattice entry points of the C ABI (include/clbm.h)
// and the kernels they launch besides the fused step: initialisation,
// macroscopic fields, population export and the diagnostics reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "clbm_host.h"
#include "clbm_aux_kernels.h"

namespace clbm {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

static thread_local char g_last_error[512] = "";

void set_last_hip_error(hipError_t e, const char* what, const char* file, int line)
{
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%s:%d)", hipGetErrorString(e), what,
                  file, line);
}

// ---------------------------------------------------------------------------
// Parameters
// ---------------------------------------------------------------------------

static bool in_open_02(double v) { return v > 0.0 && v < 2.0; }

clbm_status derive_rates(const clbm_params* p, Rates* r)
{
    if (!p || !r) return CLBM_ERR_INVALID_ARG;
    if (!(p->nu > 0.0) || !(p->alpha > 0.0) || !std::isfinite(p->nu) || !std::isfinite(p->alpha))
        return CLBM_ERR_INVALID_ARG;
    r->s_nu = 1.0 / (3.0 * p->nu + 0.5);
    r->s_b = std::isnan(p->s_b) ? 1.0 : p->s_b;
    r->s_4 = std::isnan(p->s_4) ? 1.0 : p->s_4;
    r->s_3 = std::isnan(p->s_3) ? (16.0 - 8.0 * r->s_nu) / (8.0 - r->s_nu) : p->s_3;
    r->l0 = std::isnan(p->lambda_0) ? 1.0 : p->lambda_0;
    r->l1 = 1.0 / (p->alpha / 0.4 + 0.5);
    r->l2 = std::isnan(p->lambda_2) ? 12.0 * (r->l1 - 2.0) / (r->l1 - 12.0) : p->lambda_2;
    const double all[7] = {r->s_nu, r->s_b, r->s_3, r->s_4, r->l0, r->l1, r->l2};
    for (double v : all)
        if (!in_open_02(v)) return CLBM_ERR_UNSTABLE_PARAMS;
    return CLBM_OK;
}

size_t row_elems(int nx) { return ((size_t)nx + kBlock - 1) / kBlock * kBlockElems; }

size_t buffer_elems(int nx, int ny) { return row_elems(nx) * (size_t)ny; }

dim3 node_grid(const LatticeConst& c, dim3 blk)
{
    const size_t nb = (size_t)((c.nx + blk.x - 1) / blk.x) * ((c.ny + blk.y - 1) / blk.y);
    return dim3((unsigned)nb, 1, 1);
}

clbm_status validate(const clbm_params* p, Rates* r)
{
    if (!p) return CLBM_ERR_INVALID_ARG;
    if (p->nx < 1 || p->ny < 1) return CLBM_ERR_INVALID_ARG;
    if (p->precision != CLBM_FP32 && p->precision != CLBM_FP16_SHIFTED) return CLBM_ERR_INVALID_ARG;
    const double scal[] = {p->g_beta, p->T0, p->Fx, p->Fy, p->Q};
    for (double v : scal)
        if (!std::isfinite(v)) return CLBM_ERR_INVALID_ARG;
    for (int s = 0; s < 4; ++s) {
        const clbm_side& sd = p->side[s];
        if (sd.kind != CLBM_PERIODIC && sd.kind != CLBM_WALL) return CLBM_ERR_INVALID_ARG;
        if (sd.kind == CLBM_WALL) {
            if (!std::isfinite(sd.u_wall) || !std::isfinite(sd.b1) || !std::isfinite(sd.b2) ||
                !std::isfinite(sd.b3))
                return CLBM_ERR_INVALID_ARG;
            if (8.0 * sd.b1 + 3.0 * sd.b2 == 0.0) return CLBM_ERR_INVALID_ARG;  // Eq. (28) singular
        }
    }
    if (p->side[0].kind != p->side[1].kind || p->side[2].kind != p->side[3].kind)
        return CLBM_ERR_INVALID_ARG;
    if (p->viscous_heating != 0 && p->viscous_heating != 1) return CLBM_ERR_INVALID_ARG;
    // Eq. (27) needs a second layer of nodes next to each wall.
    if (p->side[0].kind == CLBM_WALL && p->nx < 2) return CLBM_ERR_INVALID_ARG;
    if (p->side[2].kind == CLBM_WALL && p->ny < 2) return CLBM_ERR_INVALID_ARG;
    // Offsets within one row of a population buffer are 32-bit byte offsets (rows are
    // addressed with 64-bit offsets, so the lattice size is bounded by memory only).
    if ((double)row_elems(p->nx) * sizeof(float) >= 4294967295.0) return CLBM_ERR_UNSUPPORTED;
    // The per-node kernels (initialisation, exports) launch one work-item per node, in
    // blocks of 64 x 4 nodes, and a launch holds fewer than 2^32 work-items.
    if ((double)((p->nx + 63) / 64) * 64.0 * (double)((p->ny + 3) / 4) * 4.0 >= 4294967295.0)
        return CLBM_ERR_UNSUPPORTED;
    Rates tmp;
    Rates* rr = r ? r : &tmp;
    clbm_status st = derive_rates(p, rr);
    if (st != CLBM_OK) return st;
    // The dissipation source needs a temperature-independent flow, and its recovery
    // from stored post-collision moments divides by 1 - s_nu.
    if (p->viscous_heating && (p->g_beta != 0.0 || std::fabs(1.0 - rr->s_nu) < 1e-3))
        return CLBM_ERR_INVALID_ARG;
    return CLBM_OK;
}

LatticeConst make_const(const clbm_params* p, const Rates& r)
{
    LatticeConst c;
    std::memset(&c, 0, sizeof c);
    c.nx = p->nx;
    c.ny = p->ny;
    c.rowlen = (unsigned)row_elems(p->nx);
    c.periodic_x = p->side[0].kind == CLBM_PERIODIC;
    c.periodic_y = p->side[2].kind == CLBM_PERIODIC;
    const double sp = 0.5 * (r.s_b + r.s_nu), sm = 0.5 * (r.s_b - r.s_nu);
    c.sp = (float)sp;
    c.sm = (float)sm;
    c.snu = (float)r.s_nu;
    c.s3 = (float)r.s_3;
    c.half_s3c = (float)((1.0 - 0.5 * r.s_3) / 3.0);
    c.s4 = (float)r.s_4;
    c.l1 = (float)r.l1;
    c.l2 = (float)r.l2;
    c.d_sp = sp;
    c.d_sm = sm;
    c.d_snu = r.s_nu;
    c.d_s3 = r.s_3;
    c.d_h3 = (1.0 - 0.5 * r.s_3) / 3.0;
    c.d_s4 = r.s_4;
    c.d_l1 = r.l1;
    c.d_l2 = r.l2;
    c.d_src2 = (1.0 - 0.5 * r.l2) * 0.4 * p->Q;
    c.d_src2_q = (1.0 - 0.5 * r.l2) * 0.4;
    c.d_Q = p->Q;
    c.d_Fx = p->Fx;
    c.d_Fy = p->Fy;
    c.d_gb = p->g_beta;
    c.d_T0 = p->T0;
    c.src2 = (float)((1.0 - 0.5 * r.l2) * 0.4 * p->Q);
    c.src2_q = (float)((1.0 - 0.5 * r.l2) * 0.4);
    c.viscous = p->viscous_heating ? 1 : 0;
    if (c.viscous) {
        const double coef = 9.0 * p->nu * r.s_nu * r.s_nu;
        c.vh_pre = (float)coef;
        c.d_vh_pre = coef;
        c.vh_post = (float)(coef / ((1.0 - r.s_nu) * (1.0 - r.s_nu)));
    }
    c.g_beta = (float)p->g_beta;
    c.Fx = (float)p->Fx;
    c.Fy = (float)p->Fy;
    c.Q = (float)p->Q;
    c.T0 = (float)p->T0;
    c.moving = 0;
    for (int s = 0; s < 4; ++s) {
        const clbm_side& sd = p->side[s];
        if (sd.kind != CLBM_WALL) continue;
        c.uw[s] = (float)sd.u_wall;
        if (sd.u_wall != 0.0) c.moving = 1;
        // Eq. (28) with n . e_i = 1, dx = 1, in theta = T - T0.
        const double D = 8.0 * sd.b1 + 3.0 * sd.b2;
        c.a1[s] = (float)(9.0 * sd.b1 / D);
        c.a2[s] = (float)(-sd.b1 / D);
        c.a3[s] = (float)(3.0 * (sd.b3 - sd.b2 * p->T0) / D);
    }
    return c;
}

// ---------------------------------------------------------------------------
// Kernels besides the step
// ---------------------------------------------------------------------------

// Streaming copy used as the bandwidth reference (see clbm_stream_copy): one 16-byte
// element per thread.
__global__ void __launch_bounds__(256) k_stream_copy(float4* __restrict__ dst,
                                                     const float4* __restrict__ src, size_t n)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// Step launcher (shared with the graph builder)
// ---------------------------------------------------------------------------

struct StepLaunch {
    const void* fn;
    dim3 grid, block;
    int tiles_x, tiles_total, remap;
};

template <typename S, int SRC, typename O>
static const void* step_fn(int rows)
{
    switch (rows) {
        case 2: return reinterpret_cast<const void*>(&k_step<S, 2, SRC, O>);
        case 4: return reinterpret_cast<const void*>(&k_step<S, 4, SRC, O>);
        default: return reinterpret_cast<const void*>(&k_step<S, 1, SRC, O>);
    }
}

// Source terms of a lattice: viscous heating and/or a source field (kSrc* bits).
static int lattice_src(const LatticeConst& c)
{
    return (c.viscous ? kSrcVisc : 0) | (c.qfield ? kSrcField : 0);
}

// Element offsets in the step kernels: 32-bit unless a population buffer holds 2^32
// elements or more.
static bool wide_offsets(const LatticeConst& c) { return (size_t)c.rowlen * c.ny >= 0xFFFFFFFFull; }

template <typename S, typename O>
static const void* step_fn_src(int rows, int src)
{
    switch (src) {
        case kSrcVisc: return step_fn<S, kSrcVisc, O>(rows);
        case kSrcField: return step_fn<S, kSrcField, O>(rows);
        case kSrcVisc | kSrcField: return step_fn<S, kSrcVisc | kSrcField, O>(rows);
        default: return step_fn<S, 0, O>(rows);
    }
}

template <typename S>
static const void* step_fn(int rows, int src, bool wide)
{
    return wide ? step_fn_src<S, size_t>(rows, src) : step_fn_src<S, unsigned>(rows, src);
}

static StepLaunch plan_step(const LatticeConst& c, int precision, const clbm_launch& L)
{
    StepLaunch s;
    const bool wide = wide_offsets(c);
    s.fn = precision == CLBM_FP16_SHIFTED ? step_fn<__half>(L.rows_per_thread, lattice_src(c), wide)
                                          : step_fn<float>(L.rows_per_thread, lattice_src(c), wide);
    s.block = dim3(L.block_x, L.block_y, 1);
    s.tiles_x = (c.nx + L.block_x - 1) / L.block_x;
    const int rows_per_tile = L.block_y * L.rows_per_thread;
    const int tiles_y = (c.ny + rows_per_tile - 1) / rows_per_tile;
    s.tiles_total = s.tiles_x * tiles_y;
    s.remap = L.xcd_remap ? 1 : 0;
    const int g = s.remap ? (int)align_up((size_t)s.tiles_total, 8) : s.tiles_total;
    s.grid = dim3(g, 1, 1);
    return s;
}

// Tile heights of the two-step kernel and their thread counts (rows + 2 halo rows dealt to
// the waves: 64 (rows + 2) / 2 threads).

static bool launch_ok(const clbm_launch& L, int precision)
{
    if (L.steps_per_launch == 2)
        return (precision == CLBM_FP32 || precision == CLBM_FP16_SHIFTED) &&
               (L.two_step_rows == 0 || two_step_rows_ok(L.two_step_rows));
    if (L.steps_per_launch != 1) return false;
    const int threads = L.block_x * L.block_y;
    if (L.block_x < 1 || L.block_y < 1 || threads % 64 != 0 || threads > 1024) return false;
    return L.rows_per_thread == 1 || L.rows_per_thread == 2 || L.rows_per_thread == 4;
}

// The single-step shape used where none is given: 256 x 1 threads, one row each.
static clbm_launch default_single_launch()
{
    clbm_launch L;
    L.block_x = 256;
    L.block_y = 1;
    L.rows_per_thread = 1;
    L.xcd_remap = 0;
    L.steps_per_launch = 1;
    L.two_step_rows = 0;
    return L;
}

static clbm_launch default_launch(int precision)
{
    clbm_launch L = default_single_launch();
    // two steps per launch over XCD-ordered tiles (the single step that ends an odd
    // count then also takes the remap, at no measurable cost)
    L.xcd_remap = 1;
    L.steps_per_launch = 2;
    (void)precision;
    return L;
}

struct Step2Launch {
    const void* fn;
    dim3 grid, block;
    int tiles_x, tiles_total, remap;
};

template <typename S, int TY, int NT, typename O>
static const void* step2_fn_o(int src)
{
    switch (src) {
        case kSrcVisc: return reinterpret_cast<const void*>(&k_step2<S, kSrcVisc, TY, NT, O>);
        case kSrcField: return reinterpret_cast<const void*>(&k_step2<S, kSrcField, TY, NT, O>);
        case kSrcVisc | kSrcField:
            return reinterpret_cast<const void*>(&k_step2<S, kSrcVisc | kSrcField, TY, NT, O>);
        default: return reinterpret_cast<const void*>(&k_step2<S, 0, TY, NT, O>);
    }
}

template <typename S, int TY, int NT>
static const void* step2_fn(int src, bool wide)
{
    return wide ? step2_fn_o<S, TY, NT, size_t>(src) : step2_fn_o<S, TY, NT, unsigned>(src);
}

template <typename S>
static const void* step2_for_rows(int rows, int src, bool wide)
{
    if (rows == 6) return step2_fn<S, 6, 256>(src, wide);
    if (rows == 22) return step2_fn<S, 22, 512>(src, wide);
    if (rows == 30) return step2_fn<S, 30, 1024>(src, wide);
    return step2_fn<S, 14, 512>(src, wide);
}

static Step2Launch plan_step2(const LatticeConst& c, int precision, const clbm_launch& L)
{
    Step2Launch s;
    const bool f16 = precision == CLBM_FP16_SHIFTED;
    const int rows = L.two_step_rows ? L.two_step_rows : (f16 ? kTwoStepRowsF16 : kTwoStepRows);
    s.fn = f16 ? step2_for_rows<__half>(rows, lattice_src(c), wide_offsets(c))
               : step2_for_rows<float>(rows, lattice_src(c), wide_offsets(c));
    s.tiles_x = (c.nx + (int)kBlock - 1) / (int)kBlock;
    const int tiles_y = (c.ny + rows - 1) / rows;
    s.tiles_total = s.tiles_x * tiles_y;
    s.remap = L.xcd_remap ? 1 : 0;
    const int g = s.remap ? (int)align_up((size_t)s.tiles_total, 8) : s.tiles_total;
    s.grid = dim3((unsigned)g, 1, 1);
    s.block = dim3(two_step_threads(rows), 1, 1);
    return s;
}

}  // namespace clbm

using namespace clbm;

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------

struct clbm_handle {
    clbm_params p;
    Rates rates;
    LatticeConst c;
    hipStream_t stream;
    int elem;            // bytes per stored population
    size_t buf_bytes;    // bytes of one population buffer (14 populations per node)
    void* buf[2];
    float* snap;         // (u_x, u_y, T), 3 dense planes
    double* partial;     // kDiagMaxBlocks x kDiagSums
    double* result;      // kDiagSums
    int cur;             // buffer holding the current post-collision state
    long step;
    long snap_step;      // -1: no snapshot
    clbm_launch launch;
    int graph_steps;
    hipGraphExec_t gexec[2];  // graph_steps steps starting from buffer 0 / 1
    hipGraph_t graph[2];
    double* scratch;     // this GPU's copy of the library's diagnostics scratch
};

// ---------------------------------------------------------------------------
// Library-owned scratch of clbm_diagnostics_noalloc
// ---------------------------------------------------------------------------

// The diagnostics reduction's per-workgroup partial sums (kDiagMaxBlocks x kDiagSums) and
// its final sums (kDiagSums), in a fixed device array instead of the caller's workspace:
// 155 KB. Each GPU the library runs on holds its own copy until the process ends. Every
// call on one GPU shares that copy, so calls that overlap on one GPU race (order them on
// one stream). Nothing in it has to start at zero: a call writes every partial it reads.
constexpr size_t kScratchDoubles = (size_t)kDiagMaxBlocks * kDiagSums + kDiagSums;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices];

// Device address of the scratch on `device`, which must be the current device: resolved
// once per device, then reused. In host code the array's own name is not a device
// address; only this pointer may be handed to kernels.
static clbm_status scratch_address(int device, double** out)
{
    if (device < 0 || device >= kMaxDevices) return CLBM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_last_hip_error(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
            return CLBM_ERR_HIP;
        }
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return CLBM_OK;
}

namespace {

size_t layout(const clbm_params* p, size_t* buf_bytes, size_t* off_snap, size_t* off_part,
              size_t* off_res)
{
    const size_t elem = p->precision == CLBM_FP16_SHIFTED ? 2 : 4;
    const size_t bb = align_up(buffer_elems(p->nx, p->ny) * elem, kAlign);
    const size_t n = (size_t)p->nx * p->ny;
    size_t off = 2 * bb;
    const size_t snap = off;
    off = align_up(off + 3 * n * sizeof(float), kAlign);
    const size_t part = off;
    off = align_up(off + (size_t)kDiagMaxBlocks * kDiagSums * sizeof(double), kAlign);
    const size_t res = off;
    off = align_up(off + kDiagSums * sizeof(double), kAlign);
    if (buf_bytes) *buf_bytes = bb;
    if (off_snap) *off_snap = snap;
    if (off_part) *off_part = part;
    if (off_res) *off_res = res;
    return off;
}

void drop_graphs(clbm_handle* h)
{
    for (int k = 0; k < 2; ++k) {
        if (h->gexec[k]) (void)hipGraphExecDestroy(h->gexec[k]);
        if (h->graph[k]) (void)hipGraphDestroy(h->graph[k]);
        h->gexec[k] = nullptr;
        h->graph[k] = nullptr;
    }
}

// One kernel launch advancing the state by one or two steps from buffer `from`.
struct LaunchArgs {
    void* src;
    void* dst;
    LatticeConst c;
    int a0, a1, a2;
};

// The launches of n steps: two-step launches while two or more steps remain (when
// enabled), then single steps. Calls emit(fn, grid, block, args) for each.
template <typename Emit>
clbm_status plan_steps(clbm_handle* h, int n, int from, Emit emit)
{
    const bool two = h->launch.steps_per_launch == 2;
    const StepLaunch s1 = plan_step(h->c, h->p.precision, h->launch);
    const Step2Launch s2 = plan_step2(h->c, h->p.precision, h->launch);
    int cur = from;
    while (n > 0) {
        LaunchArgs a;
        a.src = h->buf[cur];
        a.dst = h->buf[cur ^ 1];
        a.c = h->c;
        if (two && n >= 2) {
            a.a0 = s2.tiles_x;
            a.a1 = s2.tiles_total;
            a.a2 = s2.remap;
            void* args[] = {&a.src, &a.dst, &a.c, &a.a0, &a.a1, &a.a2};
            clbm_status st = emit(s2.fn, s2.grid, s2.block, args);
            if (st != CLBM_OK) return st;
            n -= 2;
        } else {
            a.a0 = s1.tiles_x;
            a.a1 = s1.tiles_total;
            a.a2 = s1.remap;
            void* args[] = {&a.src, &a.dst, &a.c, &a.a0, &a.a1, &a.a2};
            clbm_status st = emit(s1.fn, s1.grid, s1.block, args);
            if (st != CLBM_OK) return st;
            n -= 1;
        }
        cur ^= 1;
    }
    return CLBM_OK;
}

// Number of launches (buffer flips) of n steps.
int launches_of(const clbm_handle* h, int n)
{
    return h->launch.steps_per_launch == 2 ? n / 2 + n % 2 : n;
}

clbm_status launch_steps_direct(clbm_handle* h, int n)
{
    clbm_status st = plan_steps(h, n, h->cur, [&](const void* fn, dim3 g, dim3 b, void** args) {
        CLBM_HIP(hipLaunchKernel(fn, g, b, args, 0, h->stream));
        return CLBM_OK;
    });
    if (st != CLBM_OK) return st;
    h->cur ^= launches_of(h, n) & 1;
    h->step += n;
    return CLBM_OK;
}

clbm_status build_graph(clbm_handle* h, int start)
{
    hipGraph_t g = nullptr;
    CLBM_HIP(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    // hipGraphAddKernelNode copies the argument values.
    clbm_status st = plan_steps(h, h->graph_steps, start, [&](const void* fn, dim3 gd, dim3 bd, void** args) {
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof kp);
        kp.func = const_cast<void*>(fn);
        kp.gridDim = gd;
        kp.blockDim = bd;
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) {
            set_last_hip_error(e, "hipGraphAddKernelNode", __FILE__, __LINE__);
            return CLBM_ERR_HIP;
        }
        prev = node;
        return CLBM_OK;
    });
    if (st != CLBM_OK) {
        (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_last_hip_error(e, "hipGraphInstantiate", __FILE__, __LINE__);
        return CLBM_ERR_HIP;
    }
    h->graph[start] = g;
    h->gexec[start] = ex;
    return CLBM_OK;
}

}  // namespace

extern "C" {

int clbm_abi_version(void) { return CLBM_ABI_VERSION; }

const char* clbm_status_string(int status)
{
    switch (status) {
        case CLBM_OK: return "ok";
        case CLBM_ERR_INVALID_ARG: return "invalid argument";
        case CLBM_ERR_UNSTABLE_PARAMS: return "relaxation rate outside (0, 2)";
        case CLBM_ERR_BUFFER_TOO_SMALL: return "workspace too small";
        case CLBM_ERR_HIP: return g_last_error[0] ? g_last_error : "HIP runtime error";
        case CLBM_ERR_NAN: return "non-finite values in the state";
        case CLBM_ERR_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

clbm_status clbm_derive_rates(const clbm_params* p, double out[7])
{
    if (!p || !out) return CLBM_ERR_INVALID_ARG;
    Rates r;
    clbm_status st = derive_rates(p, &r);
    out[0] = r.s_nu; out[1] = r.s_b; out[2] = r.s_3; out[3] = r.s_4;
    out[4] = r.l0;   out[5] = r.l1;  out[6] = r.l2;
    return st;
}

clbm_status clbm_workspace_bytes(const clbm_params* p, size_t* bytes)
{
    if (!p || !bytes) return CLBM_ERR_INVALID_ARG;
    clbm_status st = validate(p, nullptr);
    if (st != CLBM_OK) return st;
    *bytes = layout(p, nullptr, nullptr, nullptr, nullptr);
    return CLBM_OK;
}

clbm_status clbm_create(const clbm_params* p, void* d_workspace, size_t bytes, void* hip_stream,
                        clbm_handle** out)
{
    if (!p || !out) return CLBM_ERR_INVALID_ARG;
    *out = nullptr;
    Rates r;
    clbm_status st = validate(p, &r);
    if (st != CLBM_OK) return st;
    size_t bb, o_snap, o_part, o_res;
    const size_t need = layout(p, &bb, &o_snap, &o_part, &o_res);
    if (!d_workspace) return CLBM_ERR_INVALID_ARG;
    if (((uintptr_t)d_workspace) % kAlign != 0) return CLBM_ERR_INVALID_ARG;
    if (bytes < need) return CLBM_ERR_BUFFER_TOO_SMALL;
    clbm_handle* h = new (std::nothrow) clbm_handle;
    if (!h) return CLBM_ERR_INVALID_ARG;
    std::memset(h, 0, sizeof *h);
    h->p = *p;
    h->rates = r;
    h->c = make_const(p, r);
    h->stream = (hipStream_t)hip_stream;
    h->elem = p->precision == CLBM_FP16_SHIFTED ? 2 : 4;
    h->buf_bytes = bb;
    char* ws = (char*)d_workspace;
    h->buf[0] = ws;
    h->buf[1] = ws + bb;
    h->snap = (float*)(ws + o_snap);
    h->partial = (double*)(ws + o_part);
    h->result = (double*)(ws + o_res);
    h->launch = default_launch(p->precision);
    h->graph_steps = 0;
    h->snap_step = -1;
    int device = -1;
    const hipError_t de = hipGetDevice(&device);
    if (de != hipSuccess) {
        set_last_hip_error(de, "hipGetDevice", __FILE__, __LINE__);
        delete h;
        return CLBM_ERR_HIP;
    }
    st = scratch_address(device, &h->scratch);
    if (st != CLBM_OK) {
        delete h;
        return st;
    }
    st = clbm_init_from_fields(h, nullptr, nullptr, nullptr, nullptr);
    if (st != CLBM_OK) {
        delete h;
        return st;
    }
    *out = h;
    return CLBM_OK;
}

void clbm_destroy(clbm_handle* h)
{
    if (!h) return;
    drop_graphs(h);
    delete h;
}

clbm_status clbm_init_from_fields(clbm_handle* h, const float* d_rho, const float* d_ux,
                                  const float* d_uy, const float* d_T)
{
    if (!h) return CLBM_ERR_INVALID_ARG;
    const dim3 blk(64, 4, 1);
    const dim3 grd = node_grid(h->c, blk);
    if (h->p.precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_init<__half>, grd, blk, 0, h->stream, (__half*)h->buf[0], h->c, d_rho,
                           d_ux, d_uy, d_T);
    else
        hipLaunchKernelGGL(k_init<float>, grd, blk, 0, h->stream, (float*)h->buf[0], h->c, d_rho,
                           d_ux, d_uy, d_T);
    CLBM_HIP(hipGetLastError());
    h->cur = 0;
    h->step = 0;
    h->snap_step = -1;
    return CLBM_OK;
}

clbm_status clbm_step(clbm_handle* h, int nsteps)
{
    if (!h || nsteps < 0) return CLBM_ERR_INVALID_ARG;
    int left = nsteps;
    if (h->graph_steps > 0) {
        while (left >= h->graph_steps) {
            if (!h->gexec[h->cur]) {
                clbm_status st = build_graph(h, h->cur);
                if (st != CLBM_OK) return st;
            }
            CLBM_HIP(hipGraphLaunch(h->gexec[h->cur], h->stream));
            h->cur ^= launches_of(h, h->graph_steps) & 1;
            h->step += h->graph_steps;
            left -= h->graph_steps;
        }
    }
    return launch_steps_direct(h, left);
}

clbm_status clbm_macros(clbm_handle* h, float* d_rho, float* d_ux, float* d_uy, float* d_T)
{
    if (!h) return CLBM_ERR_INVALID_ARG;
    const dim3 blk(64, 4, 1);
    const dim3 grd = node_grid(h->c, blk);
    if (h->p.precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_macros<__half>, grd, blk, 0, h->stream, (const __half*)h->buf[h->cur],
                           h->c, d_rho, d_ux, d_uy, d_T);
    else
        hipLaunchKernelGGL(k_macros<float>, grd, blk, 0, h->stream, (const float*)h->buf[h->cur],
                           h->c, d_rho, d_ux, d_uy, d_T);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_populations(clbm_handle* h, float* d_f, float* d_g)
{
    if (!h) return CLBM_ERR_INVALID_ARG;
    const dim3 blk(64, 4, 1);
    const dim3 grd = node_grid(h->c, blk);
    if (h->p.precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_populations<__half>, grd, blk, 0, h->stream,
                           (const __half*)h->buf[h->cur], h->c, d_f, d_g);
    else
        hipLaunchKernelGGL(k_populations<float>, grd, blk, 0, h->stream,
                           (const float*)h->buf[h->cur], h->c, d_f, d_g);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

}  // extern "C"

namespace {

// The diagnostics reduction with its partial sums in `partial` (kDiagMaxBlocks x
// kDiagSums doubles) and its final sums in `result` (kDiagSums doubles).
clbm_status diagnostics_into(clbm_handle* h, double* partial, double* result, clbm_diag* out)
{
    const size_t n = (size_t)h->p.nx * h->p.ny;
    const int blocks = (int)std::min<size_t>((n + kDiagBlock - 1) / kDiagBlock, kDiagMaxBlocks);
    const int have = h->snap_step >= 0 ? 1 : 0;
    if (h->p.precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_diag<__half>, dim3(blocks), dim3(kDiagBlock), 0, h->stream,
                           (const __half*)h->buf[h->cur], h->c, h->snap, have, partial);
    else
        hipLaunchKernelGGL(k_diag<float>, dim3(blocks), dim3(kDiagBlock), 0, h->stream,
                           (const float*)h->buf[h->cur], h->c, h->snap, have, partial);
    CLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, h->stream, partial, blocks, result);
    CLBM_HIP(hipGetLastError());
    double r[kDiagSums];
    CLBM_HIP(hipMemcpyAsync(r, result, sizeof r, hipMemcpyDeviceToHost, h->stream));
    CLBM_HIP(hipStreamSynchronize(h->stream));
    std::memset(out, 0, sizeof *out);
    out->step = h->step;
    out->K = have ? (int)(h->step - h->snap_step) : 0;
    out->mass = (double)n + r[0];
    out->sum_u2 = r[1];
    out->sum_du2 = r[2];
    out->sum_T2 = r[3];
    out->sum_dT2 = r[4];
    if (out->K > 0) {
        out->res_u = r[1] > 0.0 ? std::sqrt(r[2] / r[1]) / out->K : 0.0;
        out->res_T = r[3] > 0.0 ? std::sqrt(r[4] / r[3]) / out->K : 0.0;
    }
    const int len[4] = {h->p.ny, h->p.ny, h->p.nx, h->p.nx};
    for (int s = 0; s < 4; ++s) {
        if (h->p.side[s].kind != CLBM_WALL) continue;
        out->dTdn[s] = r[5 + s] / len[s];
        out->T_wall[s] = r[9 + s] / len[s];
        out->wall_flux[s] = r[15 + s] / len[s];
    }
    out->nan_count = (long)r[13];
    h->snap_step = h->step;
    return out->nan_count > 0 ? CLBM_ERR_NAN : CLBM_OK;
}

}  // namespace

extern "C" {

clbm_status clbm_diagnostics(clbm_handle* h, clbm_diag* out)
{
    if (!h || !out) return CLBM_ERR_INVALID_ARG;
    return diagnostics_into(h, h->partial, h->result, out);
}

clbm_status clbm_diagnostics_noalloc(clbm_handle* h, clbm_diag* out)
{
    if (!h || !out) return CLBM_ERR_INVALID_ARG;
    if (!h->scratch) return CLBM_ERR_HIP;
    const size_t n = (size_t)h->p.nx * h->p.ny;
    const size_t parts = std::min<size_t>((n + kDiagBlock - 1) / kDiagBlock, kDiagMaxBlocks);
    // the reduction grid is capped at kDiagMaxBlocks workgroups, so every lattice fits
    if ((parts + 1) * kDiagSums > kScratchDoubles) return CLBM_ERR_BUFFER_TOO_SMALL;
    return diagnostics_into(h, h->scratch, h->scratch + (size_t)kDiagMaxBlocks * kDiagSums, out);
}

clbm_status clbm_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* hip_stream)
{
    if (!d_dst || !d_src || bytes % 16 != 0 || ((uintptr_t)d_dst | (uintptr_t)d_src) % 16 != 0)
        return CLBM_ERR_INVALID_ARG;
    const size_t n = bytes / 16;
    if (n == 0) return CLBM_OK;
    if ((n + 255) / 256 > 0x7fffffffu) return CLBM_ERR_UNSUPPORTED;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream,
                       (float4*)d_dst, (const float4*)d_src, n);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_state_bytes(const clbm_handle* h, size_t* bytes)
{
    if (!h || !bytes) return CLBM_ERR_INVALID_ARG;
    *bytes = h->buf_bytes;
    return CLBM_OK;
}

clbm_status clbm_save(clbm_handle* h, void* d_dst)
{
    if (!h || !d_dst) return CLBM_ERR_INVALID_ARG;
    CLBM_HIP(hipMemcpyAsync(d_dst, h->buf[h->cur], h->buf_bytes, hipMemcpyDeviceToDevice, h->stream));
    return CLBM_OK;
}

clbm_status clbm_load(clbm_handle* h, const void* d_src, long step)
{
    if (!h || !d_src || step < 0) return CLBM_ERR_INVALID_ARG;
    CLBM_HIP(hipMemcpyAsync(h->buf[h->cur], d_src, h->buf_bytes, hipMemcpyDeviceToDevice, h->stream));
    h->step = step;
    h->snap_step = -1;
    return CLBM_OK;
}

clbm_status clbm_get_step(const clbm_handle* h, long* step)
{
    if (!h || !step) return CLBM_ERR_INVALID_ARG;
    *step = h->step;
    return CLBM_OK;
}

clbm_status clbm_set_launch(clbm_handle* h, const clbm_launch* launch)
{
    if (!h || !launch) return CLBM_ERR_INVALID_ARG;
    clbm_launch L = *launch;
    if (L.block_x == 0 && L.block_y == 0 && L.rows_per_thread == 0 && L.xcd_remap == 0 &&
        L.steps_per_launch == 0)
        L = default_launch(h->p.precision);
    if (L.steps_per_launch == 2) {
        // the single step that ends an odd step count uses the default shape unless a
        // valid one is given
        clbm_launch one = L;
        one.steps_per_launch = 1;
        if (!launch_ok(one, h->p.precision)) {
            const clbm_launch d = default_single_launch();
            L.block_x = d.block_x;
            L.block_y = d.block_y;
            L.rows_per_thread = d.rows_per_thread;
            L.xcd_remap = d.xcd_remap;
        }
    }
    if (!launch_ok(L, h->p.precision)) return CLBM_ERR_INVALID_ARG;
    h->launch = L;
    drop_graphs(h);
    return CLBM_OK;
}

clbm_status clbm_get_launch(const clbm_handle* h, clbm_launch* launch)
{
    if (!h || !launch) return CLBM_ERR_INVALID_ARG;
    *launch = h->launch;
    return CLBM_OK;
}

clbm_status clbm_set_source_field(clbm_handle* h, const float* d_q)
{
    if (!h) return CLBM_ERR_INVALID_ARG;
    h->c.qfield = d_q;
    // graphs hold the lattice constants by value: rebuild them with the field
    const int g = h->graph_steps;
    drop_graphs(h);
    for (int start = 0; start < 2 && g > 0; ++start) {
        const clbm_status st = build_graph(h, start);
        if (st != CLBM_OK) {
            drop_graphs(h);
            h->graph_steps = 0;
            return st;
        }
    }
    return CLBM_OK;
}

clbm_status clbm_set_graph(clbm_handle* h, int steps_per_graph)
{
    if (!h || steps_per_graph < 0 || (steps_per_graph % 2) != 0) return CLBM_ERR_INVALID_ARG;
    drop_graphs(h);
    h->graph_steps = steps_per_graph;
    // both graphs (starting from either buffer) are instantiated here, so that a later
    // clbm_step replays them without building anything
    for (int start = 0; start < 2 && steps_per_graph > 0; ++start) {
        const clbm_status st = build_graph(h, start);
        if (st != CLBM_OK) {
            drop_graphs(h);
            h->graph_steps = 0;
            return st;
        }
    }
    return CLBM_OK;
}

}  // extern "C"
