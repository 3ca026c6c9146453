// lbm_api.hip -- host side of the C ABI declared in include/lbm.h.
//
// A context holds any number of independent channels.  All of them live in
// two population buffers (A, B; post-collision values, pull scheme), one
// node-sized snapshot for the residual, a tile table mapping workgroups to
// (channel, tile) and one descriptor per channel.  A step is one launch of
// the fused kernel over every tile of every active channel; every 100th step
// also takes the float64 residual snapshot and is followed by a per-channel
// check kernel.  lbm_solve replays a captured HIP graph of 100 steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>
#include <cstddef>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

struct lbm_ctx {
    int n_inst = 0;
    int prec = 0;
    size_t elem = 8;                   // bytes per stored population
    hipStream_t stream = nullptr;
    bool own_stream = false;
    lbm_alloc_fn alloc = nullptr;
    lbm_free_fn free_fn = nullptr;
    void* user = nullptr;
    std::vector<lbm_params> params;
    std::vector<Inst> h_inst;
    std::vector<int> h_tile_inst;
    long long total_nodes = 0, total_pop = 0, total_rows = 0, total_cols = 0;
    int max_nodes = 0;
    int n_tiles = 0;
    int tx = TILE_SHAPES[0][0], ty = TILE_SHAPES[0][1];
    // device memory
    void* popA = nullptr;
    void* popB = nullptr;
    void* phi0 = nullptr;              // storage reference phi0 by row (float32 mode)
    void* phir = nullptr;              // zeroth moment of the streamed reference populations minus phi0, by row
    void* fq = nullptr;                // flux reference of f (half its y-moment) by row
    void* fr = nullptr;                // constant part of the stored post-collision y-moment of f by row
    // float32 mode: the flux reference follows the actual flux (moved after
    // every check); the set-up tables are kept to start from again
    float* fq_next = nullptr;
    float* fr_next = nullptr;
    float* fr_sw = nullptr;
    float* fq_cold = nullptr;
    float* fr_cold = nullptr;
    double* frc = nullptr;             // (1 - w_phi) r01 + w_phi M theta0 n0y by row
    double* rowpart = nullptr;         // check-step row sums of the flux deviation [rows][ceil(nx/16)]
    int max_rows = 0;
    double* twall = nullptr;           // bottom-wall temperature by column (float64 in both precisions)
    float* tref = nullptr;             // per-node temperature reference (float32 mode)
    float* tref_new = nullptr;         // references written by a check step
    int32_t* dl = nullptr;             // per-node phi-reference offsets, units of DL_Q (float32 mode)
    int32_t* dl_new = nullptr;         // offsets written by a check step
    int32_t* dlz = nullptr;            // chunk flags of dl (nonzero offsets)
    int max_chunks = 0;                // largest chunk count of one channel
    double* snap = nullptr;            // 4 * total_nodes
    double* partials = nullptr;        // n_tiles * 8 (capacity for the smallest tile)
    int partial_cap = 0;
    double* chk = nullptr;             // per-block check sums, [n_inst][chk_nb][9]
    int chk_nb = 1;
    Inst* d_inst = nullptr;
    int* d_tile_inst = nullptr;
    int tile_cap = 0;
    Result* d_res = nullptr;
    long long* d_counter = nullptr;
    double* d_tol = nullptr;
    int* d_active = nullptr;
    int* h_active = nullptr;           // pinned
    std::vector<std::pair<void*, size_t>> allocations;   // live device allocations and their sizes
    size_t device_bytes = 0;                             // sum of their sizes
    // state
    bool initialised = false;
    long long steps = 0;               // steps of the channels still active
    std::vector<char> retired;         // host copy (refreshed by sync points)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_tx = 0, graph_ty = 0, graph_ntiles = -1;
    std::string last_error;
};

namespace {

thread_local std::string g_err;

int fail_hip(lbm_ctx* c, hipError_t e, const char* what) {
    std::string s = std::string(what) + ": " + hipGetErrorString(e);
    if (c) c->last_error = s;
    g_err = s;
    (void)hipGetLastError();  // clear the sticky launch error
    return LBM_EDEVICE;
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return fail_hip(ctx, e_, #call); \
    } while (0)

void* dev_alloc(lbm_ctx* c, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (c->alloc) {
        p = c->alloc(bytes, c->user);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (p) {
        c->allocations.emplace_back(p, bytes);
        c->device_bytes += bytes;
    }
    return p;
}

// Two timing events, destroyed on every return path.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t create() {
        hipError_t e = hipEventCreate(&e0);
        return e == hipSuccess ? hipEventCreate(&e1) : e;
    }
    ~EventPair() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Free one temporary allocation made by dev_alloc.  Calls that fail after
// making a temporary leave it in the context's list, to be freed by
// lbm_destroy: work already queued on the stream may still use it.
void dev_release(lbm_ctx* c, void* p) {
    auto it = std::find_if(c->allocations.begin(), c->allocations.end(),
                           [p](const std::pair<void*, size_t>& a) { return a.first == p; });
    if (it == c->allocations.end()) return;
    c->device_bytes -= it->second;
    c->allocations.erase(it);
    if (c->free_fn) c->free_fn(p, c->user);
    else (void)hipFree(p);
}

void dev_free_all(lbm_ctx* c) {
    for (auto& a : c->allocations) {
        if (c->free_fn) c->free_fn(a.first, c->user);
        else (void)hipFree(a.first);
    }
    c->allocations.clear();
    c->device_bytes = 0;
}

int validate(const lbm_params& p) {
    if (p.nx < 4 || p.ny < 4) return LBM_EINVAL;
    if (p.n_waves <= 0 || p.nx % p.n_waves != 0) return LBM_EINVAL;
    if (p.reserved != 0) return LBM_EINVAL;
    if (!(p.W > 0) || !(p.b > p.W) || !(p.b < p.ny - p.W)) return LBM_EINVAL;
    if (!(p.M_phi > 0) || !(p.rho_a > 0) || !(p.rho_b > 0)) return LBM_EINVAL;
    if (!(p.mu_a > 0) || !(p.mu_b > 0) || !(p.k_a > 0) || !(p.k_b > 0)) return LBM_EINVAL;
    const double vals[] = {p.sigma0, p.sigma_T, p.sigma_TT, p.T_ref, p.T_h, p.dT, p.T_c, p.Fx_ext, p.Fy_ext};
    for (double v : vals)
        if (!std::isfinite(v)) return LBM_EINVAL;
    // populations are addressed by 32-bit byte offsets within a channel
    if (27LL * 8LL * p.nx * p.ny >= (1LL << 32)) return LBM_EINVAL;
    return LBM_OK;
}

int tiles_of(const lbm_params& p, int tx, int ty, int* tiles_x) {
    int txs = (p.nx + tx - 1) / tx, tys = (p.ny + ty - 1) / ty;
    if (tiles_x) *tiles_x = txs;
    return txs * tys;
}

// Tile layout of a channel: tiles_x, tiles_y and the strip width (in tiles).
// Float32: eight strips across the channel, so that a channel that fills the
// GPU hands one full-height strip to each of the eight XCDs.  Float64: four
// strips, each XCD taking half of one (measured on 4096 x 2048: 1.2% faster
// and 3% fewer HBM reads than eight strips in float64, 4% slower in float32).
void set_layout(Inst& I, const lbm_params& p, int tx, int ty, int prec) {
    I.tiles_x = (p.nx + tx - 1) / tx;
    I.tiles_y = (p.ny + ty - 1) / ty;
    const int strips = prec == LBM_FP64 ? 4 : 8;
    I.strip_w = std::max(1, (I.tiles_x + strips - 1) / strips);
}

// Build the tile table for the current tile shape over the channels whose
// host flag says active (all channels when all == true).
int build_tiles(lbm_ctx* c, bool all) {
    c->h_tile_inst.clear();
    for (int k = 0; k < c->n_inst; ++k) {
        int nt = tiles_of(c->params[k], c->tx, c->ty, nullptr);
        set_layout(c->h_inst[k], c->params[k], c->tx, c->ty, c->prec);
        c->h_inst[k].ntiles = nt;
        c->h_inst[k].tile0 = (int)c->h_tile_inst.size();
        if (all || !c->retired[k]) {
            for (int t = 0; t < nt; ++t) c->h_tile_inst.push_back(k);
        } else {
            c->h_inst[k].ntiles = 0;
        }
    }
    c->n_tiles = (int)c->h_tile_inst.size();
    if (c->n_tiles > c->tile_cap) return LBM_EINVAL;  // capacity sized for the smallest tile at create
    return LBM_OK;
}

int upload_tables(lbm_ctx* c) {
    // descriptors carry an 'active' flag owned by the device; write only the
    // layout fields, keeping the flag from the device copy
    std::vector<Inst> cur(c->n_inst);
    HIPCHK(c, hipMemcpyAsync(cur.data(), c->d_inst, sizeof(Inst) * c->n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->n_inst; ++k) c->h_inst[k].active = cur[k].active;
    HIPCHK(c, hipMemcpyAsync(c->d_inst, c->h_inst.data(), sizeof(Inst) * c->n_inst, hipMemcpyHostToDevice, c->stream));
    if (c->n_tiles > 0)
        HIPCHK(c, hipMemcpyAsync(c->d_tile_inst, c->h_tile_inst.data(), sizeof(int) * c->n_tiles,
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int grid_of(int n_tiles) { return ((n_tiles + 7) / 8) * 8; }

void step_args(lbm_ctx* c, StepArgs& a, bool parity) {
    a.insts = c->d_inst;
    a.tile_inst = c->d_tile_inst;
    a.n_tiles = c->n_tiles;
    a.src_v = parity ? c->popB : c->popA;
    a.dst_v = parity ? c->popA : c->popB;
    a.phi0_v = c->phi0;
    a.tw_v = c->twall;
    a.phir_v = c->phir;
    a.fq_v = c->fq;
    a.fr_v = c->fr;
    a.fqw_v = c->fq;
    a.rowpart = c->rowpart;
    a.tref_v = c->tref;
    a.tref_out = c->tref_new;
    a.dl_v = c->dl;
    a.dl_out = c->dl_new;
    a.dlz = c->dlz;
    for (int k = 0; k < 4; ++k) a.snap[k] = c->snap + (size_t)k * c->total_nodes;
    a.partials = c->partials;
    for (int k = 0; k < 5; ++k) a.out[k] = nullptr;
}

void fin_args(lbm_ctx* c, FinArgs& f) {
    f.insts = c->d_inst;
    f.results = c->d_res;
    f.partials = c->partials;
    f.chk = c->chk;
    f.chk_nb = c->chk_nb;
    for (int k = 0; k < 4; ++k) f.snap[k] = c->snap + (size_t)k * c->total_nodes;
    f.step_counter = c->d_counter;
    f.tol = c->d_tol;
}

void flux_args(lbm_ctx* c, FluxArgs& f) {
    f.insts = c->d_inst;
    f.fq = (float*)c->fq;
    f.fq_next = c->fq_next;
    f.fr = (float*)c->fr;
    f.fr_next = c->fr_next;
    f.fr_sw = c->fr_sw;
    f.frc = c->frc;
    f.rowpart = c->rowpart;
}

// Float32 mode: every flux table of rows [r0, r0 + n) back to the set-up one.
int reset_flux_tables(lbm_ctx* c, long long r0, long long n) {
    if (c->prec != LBM_FP32_DEV || n <= 0) return LBM_OK;
    const size_t b = (size_t)n * sizeof(float);
    float* dst[5] = {(float*)c->fq + r0, c->fq_next + r0, (float*)c->fr + r0, c->fr_next + r0, c->fr_sw + r0};
    const float* src[5] = {c->fq_cold + r0, c->fq_cold + r0, c->fr_cold + r0, c->fr_cold + r0, c->fr_cold + r0};
    for (int k = 0; k < 5; ++k)
        HIPCHK(c, hipMemcpyAsync(dst[k], src[k], b, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

// One step starting at global step index `s` (state in buffer s % 2).
int enqueue_step(lbm_ctx* c, long long s) {
    StepArgs a;
    step_args(c, a, (s & 1) != 0);
    const bool check = (s % CHECK_EVERY) == 0;
    // float32 mode: the step after a check stores its f populations against
    // the flux reference that check computed
    const bool flux_switch = c->prec == LBM_FP32_DEV && (s % CHECK_EVERY) == 1;
    if (flux_switch) {
        a.fqw_v = c->fq_next;
        a.fr_v = c->fr_sw;
    }
    if (c->n_tiles > 0) {
        hipError_t e = launch_step(c->prec, a, check ? 1 : 0, grid_of(c->n_tiles), c->tx, c->ty, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "step kernel launch");
    }
    if ((check || flux_switch) && c->prec == LBM_FP32_DEV) {
        FluxArgs fa;
        flux_args(c, fa);
        hipError_t e = check ? launch_flux_next(fa, c->max_rows, c->n_inst, c->stream)
                             : launch_flux_copy(fa, c->max_rows, c->n_inst, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "flux reference launch");
    }
    if (check && c->prec == LBM_FP32_DEV) {
        // the check step stored its populations relative to new temperature
        // and phi references; make those current (before the check may retire
        // a channel)
        TrefArgs r;
        r.insts = c->d_inst;
        r.tref = c->tref;
        r.tref_new = c->tref_new;
        r.dl = c->dl;
        r.dl_new = c->dl_new;
        hipError_t e = launch_tref_copy(r, c->max_nodes, c->n_inst, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "reference copy launch");
        e = launch_dl_flags(c->d_inst, c->dl, c->dlz, c->max_chunks, c->n_inst, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "offset flag launch");
    }
    if (check) {
        FinArgs f;
        fin_args(c, f);
        hipError_t e = launch_finalize(f, c->n_inst, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "check kernel launch");
        e = launch_counter(c->d_counter, CHECK_EVERY, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "counter kernel launch");

    }
    return LBM_OK;
}

void drop_graph(lbm_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// Capture 100 steps starting at an even global step that is a multiple of
// the check interval (state in buffer A): check step, check kernel, counter,
// then 99 plain steps.  The step count is even, so the replay ends in A.
int build_graph(lbm_ctx* c) {
    drop_graph(c);
    hipStream_t cap;
    HIPCHK(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { (void)hipStreamDestroy(cap); return fail_hip(c, e, "hipStreamBeginCapture"); }
    hipStream_t saved = c->stream;
    c->stream = cap;
    int rc = LBM_OK;
    for (long long s = 0; s < CHECK_EVERY && rc == LBM_OK; ++s) rc = enqueue_step(c, s);
    c->stream = saved;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (rc != LBM_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail_hip(c, e, "hipStreamEndCapture");
    c->graph = g;
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_graph(c); return fail_hip(c, e, "hipGraphInstantiate"); }
    c->graph_tx = c->tx;
    c->graph_ty = c->ty;
    c->graph_ntiles = c->n_tiles;
    return LBM_OK;
}

int refresh_results(lbm_ctx* c, std::vector<Result>& res) {
    res.resize(c->n_inst);
    HIPCHK(c, hipMemcpyAsync(res.data(), c->d_res, sizeof(Result) * c->n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->n_inst; ++k) c->retired[k] = res[k].retired_at > 0 ? 1 : 0;
    return LBM_OK;
}

long long inst_steps(lbm_ctx* c, const Result& r) { return r.retired_at > 0 ? r.retired_at : c->steps; }

}  // namespace

extern "C" {

const char* lbm_strerror(int status) {
    switch (status) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "device allocation failed";
        case LBM_EDEVICE: return g_err.empty() ? "HIP runtime error" : g_err.c_str();
        case LBM_EDIVERGED: return "non-finite value in the solution";
        case LBM_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

int lbm_create(const lbm_params* params, int32_t n_inst, int32_t precision, void* hip_stream,
               lbm_alloc_fn alloc, lbm_free_fn free_fn, void* user, lbm_ctx** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!params || n_inst <= 0 || (precision != LBM_FP64 && precision != LBM_FP32_DEV)) return LBM_EINVAL;
    if ((alloc == nullptr) != (free_fn == nullptr)) return LBM_EINVAL;
    for (int k = 0; k < n_inst; ++k) {
        int rc = validate(params[k]);
        if (rc) return rc;
    }
    lbm_ctx* c = new lbm_ctx();
    c->n_inst = n_inst;
    c->prec = precision;
    c->elem = precision == LBM_FP64 ? 8 : 4;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    c->params.assign(params, params + n_inst);
    c->retired.assign(n_inst, 0);
    // NULL selects the null stream (ordered with all blocking streams)
    c->stream = (hipStream_t)hip_stream;
    // layout
    c->h_inst.resize(n_inst);
    long long pop = 0, nodes = 0, rows = 0, cols = 0, chunks = 0, rp = 0;
    long long max_tiles = 0;
    for (int k = 0; k < n_inst; ++k) {
        const lbm_params& p = params[k];
        Inst& I = c->h_inst[k];
        std::memset(&I, 0, sizeof(Inst));
        I.nx = p.nx;
        I.ny = p.ny;
        I.active = 1;
        I.pop_off = pop;
        I.node_off = nodes;
        I.row_off = rows;
        I.col_off = cols;
        I.chunk_off = chunks;
        I.rp_off = rp;
        I.rp_stride = (p.nx + 15) / 16;
        I.W = p.W;
        I.M_phi = p.M_phi;
        I.w_phi = 1.0 / (3.0 * p.M_phi + 0.5);
        I.b = p.b;
        I.rho_a = p.rho_a; I.rho_b = p.rho_b; I.mu_a = p.mu_a; I.mu_b = p.mu_b;
        I.k_a = p.k_a; I.k_b = p.k_b;
        I.s0 = p.sigma0; I.sT = p.sigma_T; I.sTT = p.sigma_TT; I.T_ref = p.T_ref;
        I.T_h = p.T_h; I.dT = p.dT; I.T_c = p.T_c;
        I.kx = 2.0 * M_PI / ((double)p.nx / (double)p.n_waves);
        I.Fx = p.Fx_ext; I.Fy = p.Fy_ext;
        // storage reference of g: the rest pressure 1/3, rounded to a float
        // value so that the float32 kernel and the float64 set-up code use
        // the very same number
        I.p_r = precision == LBM_FP64 ? 0.0 : (double)(float)(1.0 / 3.0);
        const long long n = (long long)p.nx * p.ny;
        pop += 27 * n;
        nodes += n;
        rows += p.ny + 4;
        cols += p.nx;
        rp += (long long)p.ny * ((p.nx + 15) / 16);
        c->max_rows = std::max(c->max_rows, p.ny);
        {
            const long long ch = (long long)((p.nx + DLZ_CX - 1) / DLZ_CX) * ((p.ny + DLZ_CY - 1) / DLZ_CY);
            chunks += ch;
            c->max_chunks = std::max<int>(c->max_chunks, (int)ch);
        }
        c->max_nodes = std::max<long long>(c->max_nodes, n);
        // tile-table capacity: the worst case over the compiled tile shapes
        long long t = 0;
        for (auto& s : TILE_SHAPES) t = std::max<long long>(t, (long long)tiles_of(p, s[0], s[1], nullptr));
        max_tiles += t;
        c->chk_nb = std::max<int>(c->chk_nb, (int)((t + CHK_TILES - 1) / CHK_TILES));
    }
    c->total_pop = pop;
    c->total_nodes = nodes;
    c->total_rows = rows;
    c->total_cols = cols;
    c->tile_cap = (int)max_tiles;
    c->partial_cap = (int)max_tiles;
    int rc = LBM_OK;
    c->popA = dev_alloc(c, (size_t)pop * c->elem);
    c->popB = dev_alloc(c, (size_t)pop * c->elem);
    c->phi0 = dev_alloc(c, (size_t)rows * c->elem);
    c->phir = dev_alloc(c, (size_t)rows * c->elem);
    c->fq = dev_alloc(c, (size_t)rows * c->elem);
    c->fr = dev_alloc(c, (size_t)rows * c->elem);
    c->twall = (double*)dev_alloc(c, (size_t)cols * sizeof(double));
    if (precision == LBM_FP32_DEV) {
        c->tref = (float*)dev_alloc(c, (size_t)nodes * sizeof(float));
        c->tref_new = (float*)dev_alloc(c, (size_t)nodes * sizeof(float));
        c->dl = (int32_t*)dev_alloc(c, (size_t)nodes * sizeof(int32_t));
        c->dl_new = (int32_t*)dev_alloc(c, (size_t)nodes * sizeof(int32_t));
        c->dlz = (int32_t*)dev_alloc(c, (size_t)chunks * sizeof(int32_t));
        c->fq_next = (float*)dev_alloc(c, (size_t)rows * sizeof(float));
        c->fr_next = (float*)dev_alloc(c, (size_t)rows * sizeof(float));
        c->fr_sw = (float*)dev_alloc(c, (size_t)rows * sizeof(float));
        c->fq_cold = (float*)dev_alloc(c, (size_t)rows * sizeof(float));
        c->fr_cold = (float*)dev_alloc(c, (size_t)rows * sizeof(float));
        c->frc = (double*)dev_alloc(c, (size_t)rows * sizeof(double));
        c->rowpart = (double*)dev_alloc(c, (size_t)rp * sizeof(double));
        if (!c->tref || !c->tref_new || !c->dl || !c->dl_new || !c->dlz || !c->fq_next || !c->fr_next || !c->fr_sw ||
            !c->fq_cold || !c->fr_cold || !c->frc || !c->rowpart)
            rc = LBM_ENOMEM;
    }
    c->snap = (double*)dev_alloc(c, (size_t)nodes * 4 * sizeof(double));
    c->partials = (double*)dev_alloc(c, (size_t)max_tiles * 8 * sizeof(double));
    c->chk = (double*)dev_alloc(c, (size_t)n_inst * c->chk_nb * 9 * sizeof(double));
    c->d_inst = (Inst*)dev_alloc(c, sizeof(Inst) * n_inst);
    c->d_tile_inst = (int*)dev_alloc(c, sizeof(int) * max_tiles);
    c->d_res = (Result*)dev_alloc(c, sizeof(Result) * n_inst);
    c->d_counter = (long long*)dev_alloc(c, sizeof(long long));
    c->d_tol = (double*)dev_alloc(c, sizeof(double));
    c->d_active = (int*)dev_alloc(c, sizeof(int));
    if (!c->popA || !c->popB || !c->phi0 || !c->phir || !c->fq || !c->fr || !c->twall || !c->snap || !c->partials || !c->chk || !c->d_inst || !c->d_tile_inst ||
        !c->d_res || !c->d_counter || !c->d_tol || !c->d_active) {
        rc = LBM_ENOMEM;
    }
    if (rc == LBM_OK && hipHostMalloc((void**)&c->h_active, sizeof(int), hipHostMallocDefault) != hipSuccess)
        rc = LBM_ENOMEM;
    if (rc == LBM_OK) {
        // reference rows (float32 mode), rows -2 .. ny+1.  phi0: cold-start
        // tanh profile, the storage reference (float values).  A node pulls
        // populations stored relative to w_a phi0(source row) (the source row
        // of a wall link is the node's own row); dR is the zeroth moment of
        // those references taken relative to phi0(row).  dR is rounded to
        // float and then corrected by single ulps until the float values sum
        // to zero exactly, as the exact values do: the float32 step then
        // conserves sum phi up to the rounding of small deviations.
        //
        // Flux reference of f.  At the interface the post-collision first
        // moment of f (relaxed towards M theta n) is ~1e-2, far above the
        // deviations of a near-steady state, and rounding it in float32 would
        // put noise of its ulp into phi every step.  f is therefore also
        // stored relative to q_a: +A(row)/2 on (0,+1), -A(row)/2 on (0,-1),
        // whose raw moments are zero except m01 = A.  A is the fixed point of
        // the ACE first-moment relaxation of the flat reference profile at
        // rest (phi = phi0, u = 0, pull streaming, specular walls):
        //   A(j) = (1 - w) [r01(j) + (A(j-1) + A(j+1)) / 2] + w M theta0 n0y,
        // with r01 the pulled y-moment of w_a phi0 and A(-1) = -A(0),
        // A(ny) = -A(ny-1) (the wall image of q), solved as a tridiagonal
        // system.  fq = A/2 (float).  fr is what the stored post-collision
        // y-moment keeps of the references after that subtraction,
        //   fr(j) = (1 - w)(r01 + fq(j-1) + fq(j+1)) + w M theta0 n0y - 2 fq(j),
        // with theta0, n0y of the reference profile as the step kernel forms
        // them, so the kernel relaxes only deviations (tiny near steady
        // state).  Any A is exact up to rounding; this one makes the stored
        // values small.
        std::vector<double> t0(rows, 0.0), tr(rows, 0.0), tq(rows, 0.0), tf(rows, 0.0), tc(rows, 0.0);
        if (precision == LBM_FP32_DEV) {
            const int EYh[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
            const double Wh[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
            for (int k = 0; k < n_inst; ++k) {
                const lbm_params& p = params[k];
                const int ny = p.ny;
                double* q0 = &t0[c->h_inst[k].row_off + 2];
                double* qr = &tr[c->h_inst[k].row_off + 2];
                double* qq = &tq[c->h_inst[k].row_off + 2];
                double* qf = &tf[c->h_inst[k].row_off + 2];
                for (int j = 0; j < ny; ++j)
                    q0[j] = (double)(float)(0.5 * (1.0 + std::tanh(2.0 * ((p.b - 0.5) - (double)j) / p.W)));
                // ghost rows mirror the rows next to the walls, as phi does
                q0[-1] = q0[0]; q0[-2] = q0[1];
                q0[ny] = q0[ny - 1]; q0[ny + 1] = q0[ny - 2];
                std::vector<double> r01(ny);
                for (int j = 0; j < ny; ++j) {
                    double s0 = 0.0, s1 = 0.0;
                    for (int a2 = 0; a2 < 9; ++a2) {
                        int js = j - EYh[a2];
                        if (js < 0 || js >= ny) js = j;
                        s0 += Wh[a2] * (q0[js] - q0[j]);
                        s1 += Wh[a2] * EYh[a2] * q0[js];
                    }
                    qr[j] = (double)(float)s0;
                    r01[j] = s1;
                }
                // exact-sum correction of the rounded dR (compensated sum)
                auto fsum = [&]() {
                    double s = 0.0, comp = 0.0;
                    for (int j = 0; j < ny; ++j) {
                        double y = qr[j] - comp, t = s + y;
                        comp = (t - s) - y;
                        s = t;
                    }
                    return s;
                };
                for (int it = 0; it < 4 * ny; ++it) {
                    const double S = fsum();
                    if (S == 0.0) break;
                    // adjust the row whose float step best matches the residual
                    int best = -1;
                    double bestv = 0.0, bestr = std::fabs(S);
                    for (int j = 0; j < ny; ++j) {
                        const float o = (float)qr[j];
                        const float nv = S > 0 ? std::nextafter(o, -INFINITY) : std::nextafter(o, INFINITY);
                        const double r = std::fabs(S + ((double)nv - (double)o));
                        if (r < bestr) { bestr = r; best = j; bestv = nv; }
                    }
                    if (best < 0) break;
                    qr[best] = bestv;
                }
                // flux reference: tridiagonal solve (Thomas), rows 0 .. ny-1
                const double w = 1.0 / (3.0 * p.M_phi + 0.5), cc = 0.5 * (1.0 - w);
                const double eps2 = EPS_N * EPS_N;
                auto mth = [&](double ph, double gy) {   // M theta n_y of a flat profile
                    return p.M_phi * 4.0 * ph * (1.0 - ph) / p.W * (gy / std::sqrt(gy * gy + eps2));
                };
                std::vector<double> lo(ny), di(ny), up(ny), rhs(ny), A(ny);
                for (int j = 0; j < ny; ++j) {
                    // the physical profile: phi mirrored about the walls
                    const double pm = j > 0 ? q0[j - 1] : q0[0], pp = j < ny - 1 ? q0[j + 1] : q0[ny - 1];
                    rhs[j] = (1.0 - w) * r01[j] + w * mth(q0[j], 0.5 * (pp - pm));
                    lo[j] = -cc;
                    up[j] = -cc;
                    di[j] = 1.0;
                }
                di[0] += cc;            // A(-1) = -A(0)
                di[ny - 1] += cc;       // A(ny) = -A(ny-1)
                if (ny == 1) di[0] = 1.0 + 2.0 * cc;
                for (int j = 1; j < ny; ++j) {
                    const double m = lo[j] / di[j - 1];
                    di[j] -= m * up[j - 1];
                    rhs[j] -= m * rhs[j - 1];
                }
                A[ny - 1] = rhs[ny - 1] / di[ny - 1];
                for (int j = ny - 2; j >= 0; --j) A[j] = (rhs[j] - up[j] * A[j + 1]) / di[j];
                for (int j = 0; j < ny; ++j) qq[j] = (double)(float)(0.5 * A[j]);
                qq[-1] = -qq[0];
                qq[ny] = -qq[ny - 1];
                for (int j = 0; j < ny; ++j) {
                    // reference theta0, n0y as the step kernel forms them
                    // (mirrored ghost rows)
                    const double fq_sum = qq[j - 1] + qq[j + 1];
                    const double rest = mth(q0[j], 0.5 * (q0[j + 1] - q0[j - 1]));
                    qf[j] = (double)(float)((1.0 - w) * (r01[j] + fq_sum) + w * rest - 2.0 * qq[j]);
                    tc[c->h_inst[k].row_off + 2 + j] = (1.0 - w) * r01[j] + w * rest;
                }
            }
        }
        // every set-up copy goes on the context's stream (which the caller
        // may have created non-blocking) and completes before its host
        // source goes out of scope
        auto upload = [&](void* dst, const std::vector<double>& v) -> hipError_t {
            hipError_t e;
            if (precision == LBM_FP64) {
                e = hipMemcpyAsync(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            } else {
                std::vector<float> f(v.begin(), v.end());
                e = hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            }
            return e;
        };
        if (upload(c->phi0, t0) != hipSuccess || upload(c->phir, tr) != hipSuccess || upload(c->fq, tq) != hipSuccess ||
            upload(c->fr, tf) != hipSuccess)
            rc = fail_hip(c, hipErrorUnknown, "upload reference rows");
        if (rc == LBM_OK && precision == LBM_FP32_DEV) {
            // the set-up flux tables, kept to start from again (lbm_init, lbm_restart)
            std::vector<float> q32(tq.begin(), tq.end()), f32(tf.begin(), tf.end());
            hipError_t e = hipMemcpyAsync(c->fq_cold, q32.data(), rows * sizeof(float), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->fr_cold, f32.data(), rows * sizeof(float), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->frc, tc.data(), rows * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rc = fail_hip(c, e, "upload flux tables");
        }
    }
    if (rc == LBM_OK) {
        // bottom-wall temperature T_h + dT cos(2 pi i / l) for every column
        std::vector<double> td(cols);
        for (int k = 0; k < n_inst; ++k) {
            const lbm_params& p = params[k];
            const double l = (double)p.nx / (double)p.n_waves;
            for (int i = 0; i < p.nx; ++i)
                td[c->h_inst[k].col_off + i] = p.T_h + p.dT * std::cos(2.0 * M_PI * (double)i / l);
        }
        hipError_t e;
        e = hipMemcpyAsync(c->twall, td.data(), cols * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = fail_hip(c, e, "upload wall temperatures");
    }
    if (rc == LBM_OK) rc = build_tiles(c, true);
    if (rc == LBM_OK) {
        const double tol = -1.0;
        if (hipMemcpyAsync(c->d_inst, c->h_inst.data(), sizeof(Inst) * n_inst, hipMemcpyHostToDevice, c->stream) !=
                hipSuccess ||
            hipMemcpyAsync(c->d_tile_inst, c->h_tile_inst.data(), sizeof(int) * c->n_tiles, hipMemcpyHostToDevice,
                           c->stream) != hipSuccess ||
            hipMemsetAsync(c->d_res, 0, sizeof(Result) * n_inst, c->stream) != hipSuccess ||
            hipMemsetAsync(c->d_counter, 0, sizeof(long long), c->stream) != hipSuccess ||
            hipMemcpyAsync(c->d_tol, &tol, sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = fail_hip(c, hipErrorUnknown, "upload descriptors");
        }
    }
    if (rc != LBM_OK) {
        lbm_destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    dev_free_all(c);
    if (c->h_active) (void)hipHostFree(c->h_active);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int lbm_set_tile(lbm_ctx* c, int32_t tx, int32_t ty) {
    if (!c) return LBM_EINVAL;
    if (tx == 0 && ty == 0) { tx = TILE_SHAPES[0][0]; ty = TILE_SHAPES[0][1]; }
    bool ok = false;
    for (auto& s : TILE_SHAPES) ok = ok || (s[0] == tx && s[1] == ty);
    if (!ok) return LBM_EINVAL;
    // the tile shape may change at any step: the buffers do not depend on it
    c->tx = tx;
    c->ty = ty;
    int rc = build_tiles(c, !c->initialised);
    if (rc) return rc;
    return upload_tables(c);
}

static int init_impl(lbm_ctx* c, const double* fields, bool device) {
    if (!c) return LBM_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // reset descriptors (all active), results, counter
    for (int k = 0; k < c->n_inst; ++k) { c->h_inst[k].active = 1; c->retired[k] = 0; }
    int rc = build_tiles(c, true);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->d_inst, c->h_inst.data(), sizeof(Inst) * c->n_inst, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_tile_inst, c->h_tile_inst.data(), sizeof(int) * c->n_tiles, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_res, 0, sizeof(Result) * c->n_inst, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_counter, 0, sizeof(long long), c->stream));
    HIPCHK(c, hipMemsetAsync(c->snap, 0, sizeof(double) * 4 * c->total_nodes, c->stream));
    rc = reset_flux_tables(c, 0, c->total_rows);
    if (rc) return rc;
    InitArgs a;
    a.insts = c->d_inst;
    a.dst_v = c->popA;
    a.phi0_v = c->phi0;
    a.fq_v = c->fq;
    a.tw_v = c->twall;
    a.tref = c->tref;
    a.dl = c->dl;
    a.cold = fields ? 0 : 1;
    a.field_base = 0;
    double* dfields = nullptr;
    if (fields) {
        if (!device)
            for (long long q = 0; q < 4 * c->total_nodes; ++q)
                if (!std::isfinite(fields[q])) return LBM_EINVAL;
        dfields = (double*)dev_alloc(c, sizeof(double) * 4 * c->total_nodes);
        if (!dfields) return LBM_ENOMEM;
        // input layout: per instance [phi|ux|uy|T]; kernel layout: field-major over all nodes
        const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        for (int k = 0; k < c->n_inst; ++k) {
            const long long n = (long long)c->params[k].nx * c->params[k].ny;
            const double* src = fields + 4 * c->h_inst[k].node_off;
            for (int f = 0; f < 4; ++f)
                HIPCHK(c, hipMemcpyAsync(dfields + f * c->total_nodes + c->h_inst[k].node_off, src + f * n,
                                         sizeof(double) * n, kind, c->stream));
        }
        for (int f = 0; f < 4; ++f) a.fields[f] = dfields + f * c->total_nodes;
    } else {
        for (int f = 0; f < 4; ++f) a.fields[f] = nullptr;
    }
    hipError_t e = launch_init(c->prec, a, c->max_nodes, c->n_inst, c->stream);
    if (e != hipSuccess) return fail_hip(c, e, "init kernel launch");
    if (c->prec == LBM_FP32_DEV) {
        e = launch_dl_flags(c->d_inst, c->dl, c->dlz, c->max_chunks, c->n_inst, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "offset flag launch");
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (dfields) dev_release(c, dfields);
    c->steps = 0;
    c->initialised = true;
    return LBM_OK;
}

int lbm_init(lbm_ctx* c, const double* fields) { return init_impl(c, fields, false); }

int lbm_init_device(lbm_ctx* c, const double* fields) {
    if (!fields) return LBM_EINVAL;
    return init_impl(c, fields, true);
}

int lbm_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    for (int64_t k = 0; k < n; ++k) {
        int rc = enqueue_step(c, c->steps);
        if (rc) return rc;
        c->steps += 1;
    }
    return LBM_OK;
}

int lbm_solve(lbm_ctx* c, double r_tol, int64_t max_steps, int32_t* n_active) {
    if (!c || !(r_tol > 0) || max_steps < 0) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    HIPCHK(c, hipMemcpyAsync(c->d_tol, &r_tol, sizeof(double), hipMemcpyHostToDevice, c->stream));
    int64_t done = 0;
    int rc = LBM_OK;
    std::vector<Result> res;
    // align to the check interval with single steps
    while (done < max_steps && (c->steps % CHECK_EVERY) != 0) {
        rc = enqueue_step(c, c->steps);
        if (rc) break;
        c->steps += 1;
        ++done;
    }
    int last_active = c->n_inst;
    while (rc == LBM_OK && done + CHECK_EVERY <= max_steps) {
        if (!c->graph_exec || c->graph_tx != c->tx || c->graph_ty != c->ty || c->graph_ntiles != c->n_tiles) {
            rc = build_graph(c);
            if (rc) break;
        }
        hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);
        if (e != hipSuccess) { rc = fail_hip(c, e, "hipGraphLaunch"); break; }
        c->steps += CHECK_EVERY;
        done += CHECK_EVERY;
        e = launch_count_active(c->d_inst, c->n_inst, c->d_active, c->stream);
        if (e != hipSuccess) { rc = fail_hip(c, e, "count kernel"); break; }
        e = hipMemcpyAsync(c->h_active, c->d_active, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) { rc = fail_hip(c, e, "hipMemcpyAsync"); break; }
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) { rc = fail_hip(c, e, "hipStreamSynchronize"); break; }
        const int act = *c->h_active;
        if (act == 0) break;
        if (act <= (3 * last_active) / 4 && c->n_inst > 1) {
            // drop the tiles of retired channels from the launch
            rc = refresh_results(c, res);
            if (rc) break;
            rc = build_tiles(c, false);
            if (rc) break;
            rc = upload_tables(c);
            if (rc) break;
            last_active = act;
        }
    }
    double off = -1.0;
    (void)hipMemcpyAsync(c->d_tol, &off, sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (rc) return rc;
    rc = refresh_results(c, res);
    if (rc) return rc;
    int act = 0;
    bool bad = false;
    for (int k = 0; k < c->n_inst; ++k) {
        if (res[k].retired_at == 0) ++act;
        if (res[k].bad > 0) bad = true;
    }
    if (n_active) *n_active = act;
    return bad ? LBM_EDIVERGED : LBM_OK;
}

int lbm_retire(lbm_ctx* c, int32_t inst) {
    if (!c || inst < 0 || inst >= c->n_inst) return LBM_EINVAL;
    // a retirement step of 0 would read as "not retired"
    if (!c->initialised || c->steps == 0) return LBM_ESTATE;
    std::vector<Result> res;
    int rc = refresh_results(c, res);
    if (rc) return rc;
    if (res[inst].retired_at > 0) return LBM_OK;          // already retired
    // the channel keeps the state of the current step: record it as retired
    // there, switch its descriptor off and drop its tiles from the launches
    Result R = res[inst];
    R.retired_at = c->steps;
    const int off = 0;
    HIPCHK(c, hipMemcpyAsync(c->d_res + inst, &R, sizeof(Result), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync((char*)(c->d_inst + inst) + offsetof(Inst, active), &off, sizeof(int),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->retired[inst] = 1;
    rc = build_tiles(c, false);
    if (rc) return rc;
    return upload_tables(c);
}

int lbm_restart(lbm_ctx* c, int32_t inst, const double* fields) {
    if (!c || inst < 0 || inst >= c->n_inst) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    const long long n = (long long)c->params[inst].nx * c->params[inst].ny;
    if (fields)
        for (long long q = 0; q < 4 * n; ++q)
            if (!std::isfinite(fields[q])) return LBM_EINVAL;
    // bring the host's retirement flags up to date, then take this channel
    // back into the launches with a fresh residual history
    std::vector<Result> res;
    int rc = refresh_results(c, res);
    if (rc) return rc;
    const Inst& I = c->h_inst[inst];
    InitArgs a;
    a.insts = c->d_inst + inst;                   // one instance: blockIdx.y == 0
    a.dst_v = (c->steps & 1) ? c->popB : c->popA; // the buffer the next step gathers from
    a.phi0_v = c->phi0;
    a.fq_v = c->fq;
    a.tw_v = c->twall;
    a.tref = c->tref;
    a.dl = c->dl;
    a.cold = fields ? 0 : 1;
    a.field_base = I.node_off;
    double* dfields = nullptr;
    for (int f = 0; f < 4; ++f) a.fields[f] = nullptr;
    if (fields) {
        dfields = (double*)dev_alloc(c, sizeof(double) * 4 * n);
        if (!dfields) return LBM_ENOMEM;
        HIPCHK(c, hipMemcpyAsync(dfields, fields, sizeof(double) * 4 * n, hipMemcpyHostToDevice, c->stream));
        for (int f = 0; f < 4; ++f) a.fields[f] = dfields + f * n;
    }
    rc = reset_flux_tables(c, I.row_off, (long long)c->params[inst].ny + 4);
    if (rc) return rc;
    const Result zero{};
    const int one = 1;
    HIPCHK(c, hipMemcpyAsync(c->d_res + inst, &zero, sizeof(Result), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync((char*)(c->d_inst + inst) + offsetof(Inst, active), &one, sizeof(int),
                             hipMemcpyHostToDevice, c->stream));
    hipError_t e = launch_init(c->prec, a, (int)n, 1, c->stream);
    if (e != hipSuccess) return fail_hip(c, e, "init kernel launch");
    if (c->prec == LBM_FP32_DEV) {
        e = launch_dl_flags(c->d_inst, c->dl, c->dlz, c->max_chunks, c->n_inst, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "offset flag launch");
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (dfields) dev_release(c, dfields);
    c->retired[inst] = 0;
    rc = build_tiles(c, false);
    if (rc) return rc;
    return upload_tables(c);
}

int lbm_fields(lbm_ctx* c, int32_t inst, double* phi, double* ux, double* uy, double* T, double* p) {
    if (!c || inst < 0 || inst >= c->n_inst) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    std::vector<Result> res;
    int rc = refresh_results(c, res);
    if (rc) return rc;
    const long long s = inst_steps(c, res[inst]);
    const lbm_params& P = c->params[inst];
    const long long n = (long long)P.nx * P.ny;
    double* out = (double*)dev_alloc(c, sizeof(double) * 5 * n);
    if (!out) return LBM_ENOMEM;
    // a one-channel tile table for this launch
    std::vector<int> tiles;
    int txs = 0;
    int nt = tiles_of(P, c->tx, c->ty, &txs);
    Inst I = c->h_inst[inst];
    I.tile0 = 0;
    set_layout(I, P, c->tx, c->ty, c->prec);
    I.ntiles = nt;
    I.active = 1;
    Inst* dI = (Inst*)dev_alloc(c, sizeof(Inst));
    int* dT = (int*)dev_alloc(c, sizeof(int) * nt);
    if (!dI || !dT) return LBM_ENOMEM;
    tiles.assign(nt, 0);
    HIPCHK(c, hipMemcpyAsync(dI, &I, sizeof(Inst), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dT, tiles.data(), sizeof(int) * nt, hipMemcpyHostToDevice, c->stream));
    StepArgs a;
    step_args(c, a, (s & 1) != 0);
    a.insts = dI;
    a.tile_inst = dT;
    a.n_tiles = nt;
    // the kernel writes at node_off + (j nx + i): shift the output pointers
    for (int k = 0; k < 5; ++k) a.out[k] = out + (size_t)k * n - I.node_off;
    hipError_t e = launch_step(c->prec, a, 2, grid_of(nt), c->tx, c->ty, c->stream);
    if (e != hipSuccess) return fail_hip(c, e, "fields kernel launch");
    double* dst[5] = {phi, ux, uy, T, p};
    for (int k = 0; k < 5; ++k)
        if (dst[k]) HIPCHK(c, hipMemcpyAsync(dst[k], out + (size_t)k * n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (void* q : {(void*)dT, (void*)dI, (void*)out}) dev_release(c, q);
    return LBM_OK;
}

int lbm_residual(lbm_ctx* c, int32_t inst, double* r, double* sum_phi, double* sum_mass, double* u_int_peak,
                 int64_t* steps_done) {
    if (!c || inst < 0 || inst >= c->n_inst) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    std::vector<Result> res;
    int rc = refresh_results(c, res);
    if (rc) return rc;
    const Result& R = res[inst];
    if (r) *r = R.have_prev ? R.r : INFINITY;
    if (sum_phi) *sum_phi = R.sum_phi;
    if (sum_mass) *sum_mass = R.sum_rho;
    if (u_int_peak) *u_int_peak = R.u_peak;
    if (steps_done) *steps_done = inst_steps(c, R);
    return R.bad > 0 ? LBM_EDIVERGED : LBM_OK;
}

static int state_io(lbm_ctx* c, int32_t inst, double* host, int dir) {
    if (!c || inst < 0 || inst >= c->n_inst || !host) return LBM_EINVAL;
    if (dir == 0 && !c->initialised) return LBM_ESTATE;
    std::vector<Result> res;
    int rc = refresh_results(c, res);
    if (rc) return rc;
    const long long s = c->initialised ? inst_steps(c, res[inst]) : 0;
    const lbm_params& P = c->params[inst];
    const long long n = (long long)P.nx * P.ny;
    double* d = (double*)dev_alloc(c, sizeof(double) * 27 * n);
    if (!d) return LBM_ENOMEM;
    StateArgs a;
    a.insts = c->d_inst;
    a.inst = inst;
    a.dir = dir;
    a.buf_v = (s & 1) ? c->popB : c->popA;
    a.phi0_v = c->phi0;
    a.fq_v = c->fq;
    a.tw_v = c->twall;
    a.tref = c->tref;
    a.dl = c->dl;
    a.state = d;
    if (dir == 1) HIPCHK(c, hipMemcpyAsync(d, host, sizeof(double) * 27 * n, hipMemcpyHostToDevice, c->stream));
    hipError_t e = launch_state(c->prec, a, (int)n, c->stream);
    if (e != hipSuccess) return fail_hip(c, e, "state kernel launch");
    if (dir == 0) HIPCHK(c, hipMemcpyAsync(host, d, sizeof(double) * 27 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dev_release(c, d);
    return LBM_OK;
}

int lbm_get_state(lbm_ctx* c, int32_t inst, double* pop) { return state_io(c, inst, pop, 0); }

int lbm_set_state(lbm_ctx* c, int32_t inst, const double* pop) {
    if (!c || inst < 0 || inst >= c->n_inst || !pop) return LBM_EINVAL;
    const long long n = 27LL * c->params[inst].nx * c->params[inst].ny;
    for (long long q = 0; q < n; ++q)
        if (!std::isfinite(pop[q])) return LBM_EINVAL;
    if (!c->initialised) {
        // a context that was never initialised starts at step 0 (cold start
        // for the other channels) and takes this state for channel inst
        int rc = lbm_init(c, nullptr);
        if (rc) return rc;
    }
    return state_io(c, inst, const_cast<double*>(pop), 1);
}

int lbm_profile_steps(lbm_ctx* c, int64_t n, double* ms) {
    if (!c || n <= 0 || !ms) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    EventPair ev;
    HIPCHK(c, ev.create());
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int64_t k = 0; k < n; ++k) {
        StepArgs a;
        step_args(c, a, (c->steps & 1) != 0);
        hipError_t e = launch_step(c->prec, a, 0, grid_of(c->n_tiles), c->tx, c->ty, c->stream);
        if (e != hipSuccess) return fail_hip(c, e, "step kernel launch");
        c->steps += 1;
    }
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / (double)n;
    // profiled steps record no checks: move the check counter to the step
    // index of the next check so that later checks report their own step
    long long next = ((c->steps + CHECK_EVERY - 1) / CHECK_EVERY) * CHECK_EVERY;
    HIPCHK(c, hipMemcpyAsync(c->d_counter, &next, sizeof(long long), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* tx_out, int32_t* ty_out, double* ms_out) {
    if (!c || reps <= 0) return LBM_EINVAL;
    if (!c->initialised) return LBM_ESTATE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    EventPair ev;
    HIPCHK(c, ev.create());
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    int best = -1;
    double best_ms = 0.0;
    const int tx0 = c->tx, ty0 = c->ty;
    int rc = LBM_OK;
    for (int s = 0; s < N_TILE_SHAPES && rc == LBM_OK; ++s) {
        rc = lbm_set_tile(c, TILE_SHAPES[s][0], TILE_SHAPES[s][1]);
        if (rc) break;
        // the state buffer is only read: every launch gathers from it and
        // writes the other buffer, which the next real step overwrites
        StepArgs a;
        step_args(c, a, (c->steps & 1) != 0);
        for (int w = 0; w < 2 + reps && rc == LBM_OK; ++w) {
            if (w == 2) {
                if (hipEventRecord(e0, c->stream) != hipSuccess) rc = fail_hip(c, hipErrorUnknown, "event");
            }
            hipError_t e = launch_step(c->prec, a, 0, grid_of(c->n_tiles), c->tx, c->ty, c->stream);
            if (e != hipSuccess) rc = fail_hip(c, e, "step kernel launch");
        }
        if (rc) break;
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
        const double ms = (double)t / reps;
        if (best < 0 || ms < best_ms) { best = s; best_ms = ms; }
    }
    if (rc) {
        (void)lbm_set_tile(c, tx0, ty0);
        return rc;
    }
    rc = lbm_set_tile(c, TILE_SHAPES[best][0], TILE_SHAPES[best][1]);
    if (rc) return rc;
    if (tx_out) *tx_out = TILE_SHAPES[best][0];
    if (ty_out) *ty_out = TILE_SHAPES[best][1];
    if (ms_out) *ms_out = best_ms;
    return LBM_OK;
}

int lbm_info(lbm_ctx* c, int64_t* nodes, int64_t* device_bytes) {
    if (!c) return LBM_EINVAL;
    if (nodes) *nodes = c->total_nodes;
    if (device_bytes) *device_bytes = (int64_t)c->device_bytes;
    return LBM_OK;
}

}  // extern "C"
