// lbm_internal.h -- structures shared by the host API and the device code of
// the HIP library (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Residual, conserved sums and interface peak are recorded every CHECK_EVERY
// steps (counted from initialisation).
constexpr int CHECK_EVERY = 100;
// Tiles per block of the check step's first pass (one tile per thread).
constexpr int CHK_TILES = 256;

// Tile shapes (nodes per workgroup, x by y) compiled for the fused step
// kernel; the first one is the default.
constexpr int N_TILE_SHAPES = 6;
constexpr int TILE_SHAPES[N_TILE_SHAPES][2] = {{64, 8}, {32, 8}, {64, 4}, {16, 16}, {64, 16}, {128, 8}};

// Regularisation of the interface normal where grad phi vanishes:
// n = grad phi / sqrt(|grad phi|^2 + EPS_N^2).
constexpr double EPS_N = 1e-6;
// Float32 mode: the per-node phi-reference offset is k DL_Q with integer k.
// With weights w = m / 36 (m = 16, 4, 1) every w dl is the integer m k times
// 2^-28, so the reference mass that pullers add back sums exactly (integer
// arithmetic) to the mass that writers removed.
constexpr double DL_U = 1.0 / 268435456.0;   // 2^-28
constexpr double DL_Q = 36.0 * DL_U;
// Flag table over 64 x 8 node chunks: nonzero where any phi-reference offset
// of the chunk is nonzero (float32 mode).  Lets a tile whose offsets are all
// zero skip reading them and summing them.
constexpr int DLZ_CX = 64, DLZ_CY = 8;

// Per-channel descriptor in device memory.
struct Inst {
    int nx, ny, tiles_x, tile0;   // tile0: first entry of this channel in the tile table
    int ntiles, active, tiles_y, strip_w;  // tiles are ordered in column strips of strip_w tiles
    long long pop_off;            // element offset of the channel in the population buffers
    long long node_off;           // element offset in node-sized arrays
    long long row_off;            // offset in the reference-row table (ny + 4 rows)
    long long col_off;            // offset in the bottom-wall temperature table (nx columns)
    long long chunk_off;          // offset in the phi-offset flag table (ceil(nx/64) x ceil(ny/8) chunks)
    long long rp_off;             // offset in the row-partial table of the flux reference (ny x rp_stride)
    int rp_stride, pad3;          // rp_stride = ceil(nx / 16): tile columns of the narrowest tile shape
    double W, M_phi, w_phi, b;
    double rho_a, rho_b, mu_a, mu_b, k_a, k_b;
    double s0, sT, sTT, T_ref;
    double T_h, dT, T_c, kx;      // kx = 2 pi / l
    double Fx, Fy;
    double p_r, pad2;             // storage reference of g (0 in float64 mode)
};

struct Result {
    double r, sum_phi, sum_rho, u_peak, bad;
    long long check_step, retired_at;
    int have_prev, pad;
};

struct StepArgs {
    const Inst* insts;
    const int* tile_inst;
    int n_tiles;
    const void* src_v;
    void* dst_v;
    const void* phi0_v;           // reference rows (compute type)
    const void* tw_v;             // bottom-wall temperature by column (float64)
    const void* phir_v;           // zeroth moment of the streamed reference populations minus phi0, by row
    const void* fq_v;             // flux reference: half the reference y-moment of f, by row
    const void* fr_v;             // constant part of the stored post-collision y-moment of f, by row
    const void* fqw_v;            // flux reference the writer subtracts (float32 mode): fq_v, except on
                                  // the step after a check, which moves to the new table
    double* rowpart;              // check steps: per row and tile column, sum of the f flux deviations
    const void* tref_v;           // per-node temperature reference (float32 mode)
    void* tref_out;               // new references written by a check step
    const int32_t* dl_v;          // per-node phi-reference offset from phi0(row), in units of DL_Q (float32 mode)
    int32_t* dl_out;              // new offsets written by a check step
    const int32_t* dlz;           // chunk flags of dl_v
    double* snap[4];              // ux, uy, T, phi at the last check
    double* partials;             // [tile][8]
    double* out[5];               // fields: phi, ux, uy, T, p
};

struct FinArgs {
    Inst* insts;
    Result* results;
    const double* partials;
    double* chk;                  // [instance][chk_nb][9]: per-block sums of the partials and interface peak
    int chk_nb;                   // blocks per instance of the first check pass (capacity)
    double* snap[4];
    const long long* step_counter;
    const double* tol;
};

struct InitArgs {
    const Inst* insts;
    void* dst_v;
    const void* phi0_v;
    const void* fq_v;
    const void* tw_v;
    float* tref;
    int32_t* dl;                  // phi-reference offsets, units of DL_Q (float32 mode)
    const double* fields[4];      // phi, ux, uy, T (device), when not cold
    long long field_base;         // node offset of the first node the field arrays hold
    int cold;
};

struct StateArgs {
    const Inst* insts;
    int inst;
    int dir;                      // 0: buffer -> state, 1: state -> buffer
    void* buf_v;
    const void* phi0_v;
    const void* fq_v;
    const void* tw_v;
    const float* tref;
    const int32_t* dl;
    double* state;                // device [3][9][ny][nx] float64
};

// Flux reference of f (float32 mode), moved after every check to the row
// mean of the actual flux (see flux_next_kernel).  Tables by row (ny + 4 per
// channel, float values): fq = A/2 read by the pulls, fr its companion.
struct FluxArgs {
    const Inst* insts;
    float* fq;                    // current
    float* fq_next;               // after the next switch step
    float* fr;                    // current
    float* fr_next;               // after the switch step
    float* fr_sw;                 // for the switch step itself (reads fq, writes fq_next)
    const double* frc;            // (1 - w_phi) r01 + w_phi M theta0 n0y by row (float64)
    const double* rowpart;
};

struct TrefArgs {
    const Inst* insts;
    float* tref;
    const float* tref_new;
    int32_t* dl;
    const int32_t* dl_new;
};

hipError_t launch_step(int prec, const StepArgs& a, int mode, int grid, int tx, int ty, hipStream_t st);
hipError_t launch_finalize(const FinArgs& a, int n_inst, hipStream_t st);
hipError_t launch_counter(long long* c, long long n, hipStream_t st);
hipError_t launch_count_active(const Inst* insts, int n, int* out, hipStream_t st);
hipError_t launch_init(int prec, const InitArgs& a, int max_nodes, int n_inst, hipStream_t st);
hipError_t launch_state(int prec, const StateArgs& a, int nodes, hipStream_t st);
hipError_t launch_tref_copy(const TrefArgs& a, int max_nodes, int n_inst, hipStream_t st);
hipError_t launch_flux_next(const FluxArgs& a, int max_rows, int n_inst, hipStream_t st);
hipError_t launch_flux_copy(const FluxArgs& a, int max_rows, int n_inst, hipStream_t st);
hipError_t launch_dl_flags(const Inst* insts, const int32_t* dl, int32_t* dlz, int max_chunks, int n_inst,
                           hipStream_t st);

}  // namespace lbm
