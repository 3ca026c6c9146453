// lbm_kernels.hip -- device code of the coupled central-moment LBM step for
// gfx950 (arXiv 2210.07501, Secs. 3-4, App. B).
//
// One workgroup owns a TX x TY tile of lattice nodes of one channel.  The
// fused step kernel
//   1. pulls the streamed populations f, g, h of the tile and of a halo ring
//      (2 nodes for phi, 1 node for T and p*), applying the wall schemes of
//      Sec. 5 on the fly, and stages phi, T, p* in LDS;
//   2. fills the ghost rows behind the walls and computes the interface
//      normal on the tile plus a 1-node ring (isotropic gradients);
//   3. per node: curvature, surface-tension gradient, pressure force, the
//      CSF force of Sec. 3, the corrected velocity and pressure of Sec. 4.2,
//      and the three central-moment collisions of Secs. 4.1-4.3;
//   4. writes the 27 post-collision populations at the node (pull scheme:
//      the next step gathers them), coalesced along x.
// The moment maps P, F(u), F(-u), P^-1 of App. B factor into 1-D maps along
// x and y on the D2Q9 tensor lattice; they are applied in that factored form
// and only the central moments that actually relax are formed.
//
// Storage: per channel, populations [ny][3][9][nx] (the 27 values of a
// lattice row are 27 consecutive runs of nx).  In float32 mode the stored
// numbers are deviations from reference equilibria w_a X_ref: for f,
// X_ref = phi0(row) (the cold-start tanh profile) plus a per-node offset, and
// a flux reference on the two vertical directions; p_r for g; a per-node
// temperature reference for h.  The per-node references move at check steps
// when a node has drifted; each stored value is relative to its writer's
// references, which the pulling node adds back.  In float64 mode all
// references are zero and the numbers are the populations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {

__device__ __forceinline__ int wrapx(int i, int nx) {
    return i < 0 ? i + nx : (i >= nx ? i - nx : i);
}
__device__ __forceinline__ int modx(int i, int nx) {
    int r = i % nx;
    return r < 0 ? r + nx : r;
}

// D2Q9: index -> (e_x, e_y), e_x = (0,1,0,-1,0,1,-1,-1,1), e_y = (0,0,1,0,-1,1,1,-1,-1);
// opposite direction; direction with e_y reversed.  Compile-time functions so
// that unrolled loops fold them to constants.
__host__ __device__ constexpr int EX(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0); }
__host__ __device__ constexpr int EY(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0); }
__host__ __device__ constexpr int OPP(int a) { return a == 0 ? 0 : (a <= 4 ? (a <= 2 ? a + 2 : a - 2) : (a <= 6 ? a + 2 : a - 2)); }
__host__ __device__ constexpr int MIRY(int a) { return a == 2 ? 4 : a == 4 ? 2 : a == 5 ? 8 : a == 8 ? 5 : a == 6 ? 7 : a == 7 ? 6 : a; }
// (1-D velocity index 0: 0, 1: +1, 2: -1) pair -> D2Q9 index
__host__ __device__ constexpr int DIR(int cx, int cy) {
    return cx == 0 ? (cy == 0 ? 0 : cy == 1 ? 2 : 4) : cx == 1 ? (cy == 0 ? 1 : cy == 1 ? 5 : 8) : (cy == 0 ? 3 : cy == 1 ? 6 : 7);
}

template <class R> struct W9 {
    static __device__ __forceinline__ R w(int a) {
        return a == 0 ? R(4) / R(9) : (a < 5 ? R(1) / R(9) : R(1) / R(36));
    }
};

// Parameters of one channel converted to the compute type.
template <class R> struct P {
    int nx, ny;
    R W, inv_W, M, w_phi, drho, rho_a, mu_a, dmu, k_a, dk;
    R s0, sT, sTT, Tsig;   // Tsig: T_ref of the surface-tension law
    R T_h, dT, T_c, kx, Fx, Fy, p_r;
    double T_top;         // top-wall temperature, kept in float64 for the wall scheme
    __device__ void load(const Inst& I) {
        nx = I.nx; ny = I.ny;
        W = R(I.W); inv_W = R(1.0 / I.W); M = R(I.M_phi); w_phi = R(I.w_phi);
        rho_a = R(I.rho_a); drho = R(I.rho_b - I.rho_a);
        mu_a = R(I.mu_a); dmu = R(I.mu_b - I.mu_a);
        k_a = R(I.k_a); dk = R(I.k_b - I.k_a);
        s0 = R(I.s0); sT = R(I.sT); sTT = R(I.sTT); Tsig = R(I.T_ref);
        T_h = R(I.T_h); dT = R(I.dT); T_c = R(I.T_c); kx = R(I.kx); T_top = I.T_c;
        Fx = R(I.Fx); Fy = R(I.Fy); p_r = R(I.p_r);
    }
};

// Reciprocal and square root: correctly rounded in float64; in float32 the
// hardware instructions (about 1 ulp), well inside the float32 tolerance.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }

// Element index of population (d, a) at node (i, j) in a channel's [ny][3][9][nx] buffer.
__device__ __forceinline__ size_t pidx(int nx, int ny, int d, int a, int j, int i) {
    (void)ny;
    return (((size_t)j * 27 + (size_t)(d * 9 + a)) * (size_t)nx + (size_t)i);
}

// ---------------------------------------------------------------------------
// Factored moment maps on the D2Q9 tensor lattice.  Index m[3 * mx + my].

// raw moments r[mx][my] = sum_a f_a e_x^mx e_y^my
template <class R> __device__ __forceinline__ void raw_moments(const R* f, R* r) {
    R s[3][3];  // s[cx][my]
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
        R f0 = f[DIR(cx, 0)], fp = f[DIR(cx, 1)], fm = f[DIR(cx, 2)];
        s[cx][0] = f0 + fp + fm;
        s[cx][1] = fp - fm;
        s[cx][2] = fp + fm;
    }
#pragma unroll
    for (int my = 0; my < 3; ++my) {
        r[0 * 3 + my] = s[0][my] + s[1][my] + s[2][my];
        r[1 * 3 + my] = s[1][my] - s[2][my];
        r[2 * 3 + my] = s[1][my] + s[2][my];
    }
}

// raw moments from central moments (F(-u)): (e - u + u)^m binomially
template <class R> __device__ __forceinline__ void central_to_raw(R* c, R ux, R uy) {
#pragma unroll
    for (int mx = 0; mx < 3; ++mx) {
        R c0 = c[mx * 3 + 0], c1 = c[mx * 3 + 1], c2 = c[mx * 3 + 2];
        c[mx * 3 + 1] = c1 + uy * c0;
        c[mx * 3 + 2] = c2 + R(2) * uy * c1 + uy * uy * c0;
    }
#pragma unroll
    for (int my = 0; my < 3; ++my) {
        R c0 = c[0 * 3 + my], c1 = c[1 * 3 + my], c2 = c[2 * 3 + my];
        c[1 * 3 + my] = c1 + ux * c0;
        c[2 * 3 + my] = c2 + R(2) * ux * c1 + ux * ux * c0;
    }
}

// distributions from raw moments (P^-1), 1-D inverse along y then x
template <class R> __device__ __forceinline__ void raw_to_dist(const R* r, R* f) {
    R s[3][3];  // s[cx][my]
#pragma unroll
    for (int my = 0; my < 3; ++my) {
        R r0 = r[0 * 3 + my], r1 = r[1 * 3 + my], r2 = r[2 * 3 + my];
        s[0][my] = r0 - r2;
        s[1][my] = R(0.5) * (r1 + r2);
        s[2][my] = R(0.5) * (r2 - r1);
    }
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
        f[DIR(cx, 0)] = s[cx][0] - s[cx][2];
        f[DIR(cx, 1)] = R(0.5) * (s[cx][1] + s[cx][2]);
        f[DIR(cx, 2)] = R(0.5) * (s[cx][2] - s[cx][1]);
    }
}

// Post-collision populations are read again only by the next step, long
// after this tile: stream them past the caches (non-temporal stores) so that
// the halo rows still needed by neighbouring tiles stay in L2.
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif
template <class S> __device__ __forceinline__ void store_pop(S* p, S v) {
#if LBM_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// ---------------------------------------------------------------------------
// Populations: buffer layout [ny][3][9][nx] per channel -- the 27 values of
// a lattice row are 27 consecutive runs of nx, so the 54 streams of a step
// walk through one region of memory together rather than 27 planes far
// apart (measured 5-7% more bandwidth for the same accesses).  "Plane"
// (d, a) of row 0 starts at base + (d * 9 + a) * nx; the node offset is
// j * 27 nx + i, a 32-bit index (the channel size is limited so that the
// byte offset stays below 4 GiB).
template <class S> struct Pop {
    S* base;
    uint32_t nx;
    __device__ __forceinline__ S* plane(int d, int a) const { return base + (size_t)(d * 9 + a) * nx; }
    __device__ __forceinline__ uint32_t rows(int j) const { return (uint32_t)j * 27u * nx; }
    // value at node offset `off` (rows(j) + i) of population (d, a): a 32-bit
    // byte offset from a workgroup-uniform base
    __device__ __forceinline__ S ld(int d, int a, uint32_t off) const {
        return *(const S*)((const char*)plane(d, a) + (off * (uint32_t)sizeof(S)));
    }
};

// Gather the streamed populations of node (i, j) (0 <= j < ny) from the
// post-collision buffer, with the wall schemes of Sec. 5: g half-way
// bounce-back, h anti-bounce-back to the wall temperature, f specular
// (free-slip).  Returned as deviations relative to the references of node
// (i, j): phi0 of row j, p_r, and Tro, the node's own temperature reference.
// NEED: bit 0 f, bit 1 g, bit 2 h.  tw: bottom-wall temperature by column
// (float64 in both precisions: the wall value of the anti-bounce-back is a
// boundary condition, not a deviation, and is formed before rounding).
template <class S, class R, int NEED>
__device__ __forceinline__ void pull_node(const Pop<S>& src, const double* __restrict__ tw, const P<R>& p, int i,
                                          int j, R Tro, R* f, R* g, R* h) {
    const int nx = p.nx, ny = p.ny;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const bool wall_s = j == 0, wall_n = j == ny - 1;
    const uint32_t RS = 27u * (uint32_t)nx;                 // row stride
    const uint32_t r0 = src.rows(j);
    const uint32_t rs = wall_s ? r0 : r0 - RS;   // clamped at the walls
    const uint32_t rn = wall_n ? r0 : r0 + RS;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int ex = EX(a), ey = EY(a);
        const int is = ex == 0 ? i : (ex > 0 ? im : ip);
        const uint32_t off = (ey == 0 ? r0 : (ey > 0 ? rs : rn)) + (uint32_t)is;
        if (NEED & 1) f[a] = R(src.ld(0, a, off));
        if (NEED & 2) g[a] = R(src.ld(1, a, off));
        if (NEED & 4) h[a] = R(src.ld(2, a, off));
        if (ey != 0) {
            const bool wall = ey > 0 ? wall_s : wall_n;
            if (wall) {
                const uint32_t o0 = r0 + (uint32_t)is, oi = r0 + (uint32_t)i;
                if (NEED & 1) f[a] = R(src.ld(0, MIRY(a), o0));
                if (NEED & 2) g[a] = R(src.ld(1, OPP(a), oi));
                if (NEED & 4) {
                    const double Tw = (ey > 0) ? tw[i] : p.T_top;
                    h[a] = -R(src.ld(2, OPP(a), oi)) + R(2.0 * W9<double>::w(a) * (Tw - (double)Tro));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Block reduction of NV doubles (wavefront shuffles + LDS), fixed order.
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double* v, double* red /* LDS [NT/64][NV] */) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        v[k] = x;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wv * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
            v[k] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused step kernel.
// MODE 0: step; 1: step + residual snapshot; 2: fields only (no step).
// The float32 step kernel is held to 80 VGPRs (six waves per SIMD), which it
// fits without spilling; left alone the compiler takes 86 (five waves), and
// the step runs about 10% slower.  The float64 kernels would spill there.
#ifndef LBM_WAVES_PER_EU
#define LBM_WAVES_PER_EU 0
#endif
template <int TX, int TY, class S, class R, bool DEV, int MODE>
__global__ __launch_bounds__(TX * TY)
#if LBM_WAVES_PER_EU > 0
__attribute__((amdgpu_waves_per_eu(LBM_WAVES_PER_EU)))
#else
__attribute__((amdgpu_waves_per_eu((DEV && MODE == 0) ? 6 : 1)))
#endif
void step_kernel(StepArgs a) {
    constexpr int NT = TX * TY;
    constexpr int LX2 = TX + 4, LY2 = TY + 4;   // phi and T-reference region (halo 2)
    constexpr int LX1 = TX + 2, LY1 = TY + 2;   // T, p*, n region (halo 1)
    constexpr int RING = LX2 * LY2 - TX * TY;

    __shared__ R s_phd[LY2 * LX2];  // phi - phi0(row) - dl DL_Q (the node's own reference; dl = 0 in float64 mode)
    __shared__ R s_Tr[LY2 * LX2];   // temperature reference (float32 mode)
    constexpr int LX3 = TX + 6, LY3 = TY + 6;   // phi-reference offset region (halo 3)
    __shared__ int32_t s_dl[DEV ? LY3 * LX3 : 1];   // phi reference minus phi0(row), units of DL_Q
    __shared__ R s_Tb[LY1 * LX1];   // T - Tr
    __shared__ R s_pb[LY1 * LX1];   // p* - p_r
    __shared__ R s_nx[LY1 * LX1];
    __shared__ R s_dny[LY1 * LX1];  // n_y - n0_y
    __shared__ R s_phi0[LY2];       // storage reference phi0 of rows y0-2 .. y0+TY+1
    __shared__ R s_dR[LY2];         // phi of the streamed reference populations minus phi0, same rows
    __shared__ R s_fq[LY2 + 2];     // flux reference of f (A/2), rows y0-3 .. y0+TY+2
    __shared__ R s_fr[LY2];         // constant part of the stored post-collision y-moment of f
    __shared__ R s_n0y[LY1];        // reference normal of rows y0-1 .. y0+TY
    __shared__ double s_red[(NT / 64) * 8];

    // XCD-aware mapping: consecutive tiles share an XCD (and its L2)
    const int G = gridDim.x, per = G >> 3;
    const int tile = (per > 0) ? ((blockIdx.x & 7) * per + (blockIdx.x >> 3)) : blockIdx.x;
    if (tile >= a.n_tiles) return;
    const int inst = a.tile_inst[tile];
    const Inst& I = a.insts[inst];
    if (MODE != 2 && !I.active) return;
    P<R> p;
    p.load(I);
    const int nx = p.nx, ny = p.ny;
    // tile order within a channel: column strips of strip_w tiles, each
    // strip row-major, so that a run of consecutive tiles (one XCD's share)
    // covers a strip whose halo rows are still in that XCD's L2
    int tcol, trow;
    {
        const int lt = tile - I.tile0;
        const int SW = I.strip_w, full = I.tiles_x / SW, per = SW * I.tiles_y;
        if (lt < full * per) {
            const int s = lt / per, q = lt - s * per;
            trow = q / SW;
            tcol = s * SW + (q - trow * SW);
        } else {
            const int rw = I.tiles_x - full * SW, q = lt - full * per;
            trow = q / rw;
            tcol = full * SW + (q - trow * rw);
        }
    }
    const int x0 = tcol * TX, y0 = trow * TY;

    Pop<S> src{(S*)a.src_v + I.pop_off, (uint32_t)nx};
    const double* __restrict__ tw = (const double*)a.tw_v + I.col_off;
    const int tid = threadIdx.x;
    auto colwrap = [&](int ii) {
        ii = ii < 0 ? ii + nx : ii;
        return ii >= nx ? ((ii - nx < nx) ? ii - nx : modx(ii, nx)) : ii;
    };

    // float32 mode: dz when every phi-reference offset in tile + 3 is zero
    // (chunk flags, refreshed whenever the offsets change); the offsets are
    // then neither read nor summed.  Uniform across the workgroup.
    bool dz = true;
    if (DEV) {
        const int32_t* __restrict__ fl = a.dlz + I.chunk_off;
        const int ncx = (nx + DLZ_CX - 1) / DLZ_CX;
        const int ya = max(y0 - 3, 0) / DLZ_CY, yb = min(y0 + TY + 2, ny - 1) / DLZ_CY;
        auto scan = [&](int xa, int xb) {   // columns xa .. xb, 0 <= xa <= xb < nx
            for (int cy = ya; cy <= yb; ++cy)
                for (int cx = xa / DLZ_CX; cx <= xb / DLZ_CX; ++cx)
                    if (fl[cy * ncx + cx]) dz = false;
        };
        const int xa = x0 - 3, xb = x0 + TX + 2;
        if (TX + 6 >= nx) scan(0, nx - 1);
        else if (xa < 0) { scan(xa + nx, nx - 1); scan(0, xb); }
        else if (xb >= nx) { scan(xa, nx - 1); scan(0, xb - nx); }
        else scan(xa, xb);
    }

    // ---- phase 0: reference rows and temperature references ---------------
    for (int k = tid; k < LY2; k += NT) {
        const int r = I.row_off + min(max(y0 - 2 + k, -2), ny + 1) + 2;
        s_phi0[k] = DEV ? R(((const S*)a.phi0_v)[r]) : R(0);
        s_dR[k] = DEV ? R(((const S*)a.phir_v)[r]) : R(0);
        s_fr[k] = DEV ? R(((const S*)a.fr_v)[r]) : R(0);
    }
    for (int k = tid; k < LY2 + 2; k += NT) {
        const int r = I.row_off + min(max(y0 - 3 + k, -2), ny + 1) + 2;
        s_fq[k] = DEV ? R(((const S*)a.fq_v)[r]) : R(0);
    }
    if (DEV) {
        // per-node references: phi offsets on tile + 3, temperatures on tile + 2
        const int32_t* __restrict__ dlv = a.dl_v + I.node_off;
        const S* __restrict__ tref = (const S*)a.tref_v + I.node_off;
        for (int k = tid; k < LY3 * LX3; k += NT) {
            const int hy = k / LX3 - 3, hx = k % LX3 - 3;
            const int jj = y0 + hy;
            const bool in = jj >= 0 && jj < ny;
            const uint32_t o = in ? (uint32_t)jj * (uint32_t)nx + (uint32_t)colwrap(x0 + hx) : 0u;
            // ghost rows take the offsets of their mirror rows (phi is mirrored
            // at the walls); the pull corrections never read ghost rows
            const int jm = jj < 0 ? -1 - jj : (jj >= ny ? 2 * ny - 1 - jj : jj);
            const uint32_t om = (jm >= 0 && jm < ny) ? (uint32_t)jm * (uint32_t)nx + (uint32_t)colwrap(x0 + hx) : 0u;
            s_dl[k] = (jm >= 0 && jm < ny && !dz) ? dlv[om] : 0;
            if (hy >= -2 && hy <= TY + 1 && hx >= -2 && hx <= TX + 1)
                s_Tr[(hy + 2) * LX2 + hx + 2] = in ? R(tref[o]) : R(0);
        }
    }
    __syncthreads();
    for (int k = tid; k < LY1; k += NT) {
        // reference normal of the x-invariant reference profile (regularised)
        const R g0 = R(0.5) * (s_phi0[k + 2] - s_phi0[k]);
        s_n0y[k] = DEV ? g0 / sqrt(g0 * g0 + R(EPS_N * EPS_N)) : R(0);
    }
    // phi-reference moments of the f populations streamed into node (hx,
    // hy): each is stored relative to w_a (phi0(row) + dl(writer)), so the
    // node adds sum_a w_a e_a^m dl(source) (m = 0, x, y), summed exactly in
    // integers (units of 2^-28).  The source of a wall link is the writer in
    // the node's own row (specular reflection).
    auto fcorr = [&](int hx, int hy, int jj, int& c0, int& cx, int& cy) {
        c0 = 0; cx = 0; cy = 0;
        if (dz) return;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int ex = EX(q), ey = EY(q);
            const bool wall = ey != 0 && (jj - ey < 0 || jj - ey >= ny);
            const int sy = wall ? hy : hy - ey, sx = hx - ex;
            const int m = q == 0 ? 16 : (q < 5 ? 4 : 1);          // 36 w_q
            const int d = m * s_dl[(sy + 3) * LX3 + sx + 3];
            c0 += d;
            if (ex) cx += ex > 0 ? d : -d;
            if (ey) cy += ey > 0 ? d : -d;
        }
    };
    // Temperature-reference moments of the populations streamed into node
    // (hx, hy): each is stored relative to its writer's reference, so the
    // node sees sum_a w_a e_a^m (Tr(source) - Tr(node)) on top of its own.
    auto tcorr = [&](int hx, int hy, int jj, R& c0, R& cx, R& cy) {
        c0 = R(0); cx = R(0); cy = R(0);
        const R t0 = s_Tr[(hy + 2) * LX2 + hx + 2];
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            const int ex = EX(q), ey = EY(q);
            if (ey != 0 && (jj - ey < 0 || jj - ey >= ny)) continue;   // wall link
            const R d = W9<R>::w(q) * (s_Tr[(hy - ey + 2) * LX2 + hx - ex + 2] - t0);
            c0 += d;
            if (ex) cx += ex > 0 ? d : -d;
            if (ey) cy += ey > 0 ? d : -d;
        }
    };

    // float32 mode: phi of a halo node relative to its own reference
    // phi0(row) + dl DL_Q, summed in float64 (the row constants dR and the flux
    // reference are not small, their rounding would vary along x)
    auto ring_phd = [&](const R* tf, int hx, int hy, int jj) -> R {
        int i0, ix, iy;
        fcorr(hx, hy, jj, i0, ix, iy);
        const int dln = dz ? 0 : s_dl[(hy + 3) * LX3 + hx + 3];
        double sd = (double)s_dR[hy + 2] + ((double)s_fq[hy + 2] - (double)s_fq[hy + 4]) + (double)(i0 - 36 * dln) * DL_U;
#pragma unroll
        for (int q = 0; q < 9; ++q) sd += (double)tf[q];
        return (R)sd;
    };

    // ---- phase 1: pull own node and the halo ring ---------------------------
    const int tx = tid % TX, ty = tid / TX;
    const int gi = (x0 + tx < nx) ? x0 + tx : modx(x0 + tx, nx), gj = y0 + ty;
    const bool own_row = gj < ny;
    const bool own_ok = own_row && (x0 + tx < nx);
    R f[9], g[9], h[9];
    R rh[9];
    double rf[9];   // moments of f and g in float64: they feed the float64 f and g collisions
    double rg[9];
    const R Tro = DEV ? s_Tr[(ty + 2) * LX2 + tx + 2] : R(0);   // this node's T reference
    double dph_d = 0.0;   // float32 mode: phi - phi0(row), accumulated in float64
    if (own_row) {
        pull_node<S, R, 7>(src, tw, p, gi, gj, Tro, f, g, h);
        {
            double fd[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) fd[q] = (double)f[q];
            raw_moments(fd, rf);
        }
        {
            double gd[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) gd[q] = (double)g[q];
            raw_moments(gd, rg);
        }
        raw_moments(h, rh);
        if (DEV) {
            R c0, cx, cy;
            tcorr(tx, ty, gj, c0, cx, cy);
            rh[0] += c0;
            rh[3] += cx;
            rh[1] += cy;
            // phi - phi0(row), summed in float64 so that the step conserves
            // sum phi up to the rounding of one small stored value.  rf[1]
            // stays the y-moment of the stored deviations alone: the
            // references' share of it is folded into the fr table.
            int d0, dxm, dym;
            fcorr(tx, ty, gj, d0, dxm, dym);
            rf[3] += (double)dxm * DL_U;
            rf[1] += (double)dym * DL_U;
            dph_d = (double)s_dR[ty + 2] + ((double)s_fq[ty + 2] - (double)s_fq[ty + 4]) + (double)d0 * DL_U;
#pragma unroll
            for (int q = 0; q < 9; ++q) dph_d += (double)f[q];
            rf[0] = dph_d;
        }
        // LDS keeps phi relative to the node's own reference phi0(row) + dl:
        // tiny near a steady state, so the small variations of phi along the
        // interface survive float32; stencils add the references' share from
        // the integer offsets, exactly
        s_phd[(ty + 2) * LX2 + tx + 2] = DEV ? (R)(dph_d - (double)s_dl[(ty + 3) * LX3 + tx + 3] * DL_Q) : rf[0];
        s_pb[(ty + 1) * LX1 + tx + 1] = rg[0];
        s_Tb[(ty + 1) * LX1 + tx + 1] = rh[0];
    }
    // Halo ring.  Float64: work items of one distribution each, so that they
    // spread evenly over the threads: phi of every ring node (depth 1 and 2),
    // then p* and T of the depth-1 ring; items of one kind are contiguous, so
    // a wave mostly takes one branch (1.8% faster than one item per node).
    // Float32 keeps one item per ring node: the split costs it a register
    // spill at its six-waves bound.
    if constexpr (!DEV) {
    constexpr int R1 = LX1 * LY1 - TX * TY;     // depth-1 ring nodes
    for (int it = tid; it < RING + 2 * R1; it += NT) {
        int hx, hy;
        if (it < RING) {   // phi: ring rows above and below, then the side columns
            const int k = it;
            if (k < 2 * LX2) { hy = -2 + k / LX2; hx = -2 + k % LX2; }
            else if (k < 4 * LX2) { int q = k - 2 * LX2; hy = TY + q / LX2; hx = -2 + q % LX2; }
            else { int q = k - 4 * LX2; hy = q / 4; int c = q % 4; hx = c < 2 ? c - 2 : TX + c - 2; }
        } else {           // p* or T of a depth-1 ring node
            const int k = (it - RING) % R1;
            if (k < LX1) { hy = -1; hx = k - 1; }
            else if (k < 2 * LX1) { hy = TY; hx = k - LX1 - 1; }
            else { int q = k - 2 * LX1; hy = q / 2; hx = (q % 2) ? TX : -1; }
        }
        const int jj = y0 + hy;
        if (jj < 0 || jj >= ny) continue;
        const int ii = colwrap(x0 + hx);
        R tf[9], tg[9], th[9];
        if (it < RING) {
            pull_node<S, R, 1>(src, tw, p, ii, jj, R(0), tf, tg, th);
            R s1 = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) s1 += tf[q];
            s_phd[(hy + 2) * LX2 + hx + 2] = s1;
        } else if (it < RING + R1) {
            pull_node<S, R, 2>(src, tw, p, ii, jj, R(0), tf, tg, th);
            R s2 = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) s2 += tg[q];
            s_pb[(hy + 1) * LX1 + hx + 1] = s2;
        } else {
            pull_node<S, R, 4>(src, tw, p, ii, jj, R(0), tf, tg, th);
            R s3 = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) s3 += th[q];
            s_Tb[(hy + 1) * LX1 + hx + 1] = s3;
        }
    }
    } else {
    for (int k = tid; k < RING; k += NT) {
        int hx, hy;
        if (k < 2 * LX2) { hy = -2 + k / LX2; hx = -2 + k % LX2; }
        else if (k < 4 * LX2) { int q = k - 2 * LX2; hy = TY + q / LX2; hx = -2 + q % LX2; }
        else { int q = k - 4 * LX2; hy = q / 4; int c = q % 4; hx = c < 2 ? c - 2 : TX + c - 2; }
        const int jj = y0 + hy;
        if (jj < 0 || jj >= ny) continue;
        const int ii = colwrap(x0 + hx);
        const bool h1 = hx >= -1 && hx <= TX && hy >= -1 && hy <= TY;
        R tf[9], tg[9], th[9];
        if (h1) {
            const R Trr = s_Tr[(hy + 2) * LX2 + hx + 2];
            pull_node<S, R, 7>(src, tw, p, ii, jj, Trr, tf, tg, th);
            R s2 = 0, s3 = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) { s2 += tg[q]; s3 += th[q]; }
            R c0, cx, cy;
            tcorr(hx, hy, jj, c0, cx, cy);
            s3 += c0;
            s_phd[(hy + 2) * LX2 + hx + 2] = ring_phd(tf, hx, hy, jj);
            s_pb[(hy + 1) * LX1 + hx + 1] = s2;
            s_Tb[(hy + 1) * LX1 + hx + 1] = s3;
        } else {
            pull_node<S, R, 1>(src, tw, p, ii, jj, R(0), tf, tg, th);
            s_phd[(hy + 2) * LX2 + hx + 2] = ring_phd(tf, hx, hy, jj);
        }
    }
    }
    __syncthreads();

    // ---- ghost rows: phi, p* mirrored, T = 2 T_w - T ------------------------
    // (only tiles whose LDS rows reach past a wall or past the last row have
    // any; the condition is uniform across the work-group)
    if (y0 < 2 || y0 + TY + 2 > ny) {
    for (int k = tid; k < LY2 * LX2; k += NT) {
        const int hy = k / LX2 - 2, hx = k % LX2 - 2;
        const int jj = y0 + hy;
        if (jj >= 0 && jj < ny) continue;
        const int mj = jj < 0 ? -1 - jj : 2 * ny - 1 - jj;      // mirror row
        const int mhy = mj - y0;
        const bool valid = (jj >= -2 && jj <= ny + 1) && mhy >= -2 && mhy <= TY + 1;
        R v = R(0);
        // phi0 and the offsets are mirrored in the ghost rows too
        if (valid) v = s_phd[(mhy + 2) * LX2 + hx + 2];
        s_phd[k] = v;
        if (hx >= -1 && hx <= TX && hy >= -1 && hy <= TY) {
            R vp = R(0), vT = R(0), vr = R(0);
            if (valid && (jj == -1 || jj == ny)) {
                vp = s_pb[(mhy + 1) * LX1 + hx + 1];
                const R Tm = s_Tb[(mhy + 1) * LX1 + hx + 1];
                vr = DEV ? s_Tr[(mhy + 2) * LX2 + hx + 2] : R(0);   // ghost reference := mirror's
                const double Tw = (jj < 0) ? tw[colwrap(x0 + hx)] : p.T_top;
                // T_ghost = 2 T_w - T_mirror; deviation from vr formed exactly
                vT = R(2.0 * ((double)Tw - (double)vr)) - Tm;
            }
            s_pb[(hy + 1) * LX1 + hx + 1] = vp;
            s_Tb[(hy + 1) * LX1 + hx + 1] = vT;
            if (DEV) s_Tr[k] = vr;
        }
    }
    __syncthreads();
    }

    // Isotropic gradient of phi - phi0(row) at halo position (hx, hy): the
    // stencil of the LDS deviations plus that of the reference offsets,
    // taken in integers (exact) and scaled once.
    auto grad_phi = [&](int hx, int hy, R& gx, R& gy) {
        const R* v = &s_phd[(hy + 2) * LX2 + hx + 2];
        const R E = v[1], Wv = v[-1], N = v[LX2], Sv = v[-LX2];
        const R NE = v[LX2 + 1], NW = v[LX2 - 1], SE = v[-LX2 + 1], SW = v[-LX2 - 1];
        gx = (E - Wv) * (R(1) / R(3)) + (NE - NW + SE - SW) * (R(1) / R(12));
        gy = (N - Sv) * (R(1) / R(3)) + (NE + NW - SE - SW) * (R(1) / R(12));
        if (DEV && !dz) {
            const int32_t* d = &s_dl[(hy + 3) * LX3 + hx + 3];
            const int sx = 4 * (d[1] - d[-1]) + (d[LX3 + 1] - d[LX3 - 1] + d[-LX3 + 1] - d[-LX3 - 1]);
            const int sy = 4 * (d[LX3] - d[-LX3]) + (d[LX3 + 1] + d[LX3 - 1] - d[-LX3 + 1] - d[-LX3 - 1]);
            gx += R(sx) * R(DL_Q / 12.0);
            gy += R(sy) * R(DL_Q / 12.0);
        }
    };

    // ---- phase 2: interface normal on the tile + 1 ring ----------------------
    // n = grad phi / sqrt(|grad phi|^2 + eps^2); stored as n_x and the
    // deviation n_y - n0_y from the reference normal.  With G = G0 + g (g the
    // deviation part), D^2 = |G|^2 + eps^2 and D0^2 = G0_y^2 + eps^2:
    //   float64 arithmetic (with a reference profile):
    //             D0 - D = (-g_y (G_y + G0_y) - G_x^2) / (D0 + D),
    //             n_y - n0_y = (G0_y (D0 - D) + g_y D0) / (D D0);
    //   float32:  n_y^2 - n0_y^2 = (eps^2 g_y (G_y + G0_y) - G0_y^2 G_x^2) / (D^2 D0^2),
    //             n_y - n0_y = (n_y^2 - n0_y^2) / (n_y + n0_y).
    // The float32 form has no cancellation at all: near a flat interface
    // n_y - n0_y is second order in G_x, while the two terms of the float64
    // form are first order in g_y and cancel, so in float32 their rounding
    // (relative to g_y, not to the result) dominated the curvature of
    // weakly driven channels.  Where n_y and n0_y differ in sign (only far
    // from the interface, |G| ~ eps) the direct difference is used.
    for (int k = tid; k < LY1 * LX1; k += NT) {
        const int hy = k / LX1 - 1, hx = k % LX1 - 1;
        const int jj = y0 + hy;
        R nxv = R(0), dny = R(0);
        if (jj >= -1 && jj <= ny) {
            R Gx, gy;
            grad_phi(hx, hy, Gx, gy);
            const R G0y = R(0.5) * (s_phi0[hy + 3] - s_phi0[hy + 1]);
            const R Gy = gy + G0y;
            const R eps2 = R(EPS_N * EPS_N);
            const R D2 = Gx * Gx + Gy * Gy + eps2, D02 = G0y * G0y + eps2;
            if (!DEV) {
                // float64: no reference profile (G0 = 0, n0 = 0), n = G / D
                const R rD = R(1) / sqrt(D2);
                nxv = Gx * rD;
                dny = Gy * rD;
            } else if (sizeof(R) == 8) {
                const R D = sqrt(D2), D0 = sqrt(D02);
                const R dD = (-gy * (Gy + G0y) - Gx * Gx) / (D0 + D);
                nxv = Gx / D;
                dny = (G0y * dD + gy * D0) / (D * D0);
            } else {
                const R rD = rsqrt_(D2), rD0 = rsqrt_(D02);
                const R ny1 = Gy * rD, ny0 = G0y * rD0;
                const R num = eps2 * gy * (Gy + G0y) - (G0y * G0y) * (Gx * Gx);
                nxv = Gx * rD;
                dny = (ny1 * ny0 > R(0)) ? num * rcp((D2 * D02) * (ny1 + ny0)) : ny1 - ny0;
            }
        }
        s_nx[k] = nxv;
        s_dny[k] = dny;
    }
    __syncthreads();

    // ---- phase 3: forces, velocity, collisions -------------------------------
    double red[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double flux_dev = 0.0;   // float32 check steps: this node's stored f flux deviation t01 - A
    if (own_row) {
        const R cs2 = R(1) / R(3);
        const int c2 = (ty + 2) * LX2 + tx + 2, c1 = (ty + 1) * LX1 + tx + 1;
        // isotropic gradient helper on an LDS array with row stride L
        auto grad = [&](const R* arr, int c, int L, R& gx, R& gy) {
            const R E = arr[c + 1], Wv = arr[c - 1], N = arr[c + L], Sv = arr[c - L];
            const R NE = arr[c + L + 1], NW = arr[c + L - 1], SE = arr[c - L + 1], SW = arr[c - L - 1];
            gx = (E - Wv) * (R(1) / R(3)) + (NE - NW + SE - SW) * (R(1) / R(12));
            gy = (N - Sv) * (R(1) / R(3)) + (NE + NW - SE - SW) * (R(1) / R(12));
        };
        R Gx, Gy;
        grad_phi(tx, ty, Gx, Gy);
        Gy += R(0.5) * (s_phi0[ty + 3] - s_phi0[ty + 1]);
        const R g2 = Gx * Gx + Gy * Gy;
        const R nxv = s_nx[c1];
        const R nyv = s_n0y[ty + 1] + s_dny[c1];
        R dnx_dx, dnx_dy, ddy_dx, ddy_dy;
        grad(s_nx, c1, LX1, dnx_dx, dnx_dy);
        grad(s_dny, c1, LX1, ddy_dx, ddy_dy);
        const R curv = dnx_dx + ddy_dy + R(0.5) * (s_n0y[ty + 2] - s_n0y[ty]);
        // surface tension (Eq. ST_SRF) and its isotropic gradient.  Each
        // stencil difference sigma(T1) - sigma(T2) is formed as
        // (T1 - T2) (s_T + s_TT (d1 + d2)), d = T - T_ref, with T1 - T2 taken
        // as (reference difference) + (deviation difference): exact up to
        // the rounding of the small deviations.
        // the temperature reference is zero in float64 mode (s_Tr unused)
        auto Tr_at = [&](int dx, int dy) { return DEV ? s_Tr[c2 + dy * LX2 + dx] : R(0); };
        auto Tb_at = [&](int dx, int dy) { return s_Tb[c1 + dy * LX1 + dx]; };
        auto dref = [&](int dx, int dy) { return (Tr_at(dx, dy) - p.Tsig) + Tb_at(dx, dy); };
        auto dsig = [&](int x1, int y1, int x2, int y2) {
            const R dT12 = (Tr_at(x1, y1) - Tr_at(x2, y2)) + (Tb_at(x1, y1) - Tb_at(x2, y2));
            return dT12 * (p.sT + p.sTT * (dref(x1, y1) + dref(x2, y2)));
        };
        const R dsx = dsig(1, 0, -1, 0) * (R(1) / R(3)) +
                      (dsig(1, 1, -1, 1) + dsig(1, -1, -1, -1)) * (R(1) / R(12));
        const R dsy = dsig(0, 1, 0, -1) * (R(1) / R(3)) +
                      (dsig(1, 1, 1, -1) + dsig(-1, 1, -1, -1)) * (R(1) / R(12));
        const R d0 = dref(0, 0);
        const R sig = p.s0 + (p.sT + p.sTT * d0) * d0;
        R dpx, dpy;
        grad(s_pb, c1, LX1, dpx, dpy);
        // CSF force (Sec. 3): 1.5 W |grad phi|^2 [ -sigma kappa n + (I - n n) grad sigma ]
        const R dl = R(1.5) * p.W * g2;
        const R Fsx = dl * (-sig * curv * nxv + (R(1) - nxv * nxv) * dsx - nxv * nyv * dsy);
        const R Fsy = dl * (-sig * curv * nyv + (R(1) - nyv * nyv) * dsy - nxv * nyv * dsx);
        const R Ftx = Fsx + p.Fx, Fty = Fsy + p.Fy;
        // pressure force F_p = -grad(p* - rho c_s^2), rho linear in phi
        const R Fpx = -dpx + cs2 * p.drho * Gx;
        const R Fpy = -dpy + cs2 * p.drho * Gy;
        // macroscopic update (Sec. 4.2).  rho is formed in float64 from phi
        // in float64: it enters p - rho c_s^2 of the g equilibrium, whose
        // float32 rounding would otherwise be re-applied to the momentum at
        // every step (float32 mode; in float64 mode these are the same values)
        const R phb = rf[0];
        const R phi = s_phi0[ty + 2] + phb;
        const double phi_d = DEV ? (double)s_phi0[ty + 2] + dph_d : (double)phi;
        const double rho_d = (double)p.rho_a + phi_d * (double)p.drho;
        const R rho = (R)rho_d;
        const R rrho = rcp(rho);
        // u in float64 as well: the g collision turns it back into momentum,
        // so a rounded 1/rho would bias the momentum at every step where
        // rho != 1
        const double rrho_d = 1.0 / rho_d;
        const double ux_d = ((double)rg[3] + 0.5 * (1.0 / 3.0) * (double)Ftx) * (3.0 * rrho_d);
        const double uy_d = ((double)rg[1] + 0.5 * (1.0 / 3.0) * (double)Fty) * (3.0 * rrho_d);
        const R ux = (R)ux_d, uy = (R)uy_d;
        const R Gam = Fpx * ux + Fpy * uy;
        const R pb = rg[0] + R(0.5) * Gam;          // p - p_r
        R Tb = rh[0];                                // T - Tro

        if (MODE == 2) {
            if (own_ok) {
                const size_t q = (size_t)I.node_off + (size_t)gj * nx + gi;
                a.out[0][q] = phi_d;
                a.out[1][q] = (double)ux;
                a.out[2][q] = (double)uy;
                a.out[3][q] = (double)Tro + (double)Tb;
                a.out[4][q] = (double)p.p_r + (double)pb;
            }
        } else {
            R Tr = Tro;
            if (MODE == 1) {
                if (own_ok) {
                    const size_t q = (size_t)I.node_off + (size_t)gj * nx + gi;
                    const double dux = (double)ux, duy = (double)uy;
                    const double Tfull = (double)Tro + (double)Tb;
                    const double dT = ((double)Tro - I.T_ref) + (double)Tb;   // T - T_ref
                    const double o_ux = a.snap[0][q], o_uy = a.snap[1][q], o_T = a.snap[2][q];
                    red[0] = (dux - o_ux) * (dux - o_ux) + (duy - o_uy) * (duy - o_uy);
                    red[1] = dux * dux + duy * duy;
                    red[2] = (Tfull - o_T) * (Tfull - o_T);
                    red[3] = dT * dT;
                    red[4] = phi_d;
                    red[5] = rho_d;
                    const bool bad = !(isfinite(dux) && isfinite(duy) && isfinite(Tfull) &&
                                       isfinite(phi_d) && isfinite((double)pb));
                    red[6] = bad ? 1.0 : 0.0;
                    a.snap[0][q] = dux;
                    a.snap[1][q] = duy;
                    a.snap[2][q] = Tfull;
                    a.snap[3][q] = phi_d;
                }
                if (DEV) {
                    // move this node's temperature reference to its current
                    // temperature when it has drifted by more than 1e-6: the
                    // values written below are stored relative to it (the
                    // next steps read the new references).  Near steady state
                    // the references stay put, so the float32 iteration can
                    // settle instead of being re-rounded at every check.
                    const R Tn = (Tb > R(1e-6) || Tb < R(-1e-6)) ? Tro + Tb : Tro;
                    Tb = Tb - (Tn - Tro);
                    Tr = Tn;
                    if (own_ok) ((S*)a.tref_out)[(size_t)I.node_off + (size_t)gj * nx + gi] = S(Tn);
                }
            }
            // local relaxation rates
            const R mu = p.mu_a + phi * p.dmu, kc = p.k_a + phi * p.dk;
            const R w_nu = rcp(R(3) * (mu * rrho) + R(0.5));
            const R w_T = rcp(R(3) * (kc * rrho) + R(0.5));
            const R ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;

            // --- ACE (Sec. 4.1): relax first central moments to M theta n ---
            // stored as f - w phi0(row of this node) - q (flux reference,
            // float32 mode).  Computed in float64 in both precisions: in
            // float32 the rounding of the collision's phi-sized terms put a
            // steady bias into the interface flux of weakly driven channels.
            {
                using D = double;
                const D uxd = ux_d, uyd = uy_d, phd = phi_d;
                const D ux2d = uxd * uxd, uy2d = uyd * uyd, uxyd = uxd * uyd, cs2d = 1.0 / 3.0;
                const D ph0 = (D)s_phi0[ty + 2];
                const D dph = DEV ? dph_d : (D)phb;               // phi - phi0(row)
                // this node's storage reference phr = phi0(row) + dl (float32
                // mode); a check step moves it to the current phi when the node
                // has drifted by more than 1e-6, so that near steady state the
                // stored values stay small
                D phr = ph0, dphr = dph;
                if (DEV) {
                    int32_t kdl = s_dl[(ty + 3) * LX3 + tx + 3];
                    if (MODE == 1) {
                        const double dd = dph_d - (double)kdl * DL_Q;
                        if (dd > 1e-6 || dd < -1e-6) kdl = (int32_t)llrint(dph_d / DL_Q);
                        if (own_ok) a.dl_out[(size_t)I.node_off + (size_t)gj * nx + gi] = kdl;
                    }
                    const double dlo = (double)kdl * DL_Q;
                    phr = ph0 + dlo;
                    dphr = dph_d - dlo;
                }
                const D wphi = (D)p.w_phi, Mphi = (D)p.M, iW = (D)p.inv_W;
                const D k10 = rf[3] - uxd * phd;
                const D theta = 4.0 * phd * (1.0 - phd) * iW;
                D t01;
                if (DEV) {
                    // deviation form: with k01 = kref + dk (kref the pulled
                    // references' share) and theta n = theta0 n0y + d,
                    //   t01 - A = (1 - w) dk + w M d + fr(row)
                    const D dk01 = rf[1] - uyd * phd;
                    const D th0 = 4.0 * ph0 * (1.0 - ph0) * iW;
                    const D dth = 4.0 * dph * (1.0 - phd - ph0) * iW;   // theta - theta0
                    const D dtn = dth * (D)nyv + th0 * (D)s_dny[c1];     // theta n_y - theta0 n0y
                    t01 = dk01 + wphi * (Mphi * dtn - dk01) + (D)s_fr[ty + 2];
                    if (MODE == 1 && own_ok) flux_dev = t01;
                } else {
                    const D k01 = rf[1] - uyd * phd;
                    t01 = k01 + wphi * (Mphi * theta * (D)nyv - k01);
                }
                const D t10 = k10 + wphi * (Mphi * theta * (D)nxv - k10);
                // post-collision central moments minus phr * (rest central moments)
                D c[9];
                c[0] = dphr;                                    // 00
                c[1] = t01 + phr * uyd;                         // 01
                c[2] = dphr * cs2d - phr * uy2d;                // 02
                c[3] = t10 + phr * uxd;                         // 10
                c[4] = -phr * uxyd;                             // 11
                c[5] = phr * uxd * (cs2d + uy2d);               // 12
                c[6] = dphr * cs2d - phr * ux2d;                // 20
                c[7] = phr * uyd * (cs2d + ux2d);               // 21
                c[8] = dphr * (cs2d * cs2d) - phr * (cs2d * (ux2d + uy2d) + ux2d * uy2d);  // 22
                if (DEV) {
                    // minus the other central moments of q (raw: m01 = A only),
                    // the flux reference this step stores against
                    const D A = 2.0 * (D)((const S*)a.fqw_v)[I.row_off + gj + 2];
                    c[2] += 2.0 * A * uyd;
                    c[4] += A * uxd;
                    c[5] -= 2.0 * A * uxyd;
                    c[7] -= A * ux2d;
                    c[8] += 2.0 * A * ux2d * uyd;
                }
                central_to_raw(c, uxd, uyd);
                D fo[9];
                raw_to_dist(c, fo);
#pragma unroll
                for (int q = 0; q < 9; ++q) f[q] = (R)fo[q];
                if (DEV) {
                    // the rest population takes the rounding of the other
                    // eight: the stored values sum to phi - phr in float64
                    double s8 = 0.0;
#pragma unroll
                    for (int q = 1; q < 9; ++q) s8 += (double)f[q];
                    f[0] = (R)(dphr - s8);
                }
            }
            // --- energy (Sec. 4.3), stored as h - w Tr(this node) ---
            {
                const R T = Tro + rh[0];
                const R c10 = rh[3] - ux * T, c01 = rh[1] - uy * T;
                R c[9];
                c[0] = Tb;
                c[1] = c01 * (R(1) - w_T) + Tr * uy;
                c[2] = Tb * cs2 - Tr * uy2;
                c[3] = c10 * (R(1) - w_T) + Tr * ux;
                c[4] = -Tr * uxy;
                c[5] = Tr * ux * (cs2 + uy2);
                c[6] = Tb * cs2 - Tr * ux2;
                c[7] = Tr * uy * (cs2 + ux2);
                c[8] = Tb * (cs2 * cs2) - Tr * (cs2 * (ux2 + uy2) + ux2 * uy2);
                central_to_raw(c, ux, uy);
                raw_to_dist(c, h);
            }
            // --- hydrodynamics (Sec. 4.2), stored as g - w p_r ---
            // computed in float64 in both precisions: in float32 its rounding,
            // relative to the O(1) pressure terms, dominates the velocity error
            {
                using D = double;
                const D cs2d = 1.0 / 3.0;
                const D uxd = ux_d, uyd = uy_d, wn = w_nu;
                const D ux2 = uxd * uxd, uy2 = uyd * uyd, uxy = uxd * uyd;
                const D Fpxd = Fpx, Fpyd = Fpy;
                const D Gd = Fpxd * uxd + Fpyd * uyd;     // Gamma = F_p . u
                const D pbd = (D)rg[0] + 0.5 * Gd;         // p - p_r
                const D pr = (D)p.p_r;
                const D vphi = pbd + (pr - rho_d * cs2d);   // p - rho c_s^2
                const D P0 = (D)rg[0] + pr;                 // sum g (full)
                const D r1 = rg[1], r2 = rg[2], r3 = rg[3], r4 = rg[4], r6 = rg[6];
                // pre-collision central moments that relax at omega_nu
                const D e2d = (r6 - r2) - 2.0 * uxd * r3 + 2.0 * uyd * r1 + (ux2 - uy2) * P0;
                const D e11 = r4 - uyd * r3 - uxd * r1 + uxy * P0;
                // sources (Sec. 4.2)
                const D s10 = cs2d * (D)Ftx - uxd * Gd, s01 = cs2d * (D)Fty - uyd * Gd;
                const D s20 = 2.0 * cs2d * Fpxd * uxd + (ux2 + cs2d) * Gd;
                const D s02 = 2.0 * cs2d * Fpyd * uyd + (uy2 + cs2d) * Gd;
                const D s11 = cs2d * (Fpxd * uyd + Fpyd * uxd) + uxy * Gd;
                const D q2d = vphi * (ux2 - uy2), q11 = vphi * uxy;
                const D t2d = e2d + wn * (q2d - e2d) + (1.0 - 0.5 * wn) * (s20 - s02);
                const D t11 = e11 + wn * (q11 - e11) + (1.0 - 0.5 * wn) * s11;
                // trace: 2 p c_s^2 + vphi u^2 + s_2s / 2, minus p_r (2 c_s^2 + u^2)
                const D t2s_dev = 2.0 * cs2d * pbd + (vphi - pr) * (ux2 + uy2) + 0.5 * (s20 + s02);
                const D t2d_dev = t2d - pr * (ux2 - uy2);
                const D pv = pr - vphi;                    // p_r - (p - rho c_s^2)
                D c[9];
                c[0] = pbd + 0.5 * Gd;                              // 00
                c[1] = pv * uyd + 0.5 * s01;                        // 01
                c[2] = 0.5 * (t2s_dev - t2d_dev);                   // 02
                c[3] = pv * uxd + 0.5 * s10;                        // 10
                c[4] = t11 - pr * uxy;                              // 11
                c[5] = pv * (uy2 + cs2d) * uxd;                     // 12
                c[6] = 0.5 * (t2s_dev + t2d_dev);                   // 20
                c[7] = pv * (ux2 + cs2d) * uyd;                     // 21
                c[8] = pbd * (cs2d * cs2d) + (pbd - rho_d * cs2d) * (cs2d * (ux2 + uy2) + ux2 * uy2);  // 22
                central_to_raw(c, uxd, uyd);
                D go[9];
                raw_to_dist(c, go);
#pragma unroll
                for (int q = 0; q < 9; ++q) g[q] = (R)go[q];
            }
            if (own_ok) {
                Pop<S> dst{(S*)a.dst_v + I.pop_off, (uint32_t)nx};
                const uint32_t bo = (dst.rows(gj) + (uint32_t)gi) * (uint32_t)sizeof(S);
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    store_pop((S*)((char*)dst.plane(0, q) + bo), S(f[q]));
                    store_pop((S*)((char*)dst.plane(1, q) + bo), S(g[q]));
                    store_pop((S*)((char*)dst.plane(2, q) + bo), S(h[q]));
                }
            }
        }
    }
    if (MODE == 1 && DEV) {
        // row sums of the stored flux deviation over this tile, in a fixed
        // order (segments of TX lanes, then the segments of a row), for the
        // flux reference that follows the actual flux
        constexpr int SEG = TX < 64 ? TX : 64;
        constexpr int NSEG = TX / SEG;
        __shared__ double s_rs[TY * NSEG];
        double v = flux_dev;
#pragma unroll
        for (int o = SEG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (tid % SEG == 0) s_rs[tid / SEG] = v;
        __syncthreads();
        if (tid < TY && y0 + tid < ny) {
            double r = 0.0;
#pragma unroll
            for (int k = 0; k < NSEG; ++k) r += s_rs[tid * NSEG + k];
            a.rowpart[I.rp_off + (size_t)(y0 + tid) * I.rp_stride + tcol] = r;
        }
    }
    if (MODE == 1) {
        block_sum<NT, 8>(red, s_red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a.partials[(size_t)tile * 8 + k] = red[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Per-instance check, in two passes so that a large channel is not reduced
// by one block.  First pass: block b of an instance sums the block partials
// of its tiles CHK_TILES b .. CHK_TILES (b + 1) - 1 (one tile per thread,
// fixed order) and takes the interface-velocity peak on the phi = 1/2 level
// over its share of the columns.  The split depends only on the instance's
// own tile count, so a channel checks the same in any batch.
__device__ __forceinline__ double interface_u(const double* ux, const double* ph, int nx, int ny, int jstart, int i) {
    for (int d = 0; d < ny; ++d) {
        for (int sgn = 0; sgn < 2; ++sgn) {
            const int j = sgn ? jstart - d : jstart + d;
            if ((sgn && d == 0) || j < 0 || j > ny - 2) continue;
            const double c0 = ph[(size_t)j * nx + i] - 0.5, c1 = ph[(size_t)(j + 1) * nx + i] - 0.5;
            if (c0 >= 0.0 && c1 < 0.0) {
                const double t = c0 / (c0 - c1);
                return (1.0 - t) * ux[(size_t)j * nx + i] + t * ux[(size_t)(j + 1) * nx + i];
            }
        }
    }
    return 0.0;
}

__device__ __forceinline__ double block_max(double x, double* s4 /* LDS [4] */) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = x;
    __syncthreads();
    return fmax(fmax(s4[0], s4[1]), fmax(s4[2], s4[3]));
}

__global__ __launch_bounds__(256) void check_sums_kernel(FinArgs a) {
    __shared__ double s_red[4 * 8];
    __shared__ double s_pk[4];
    const int inst = blockIdx.y, b = blockIdx.x;
    const Inst& I = a.insts[inst];
    if (!I.active) return;
    const int nb = (I.ntiles + CHK_TILES - 1) / CHK_TILES;
    if (b >= nb) return;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int t = b * CHK_TILES + (int)threadIdx.x;
    if (t < I.ntiles) {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = a.partials[(size_t)(I.tile0 + t) * 8 + k];
    }
    block_sum<256, 8>(v, s_red);
    // interface peak from the snapshot (ux at index 0, phi at index 3)
    const int nx = I.nx, ny = I.ny;
    const double* ux = a.snap[0] + I.node_off;
    const double* ph = a.snap[3] + I.node_off;
    int jstart = (int)I.b - 1;
    jstart = jstart < 0 ? 0 : (jstart > ny - 2 ? ny - 2 : jstart);
    const int cpb = (nx + nb - 1) / nb, i0 = b * cpb, i1 = min(nx, i0 + cpb);
    double peak = 0.0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += 256) peak = fmax(peak, fabs(interface_u(ux, ph, nx, ny, jstart, i)));
    peak = block_max(peak, s_pk);
    if (threadIdx.x == 0) {
        double* o = a.chk + ((size_t)inst * a.chk_nb + b) * 9;
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = v[k];
        o[8] = peak;
    }
}

// Second pass, one block per instance: the first pass's block sums in a
// fixed order, residual, sums, interface peak, retirement.
__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
    __shared__ double s_red[4 * 8];
    __shared__ double s_pk[4];
    const int inst = blockIdx.x;
    Inst& I = a.insts[inst];
    Result& res = a.results[inst];
    if (!I.active) return;
    const int nb = (I.ntiles + CHK_TILES - 1) / CHK_TILES;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double peak = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        const double* o = a.chk + ((size_t)inst * a.chk_nb + b) * 9;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] += o[k];
        peak = fmax(peak, o[8]);
    }
    block_sum<256, 8>(v, s_red);
    peak = block_max(peak, s_pk);
    if (threadIdx.x == 0) {
        const double K = (double)CHECK_EVERY;
        double r = INFINITY;
        if (res.have_prev) {
            const double ru = v[1] > 0 ? sqrt(v[0]) / sqrt(v[1]) : (v[0] == 0 ? 0.0 : INFINITY);
            const double rT = v[3] > 0 ? sqrt(v[2]) / sqrt(v[3]) : (v[2] == 0 ? 0.0 : INFINITY);
            r = fmax(ru, rT) / K;
        }
        res.r = r;
        res.sum_phi = v[4];
        res.sum_rho = v[5];
        res.u_peak = peak;
        res.bad = v[6];
        res.have_prev = 1;
        res.check_step = *a.step_counter;
        const double tol = *a.tol;
        if (v[6] > 0.0) {
            I.active = 0;
            res.retired_at = *a.step_counter + 1;
        } else if (tol > 0.0 && r <= tol) {
            I.active = 0;
            res.retired_at = *a.step_counter + 1;
        }
    }
}

// advance the device step counter by n (one thread)
__global__ void counter_kernel(long long* c, long long n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c += n;
}

__global__ void count_active_kernel(const Inst* insts, int n, int* out) {
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    int c = 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) c += insts[k].active ? 1 : 0;
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Storage convention (float32 mode).  The value a node writes for direction
// k is stored relative to that writer's own references: w_k phi0(row) + q_k
// (the flux reference, +-fq(row) on the two vertical directions), w_k p_r,
// w_k Tr(writer).  The node that pulls it (the neighbour at +e_k, or
// the writer itself through a wall link) adds them back.  In float64 mode all
// references are zero.

// Temperature of node (i, j) from the init fields (cold start or given).
__device__ __forceinline__ double init_T_src(const InitArgs& a, const Inst& I, int i, int j, const double* tw) {
    if (a.cold) {
        const double Tb = (double)tw[i];
        return Tb + (I.T_c - Tb) * ((double)j + 0.5) / (double)I.ny;
    }
    return a.fields[3][(size_t)(I.node_off - a.field_base) + (size_t)j * I.nx + i];
}

// Equilibrium state from fields, written into the post-collision buffer so
// that the next gather yields it (inverse of the gather, walls included).
template <class S, class R, bool DEV>
__global__ __launch_bounds__(256) void init_kernel(InitArgs a) {
    const int inst = blockIdx.y;
    const Inst& I = a.insts[inst];
    const int nx = I.nx, ny = I.ny;
    const long long n = (long long)nx * ny;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % nx), j = (int)(q / nx);
    const double cs2 = 1.0 / 3.0;
    // wall temperatures as the step kernel sees them
    const double* twr = (const double*)a.tw_v + I.col_off;
    auto tw_at = [&](int ii) { return (double)twr[ii]; };
    double phi, ux, uy;
    if (a.cold) {
        // fluid at rest, tanh interface at y = b - 1/2, T linear between walls
        phi = 0.5 * (1.0 + tanh(2.0 * ((I.b - 0.5) - (double)j) / I.W));
        ux = 0.0;
        uy = 0.0;
    } else {
        const size_t o = (size_t)(I.node_off - a.field_base) + (size_t)q;
        phi = a.fields[0][o];
        ux = a.fields[1][o];
        uy = a.fields[2][o];
    }
    double T;
    if (a.cold) {
        const double Tb = tw_at(i);
        T = Tb + (I.T_c - Tb) * ((double)j + 0.5) / (double)ny;
    } else {
        T = a.fields[3][(size_t)(I.node_off - a.field_base) + (size_t)q];
    }
    const double rho = I.rho_a + phi * (I.rho_b - I.rho_a);
    const double p0 = 1.0 / 3.0;
    const double vphi = p0 - rho * cs2;
    const double ux2 = ux * ux, uy2 = uy * uy;
    // absolute equilibria from their central moments (order [mx*3+my])
    double cf[9], cg[9], ch[9];
    for (int k = 0; k < 9; ++k) { cf[k] = 0; cg[k] = 0; ch[k] = 0; }
    cf[0] = phi; cf[2] = cs2 * phi; cf[6] = cs2 * phi; cf[8] = cs2 * cs2 * phi;
    ch[0] = T; ch[2] = cs2 * T; ch[6] = cs2 * T; ch[8] = cs2 * cs2 * T;
    cg[0] = p0; cg[3] = -vphi * ux; cg[1] = -vphi * uy;
    cg[6] = p0 * cs2 + vphi * ux2; cg[2] = p0 * cs2 + vphi * uy2; cg[4] = vphi * ux * uy;
    cg[7] = -vphi * (ux2 + cs2) * uy; cg[5] = -vphi * (uy2 + cs2) * ux;
    cg[8] = cs2 * cs2 * cs2 * rho + vphi * (ux2 + cs2) * (uy2 + cs2);
    double ef[9], eg[9], eh[9];
    central_to_raw(cf, ux, uy); raw_to_dist(cf, ef);
    central_to_raw(cg, ux, uy); raw_to_dist(cg, eg);
    central_to_raw(ch, ux, uy); raw_to_dist(ch, eh);
    const S* phi0 = (const S*)a.phi0_v + I.row_off + 2;
    const S* fq = (const S*)a.fq_v + I.row_off + 2;
    // phi-reference offset of the writer at (ii, jj): phi there minus phi0(row),
    // rounded as the step kernel stores it (float32 mode)
    auto kdl_at = [&](int ii, int jj) -> int32_t {
        if (!DEV) return 0;
        double ph;
        if (a.cold) ph = 0.5 * (1.0 + tanh(2.0 * ((I.b - 0.5) - (double)jj) / I.W));
        else ph = a.fields[0][(size_t)(I.node_off - a.field_base) + (size_t)jj * I.nx + ii];
        return (int32_t)llrint((ph - (double)phi0[jj]) / DL_Q);
    };
    auto dl_at = [&](int ii, int jj) { return (double)kdl_at(ii, jj) * DL_Q; };
    if (DEV) a.dl[I.node_off + q] = kdl_at(i, j);
    // flux reference of direction k written at row r (float32 mode)
    auto qf = [&](int kk, int r) { return (DEV && EX(kk) == 0 && EY(kk) != 0) ? EY(kk) * (double)fq[r] : 0.0; };
    const double pr = DEV ? I.p_r : 0.0;
    if (DEV) a.tref[I.node_off + q] = (float)T;
    const double Tr_self = DEV ? (double)(float)T : 0.0;
    S* dst = (S*)a.dst_v + I.pop_off;
    // inverse gather: the value that node (i, j) will pull for direction k,
    // relative to the references of its writer
    for (int k = 0; k < 9; ++k) {
        const int ex = EX(k), ey = EY(k);
        const int js = j - ey;
        const int is = wrapx(i - ex, nx);
        const double w = W9<double>::w(k);
        if (js >= 0 && js < ny) {
            const double ph_w = DEV ? (double)phi0[js] : 0.0;
            const double T_w = DEV ? (double)(float)init_T_src(a, I, is, js, twr) : 0.0;
            dst[pidx(nx, ny, 0, k, js, is)] = S(ef[k] - w * (ph_w + dl_at(is, js)) - qf(k, js));
            dst[pidx(nx, ny, 1, k, js, is)] = S(eg[k] - w * pr);
            dst[pidx(nx, ny, 2, k, js, is)] = S(eh[k] - w * T_w);
        } else {
            const int mir = MIRY(k), opp = OPP(k);
            const double Tw = (ey > 0) ? tw_at(i) : I.T_c;
            const double ph_w = DEV ? (double)phi0[j] : 0.0;
            dst[pidx(nx, ny, 0, mir, j, is)] = S(ef[k] - w * (ph_w + dl_at(is, j)) - qf(mir, j));
            dst[pidx(nx, ny, 1, opp, j, i)] = S(eg[k] - w * pr);
            // anti-bounce-back: h_k = -(stored + w Tr_self) + 2 w T_w
            dst[pidx(nx, ny, 2, opp, j, i)] = S(2.0 * w * Tw - w * Tr_self - eh[k]);
        }
    }
}

// Populations (absolute, float64) of one instance <-> post-collision buffer.
// dir 0: buffer -> state (gather), dir 1: state -> buffer (inverse gather).
template <class S, bool DEV>
__global__ __launch_bounds__(256) void state_kernel(StateArgs a) {
    const Inst& I = a.insts[a.inst];
    const int nx = I.nx, ny = I.ny;
    const long long n = (long long)nx * ny;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % nx), j = (int)(q / nx);
    const S* phi0 = (const S*)a.phi0_v + I.row_off + 2;
    const S* fq = (const S*)a.fq_v + I.row_off + 2;
    auto qf = [&](int kk, int r) { return (DEV && EX(kk) == 0 && EY(kk) != 0) ? EY(kk) * (double)fq[r] : 0.0; };
    const double* tw = (const double*)a.tw_v + I.col_off;
    const float* tref = a.tref ? a.tref + I.node_off : nullptr;
    const double pr = DEV ? I.p_r : 0.0;
    const double Tr_self = DEV ? (double)tref[q] : 0.0;
    S* buf = (S*)a.buf_v + I.pop_off;
    for (int k = 0; k < 9; ++k) {
        const int ex = EX(k), ey = EY(k);
        const int js = j - ey;
        const int is = wrapx(i - ex, nx);
        const double w = W9<double>::w(k);
        size_t kf, kg, kh;
        double ref_f, ref_h, sgn_h = 1.0, add_h = 0.0;
        if (js >= 0 && js < ny) {
            kf = pidx(nx, ny, 0, k, js, is); kg = pidx(nx, ny, 1, k, js, is); kh = pidx(nx, ny, 2, k, js, is);
            ref_f = DEV ? w * ((double)phi0[js] + (double)a.dl[I.node_off + (size_t)js * nx + is] * DL_Q) + qf(k, js) : 0.0;
            ref_h = DEV ? w * (double)tref[(size_t)js * nx + is] : 0.0;
        } else {
            const int mir = MIRY(k), opp = OPP(k);
            const double Tw = (ey > 0) ? (double)tw[i] : I.T_c;
            kf = pidx(nx, ny, 0, mir, j, is); kg = pidx(nx, ny, 1, opp, j, i); kh = pidx(nx, ny, 2, opp, j, i);
            ref_f = DEV ? w * ((double)phi0[j] + (double)a.dl[I.node_off + (size_t)j * nx + is] * DL_Q) + qf(mir, j) : 0.0;
            // h_k = -(stored + w Tr_self) + 2 w T_w
            sgn_h = -1.0;
            ref_h = 0.0;
            add_h = 2.0 * w * Tw - w * Tr_self;
        }
        const size_t o0 = ((size_t)(0 * 9 + k) * ny + j) * nx + i;
        const size_t o1 = ((size_t)(1 * 9 + k) * ny + j) * nx + i;
        const size_t o2 = ((size_t)(2 * 9 + k) * ny + j) * nx + i;
        if (a.dir == 0) {
            a.state[o0] = ref_f + (double)buf[kf];
            a.state[o1] = w * pr + (double)buf[kg];
            a.state[o2] = sgn_h * (double)buf[kh] + ref_h + add_h;
        } else {
            buf[kf] = S(a.state[o0] - ref_f);
            buf[kg] = S(a.state[o1] - w * pr);
            buf[kh] = S(sgn_h * (a.state[o2] - ref_h - add_h));
        }
    }
}

// Float32 mode: after a check step, the step kernel has stored this step's
// populations relative to new temperature references (written to a second
// array); make them current.  Channels that were active in that step only.
__global__ __launch_bounds__(256) void tref_copy_kernel(TrefArgs a) {
    const int inst = blockIdx.y;
    const Inst& I = a.insts[inst];
    if (!I.active) return;
    const long long n = (long long)I.nx * I.ny;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    a.tref[I.node_off + q] = a.tref_new[I.node_off + q];
    a.dl[I.node_off + q] = a.dl_new[I.node_off + q];
}

// Float32 mode, after a check step: the flux reference A = 2 fq of f moves
// to the row mean of the actual post-collision flux (the check step's row
// sums of the stored deviation t01 - A, over the channel's tile columns in a
// fixed order).  Near a steady, nearly flat interface the stored flux
// deviations then shrink to their variation along x.  Also forms fr for the
// new table (fr_next) and for the switch step that reads the old table and
// writes against the new one (fr_sw):
//   fr = (1 - w) (r01 + fq_read(j-1) + fq_read(j+1)) + w M theta0 n0y - 2 fq_write(j).
// One thread per row (grid: row blocks x channels); channels retired before
// this check are left alone.  A thread also forms the new table of its two
// neighbour rows (the same fixed-order sums as their own threads), so no
// second pass is needed for the remainder tables.
__global__ __launch_bounds__(256) void flux_next_kernel(FluxArgs a) {
    const Inst& I = a.insts[blockIdx.y];
    if (!I.active) return;
    const int ny = I.ny, j = blockIdx.x * 256 + (int)threadIdx.x;
    if (j >= ny) return;
    const long long r0 = I.row_off + 2;            // row j lives at r0 + j
    auto fq_new = [&](int jj) -> float {           // new table at row jj, 0 <= jj < ny
        double s = 0.0;
        for (int c = 0; c < I.tiles_x; ++c) s += a.rowpart[I.rp_off + (size_t)jj * I.rp_stride + c];
        return (float)((double)a.fq[r0 + jj] + 0.5 * s / (double)I.nx);
    };
    const float q = fq_new(j);
    const float qm = j > 0 ? fq_new(j - 1) : -q;          // wall images, as the set-up builds them
    const float qp = j < ny - 1 ? fq_new(j + 1) : -q;
    a.fq_next[r0 + j] = q;
    if (j == 0) {
        a.fq_next[r0 - 1] = -q;
        a.fq_next[r0 - 2] = a.fq[r0 - 2];
    }
    if (j == ny - 1) {
        a.fq_next[r0 + ny] = -q;
        a.fq_next[r0 + ny + 1] = a.fq[r0 + ny + 1];
    }
    const double wl = 1.0 - I.w_phi;
    const double c = a.frc[r0 + j], qn = 2.0 * (double)q;
    a.fr_next[r0 + j] = (float)(c + wl * ((double)qm + (double)qp) - qn);
    a.fr_sw[r0 + j] = (float)(c + wl * ((double)a.fq[r0 + j - 1] + (double)a.fq[r0 + j + 1]) - qn);
}

// After the switch step: the new flux tables become current (channels that
// took part in that step only); a later switch without a new check is then
// the identity.
__global__ __launch_bounds__(256) void flux_copy_kernel(FluxArgs a) {
    const Inst& I = a.insts[blockIdx.y];
    if (!I.active) return;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= I.ny + 4) return;
    const long long r = I.row_off + k;
    a.fq[r] = a.fq_next[r];
    a.fr[r] = a.fr_next[r];
    a.fr_sw[r] = a.fr_next[r];
}

// Chunk flags of the phi-reference offsets: one wave per 64 x 8 chunk, one
// lane per column; the flag is 1 when any offset in the chunk is nonzero.
__global__ __launch_bounds__(DLZ_CX) void dl_flags_kernel(const Inst* insts, const int32_t* dl, int32_t* dlz) {
    const Inst& I = insts[blockIdx.y];
    const int nx = I.nx, ny = I.ny;
    const int ncx = (nx + DLZ_CX - 1) / DLZ_CX, ncy = (ny + DLZ_CY - 1) / DLZ_CY;
    const int c = blockIdx.x;
    if (c >= ncx * ncy) return;
    const int cx = c % ncx, cy = c / ncx;
    const int col = cx * DLZ_CX + (int)threadIdx.x;
    int nz = 0;
    if (col < nx) {
        for (int r = 0; r < DLZ_CY; ++r) {
            const int row = cy * DLZ_CY + r;
            if (row < ny && dl[I.node_off + (long long)row * nx + col] != 0) nz = 1;
        }
    }
    nz = __any(nz);
    if (threadIdx.x == 0) dlz[I.chunk_off + c] = nz ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers (instantiations).
template <int TX, int TY, class S, class R, bool DEV>
static hipError_t launch_step_t(const StepArgs& a, int mode, int grid, hipStream_t st) {
    dim3 g(grid), b(TX * TY);
    if (mode == 0) hipLaunchKernelGGL((step_kernel<TX, TY, S, R, DEV, 0>), g, b, 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((step_kernel<TX, TY, S, R, DEV, 1>), g, b, 0, st, a);
    else hipLaunchKernelGGL((step_kernel<TX, TY, S, R, DEV, 2>), g, b, 0, st, a);
    return hipGetLastError();
}

template <class S, class R, bool DEV>
static hipError_t launch_step_p(const StepArgs& a, int mode, int grid, int tx, int ty, hipStream_t st) {
    if (tx == 64 && ty == 8) return launch_step_t<64, 8, S, R, DEV>(a, mode, grid, st);
    if (tx == 32 && ty == 8) return launch_step_t<32, 8, S, R, DEV>(a, mode, grid, st);
    if (tx == 64 && ty == 4) return launch_step_t<64, 4, S, R, DEV>(a, mode, grid, st);
    if (tx == 16 && ty == 16) return launch_step_t<16, 16, S, R, DEV>(a, mode, grid, st);
    if (tx == 64 && ty == 16) return launch_step_t<64, 16, S, R, DEV>(a, mode, grid, st);
    if (tx == 128 && ty == 8) return launch_step_t<128, 8, S, R, DEV>(a, mode, grid, st);
    return hipErrorInvalidValue;
}

hipError_t launch_step(int prec, const StepArgs& a, int mode, int grid, int tx, int ty, hipStream_t st) {
    if (prec == 0) return launch_step_p<double, double, false>(a, mode, grid, tx, ty, st);
    return launch_step_p<float, float, true>(a, mode, grid, tx, ty, st);
}

hipError_t launch_finalize(const FinArgs& a, int n_inst, hipStream_t st) {
    hipLaunchKernelGGL(check_sums_kernel, dim3(a.chk_nb, n_inst), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(n_inst), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_counter(long long* c, long long n, hipStream_t st) {
    hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, c, n);
    return hipGetLastError();
}

hipError_t launch_count_active(const Inst* insts, int n, int* out, hipStream_t st) {
    hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(256), 0, st, insts, n, out);
    return hipGetLastError();
}

hipError_t launch_init(int prec, const InitArgs& a, int max_nodes, int n_inst, hipStream_t st) {
    dim3 g((max_nodes + 255) / 256, n_inst), b(256);
    if (prec == 0) hipLaunchKernelGGL((init_kernel<double, double, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((init_kernel<float, float, true>), g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tref_copy(const TrefArgs& a, int max_nodes, int n_inst, hipStream_t st) {
    hipLaunchKernelGGL(tref_copy_kernel, dim3((max_nodes + 255) / 256, n_inst), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_flux_next(const FluxArgs& a, int max_rows, int n_inst, hipStream_t st) {
    hipLaunchKernelGGL(flux_next_kernel, dim3((max_rows + 255) / 256, n_inst), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_flux_copy(const FluxArgs& a, int max_rows, int n_inst, hipStream_t st) {
    hipLaunchKernelGGL(flux_copy_kernel, dim3((max_rows + 4 + 255) / 256, n_inst), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dl_flags(const Inst* insts, const int32_t* dl, int32_t* dlz, int max_chunks, int n_inst,
                           hipStream_t st) {
    if (max_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(dl_flags_kernel, dim3(max_chunks, n_inst), dim3(DLZ_CX), 0, st, insts, dl, dlz);
    return hipGetLastError();
}

hipError_t launch_state(int prec, const StateArgs& a, int nodes, hipStream_t st) {
    dim3 g((nodes + 255) / 256), b(256);
    if (prec == 0) hipLaunchKernelGGL((state_kernel<double, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((state_kernel<float, true>), g, b, 0, st, a);
    return hipGetLastError();
}

}  // namespace lbm
