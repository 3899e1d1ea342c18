// Shared device/host definitions of the L-sweeps library: complex arithmetic, the
// per-subdomain and per-solve descriptors that drive the batched kernels, and the
// kernel launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lsw {

// ---------------------------------------------------------------- complex numbers
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T re, T im) { return cx<T>{re, im}; }
template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// acc + a b as four fused multiply-adds
template <typename T>
__host__ __device__ inline cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
    if constexpr (sizeof(T) == 4) {
        acc.re = __builtin_fmaf(a.re, b.re, acc.re);
        acc.re = __builtin_fmaf(-a.im, b.im, acc.re);
        acc.im = __builtin_fmaf(a.re, b.im, acc.im);
        acc.im = __builtin_fmaf(a.im, b.re, acc.im);
    } else {
        acc.re = __builtin_fma(a.re, b.re, acc.re);
        acc.re = __builtin_fma(-a.im, b.im, acc.re);
        acc.im = __builtin_fma(a.re, b.im, acc.im);
        acc.im = __builtin_fma(a.im, b.re, acc.im);
    }
    return acc;
}
template <typename T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__host__ __device__ inline T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T>
__host__ __device__ inline cx<T> cinv(cx<T> a) {
    T d = abs2(a);
    return {a.re / d, -a.im / d};
}
// acc + a*b
template <typename T>
__host__ __device__ inline cx<T> fma(cx<T> acc, cx<T> a, cx<T> b) {
    acc.re = acc.re + a.re * b.re - a.im * b.im;
    acc.im = acc.im + a.re * b.im + a.im * b.re;
    return acc;
}
template <typename T, typename U>
__host__ __device__ inline cx<T> cvt(cx<U> a) { return {static_cast<T>(a.re), static_cast<T>(a.im)}; }

using c64 = cx<float>;
using c128 = cx<double>;

// ---------------------------------------------------------------- plan descriptors

// Sides of a subdomain; trace lines are ordered by increasing grid index.
enum Side : int { SIDE_B = 0, SIDE_R = 1, SIDE_T = 2, SIDE_L = 3 };

// What a local solve computes (its right-hand side and receiving region chi).
enum Kind : int {
    KIND_STAGE1 = 0,  // r restricted to Omega_ij (Alg. computeLocSol)
    KIND_B = 1,       // polarized from the bottom trace, chi = rows >= lo   (up sweep)
    KIND_T = 2,       // from the top trace, chi = rows < hi                 (down sweep)
    KIND_L = 3,       // from the left trace, chi = cols >= lo               (right sweep)
    KIND_R = 4,       // from the right trace, chi = cols < hi               (left sweep)
    KIND_BL = 5,      // L-shaped, bottom + left legs, upper-right quadrant  (BL->TR sweep)
    KIND_TR = 6,      // top + right legs, lower-left quadrant               (TR->BL sweep)
    KIND_BR = 7,      // bottom + right legs, upper-left quadrant            (BR->TL sweep)
    KIND_TL = 8,      // top + left legs, lower-right quadrant               (TL->BR sweep)
    KIND_FINAL = 9,   // r on Omega_ij plus the accumulated sweep right-hand sides -> z
    KIND_UNIT = 10    // unit source on one trace-line point -> one column of Q (setup)
};

// Trace-line slots of a window (W x H): the 8 lines adjacent to the 4 interfaces, each
// over the full window extent, concatenated as B0 B1 T0 T1 (W points each) and
// L0 L1 R0 R1 (H points each); line 0 of a side has the smaller grid index.
__host__ __device__ inline int slot_B0(int W, int H) { return 0; }
__host__ __device__ inline int slot_T0(int W, int H) { return 2 * W; }
__host__ __device__ inline int slot_L0(int W, int H) { return 4 * W; }
__host__ __device__ inline int slot_R0(int W, int H) { return 4 * W + 2 * H; }
__host__ __device__ inline int slot_count(int W, int H) { return 4 * W + 4 * H; }

// One local problem (window of one CDD cell).
struct SubDesc {
    int W, H;            // window points along x and y
    int wx0, wy0;        // window origin on the extended grid
    int r0, r1, c0, c1;  // Omega_ij inside the window: rows [r0, r1), cols [c0, c1)
    int i, j;            // CDD row / column
    int tx, ty;          // offsets of this window's x and y tables in the table pool
    int sides;           // bit s set if side s (Side) is an interior interface
    int mid;             // middle block row of the twisted factorisation (H / 2)
    int L;               // number of trace-line slots, 4W + 4H
    long long g_off;     // offset (elements) of G_0 in the factor pool; G_k at g_off + k*W*W
    long long gs_off;    // offset of G_0 in the packed symmetric pool; G_k at gs_off + k*sym_block(W)
                         // (3D: at gs_off + k*4096*plane3_tiles(W*H))
    long long q_off;     // offset of Q = A_ij^-1[lines, lines] (L x L, column-major) in the Q pool
    long long fw_off;    // offset of this window (H x W, row-major) in the final right-hand-side array
};

// Packed storage of a complex symmetric W x W block G (G = G^T).  A = A^T makes every Schur
// complement of the block elimination symmetric, and so every inverse G_k.  The upper triangle
// is cut into 4x4 tiles: nt = ceil(W/4) tile rows, tiles (I, J) with I <= J numbered
// tau = I nt - I (I - 1) / 2 + (J - I), NTL = nt (nt + 1) / 2 of them.  Tile tau holds
// G[4I+i][4J+j] (zero outside the W x W block; diagonal tiles in full); its entry q = 4i + j
// sits at (q / 2) * 2 NTL + 2 tau + q % 2, so that the entry pair u (q = 2u, 2u+1) of
// consecutive tiles is contiguous.  With c[J][r] = sum over tile column J of G[r][.] v[.],
//   (G v)_r = sum_J c[J][r],  c[J][4I+i] = (tile (I,J) v_J)_i  (I <= J),  (tile (J,I)^T v_J)_i  (I > J).
__host__ __device__ inline int tile_nt(int W) { return (W + 3) / 4; }
__host__ __device__ inline int tile_count(int W) { return tile_nt(W) * (tile_nt(W) + 1) / 2; }
__host__ __device__ inline long long sym_block(int W) { return 16LL * tile_count(W); }
// row stride of the per-tile-column partial sums in the substitution kernel (10 mod 16 entries)
__host__ __device__ inline int sym_cstride(int W) { return 4 * tile_nt(W) + ((10 - 4 * tile_nt(W)) % 16 + 16) % 16; }
// largest nt whose upper triangle has at most `tiles` tiles
__host__ __device__ constexpr int sym_nt_max(int tiles) {
    int nt = 0;
    while ((nt + 1) * (nt + 2) / 2 <= tiles) ++nt;
    return nt;
}

// Packed storage of a complex symmetric plane block of a 3D beam (s = W*H unknowns, G = G^T):
// the upper triangle in 64 x 64 tiles, nb = ceil(s/64) tile rows, tiles (I, J) with I <= J numbered
// tau = I nb - I (I - 1) / 2 + (J - I) (entries past s zero, diagonal tiles in full), 4096 entries
// per tile and plane3_tiles(s) tiles per plane.  Inside a tile, lane l = 16 i4 + j4 of a
// 256-lane workgroup owns rows 4 i4 + a and columns 4 j4 + b (a, b < 4); its entry q = 4a + b sits
// at (q / 2) * 512 + 2 l + q % 2, so that chunk u = q / 2 of all lanes is one contiguous run.
__host__ __device__ inline int plane3_nb(int S) { return (S + 63) / 64; }
__host__ __device__ inline int plane3_tiles(int S) { return plane3_nb(S) * (plane3_nb(S) + 1) / 2; }

// Layout of one axis table of a window with P points (offset t in the table pool):
//   t + a        : 1/alpha at integer point a            (a = 0..P-1)
//   t + P + a    : alpha at half point a - 1/2           (a = 0..P)
// so the coupling of points a and a+1 uses index t + P + a + 1.

static constexpr int kMaxOut = 4;

// One local solve inside a front.  Trace offsets are element offsets into the trace
// pool of right-hand side 0 (add rhs * trace_stride).
struct SolveDesc {
    int sub;                     // SubDesc index
    int kind;                    // Kind
    int zpart;                   // which per-sweep accumulator receives U on Omega_ij
    int kf0, kf1;                // first and last block row with a nonzero right-hand side
    int kb0, kb1;                // first and last block row whose solution is needed
    int nout;                    // number of trace outputs
    long long in_h;              // incoming horizontal trace (2 x W), -1 if none
    long long in_v;              // incoming vertical trace (2 x H), -1 if none
    long long out_off[kMaxOut];  // output trace offsets
    int out_side[kMaxOut];       // Side of each output
    int out_acc[kMaxOut];        // 1: accumulate (+=), 0: assign (=)
    int unit_k, unit_c;          // KIND_UNIT: window point of the unit source
    long long q_col;             // KIND_UNIT: element offset of the Q column written
};

// One local solve of a sweep front in the trace-compressed form: the outgoing traces are
// Q[out lines, in slots] * g[in slots], where g is the polarized right-hand side on the
// (at most four) slot ranges that carry it.
struct GemvSolve {
    int sub, kind, sweep;        // sweep 1..8
    int nin;
    int in_start[4], in_len[4];  // slot ranges of the polarized right-hand side g (= the ranges of u~)
    int nout;
    long long in_h, in_v;        // incoming traces (offsets in the trace pool), -1 if none
    long long out_off[kMaxOut];
    int out_side[kMaxOut];
    int out_acc[kMaxOut];
    long long qp_off;            // Q'_s = Q P_s of this solve: column-major [nin][ld] block in the Q' pool
    int rows;                    // rows of Q'_s: the outgoing slots of all its output sides, side by side
    int ld;                      // leading dimension: rows rounded up to 16 (128-byte aligned columns)
    int row_base[kMaxOut];       // first row of each output side in Q'_s
};

// One work item of the trace-compressed sweeps: up to 64 outgoing trace values of one output
// side of one solve, out = Q'_s[rows, :] u~, with u~ gathered from the trace pool.
struct GemvItem {
    long long qoff;              // Q' pool element (first row of this chunk, column 0)
    long long qlen;              // elements from qoff to the end of the Q'_s block
    long long rng_off[4];        // trace-pool offsets of the contiguous ranges holding u~
    long long out_off;           // trace-pool offset of the first output
    int rng_len[4];
    int ld, nrow, nin, nrng, out_acc;
    int solve;                   // index of the solve
};

// One term of the polarization map of a sweep solve: g at window point `point` of window
// `sub` receives coef * (trace-pool value at `pool`).  Used to rebuild the final right-hand side.
struct PEntry {
    c128 coef;
    long long pool;
    int sub, point;
};

// Everything a kernel needs to evaluate the local or global 5-point coefficients.
struct Geometry {
    const c128* tab;      // table pool
    const double* m;      // squared slowness on the extended grid, [z][y][x]
    int Nx, Ny;           // extended grid
    double h, omega;
    int gtx, gty;         // offsets of the global x and y tables
    int Nz;               // 1 in 2D
    int gtz;              // offset of the global z table (3D)
};

}  // namespace lsw
