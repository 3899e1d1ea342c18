// Device kernels of the 3D problem over a beam CDD.
//
//  k_f3_build   S_k = D_k - C G C (App. A 7-point operator restricted to one xy plane of a
//               beam, minus the Schur terms of the planes already eliminated), batched
//  k_f2_build   the same for the line blocks of the 2D local problems (5-point operator)
//  k_f3_panel   Gauss-Jordan elimination of one column panel of every S_k (row pivoting), in
//               register sub-panels of 4 columns; k_f3_laswp takes its row interchanges to the
//               other columns
//  k_f3_prep    operands of the rank-b update of the other columns
//  k_f3_update  that update, a batched complex FP64 GEMM on matrix cores (v_mfma_f64_16x16x4f64)
//  k_f3_finish  column interchanges and the copy of G_k = S_k^-1 into the factor pool
//  k_rhs3       right-hand sides of the local solves of a front (stage 1 or eq. DiscPol2)
//  k_step3      one plane of the twisted block substitution of every solve of a front: each
//               workgroup computes 64 rows of G_k v (v staged in LDS, G_k streamed)
//  k_tile3      the same step on packed symmetric plane blocks: one 64 x 64 tile of the upper
//  k_red3       triangle per workgroup (tile v_J and tile^T v_I), then a fixed-order sum per row
//  k_pack3      packing of the plane blocks into that tile layout
//  k_epi3       the solution on Omega_ij and the outgoing trace planes
//  k_zsum3      z = sum of the per-sweep parts
//  k_matvec3    y = A x with the 7-point operator (FP64)
#include "launch3d.h"

namespace lsw {
namespace {

constexpr uint32_t kOob3 = 0x80000000u;   // per-lane offset that reads nothing (past the range check)

__device__ inline __amdgpu_buffer_rsrc_t rsrc3(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ inline cx<T> bload3(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline cx<float> bload3<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ inline cx<double> bload3<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// ------------------------------------------------------------------ 7-point coefficients
// Tables (common.h layout): tab[t + a] = 1/alpha at integer point a, tab[t + P + a] = alpha at
// the half point a - 1/2.  Symmetric form of App. A in 3D: s_x = alpha_x/(alpha_y alpha_z) at
// x half points (and cyclically), mass term omega^2 m/(alpha_x alpha_y alpha_z).
struct Box3 {
    int tx, Px, ty, Py, tz, Pz;
};
__device__ inline c128 c3x(const c128* tab, const Box3& b, int x, int y, int z, double ih2) {
    return -ih2 * (tab[b.tx + b.Px + x + 1] * tab[b.ty + y] * tab[b.tz + z]);   // (x,y,z)-(x+1,y,z)
}
__device__ inline c128 c3y(const c128* tab, const Box3& b, int x, int y, int z, double ih2) {
    return -ih2 * (tab[b.ty + b.Py + y + 1] * tab[b.tx + x] * tab[b.tz + z]);   // (x,y,z)-(x,y+1,z)
}
__device__ inline c128 c3z(const c128* tab, const Box3& b, int x, int y, int z, double ih2) {
    return -ih2 * (tab[b.tz + b.Pz + z + 1] * tab[b.tx + x] * tab[b.ty + y]);   // (x,y,z)-(x,y,z+1)
}
__device__ inline c128 d3(const c128* tab, const Box3& b, int x, int y, int z, double ih2, double om2m) {
    const c128 ix = tab[b.tx + x], iy = tab[b.ty + y], iz = tab[b.tz + z];
    const c128 sx = tab[b.tx + b.Px + x + 1] + tab[b.tx + b.Px + x];
    const c128 sy = tab[b.ty + b.Py + y + 1] + tab[b.ty + b.Py + y];
    const c128 sz = tab[b.tz + b.Pz + z + 1] + tab[b.tz + b.Pz + z];
    return ih2 * (sx * iy * iz + sy * ix * iz + sz * ix * iy) - om2m * (ix * iy * iz);
}
__device__ inline Box3 window_box(const SubDesc& s, const Geometry& g) {
    return Box3{s.tx, s.W, s.ty, s.H, g.gtz, g.Nz};
}

// ------------------------------------------------------------------ factorisation
__global__ void k_f3_build(Fact3Args a) {
    const Fact3Item it = a.items[blockIdx.y];
    const SubDesc s = a.subs[it.sub];
    const int n = a.n, W = s.W, S = s.W * s.H;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int p = (int)(idx % n), q = (int)(idx / n);
    c128* A = a.ws + (size_t)blockIdx.y * n * n;
    if (p >= S || q >= S) {
        A[idx] = mk(p == q ? 1.0 : 0.0, 0.0);
        return;
    }
    const Geometry& g = a.geo;
    const Box3 b = window_box(s, g);
    const double ih2 = 1.0 / (g.h * g.h);
    const int k = it.k;
    const int yp = p / W, xp = p - yp * W, yq = q / W, xq = q - yq * W;
    c128 v = mk(0.0, 0.0);
    if (p == q) {
        const double m = g.m[((size_t)k * g.Ny + s.wy0 + yp) * g.Nx + s.wx0 + xp];
        v = d3(g.tab, b, xp, yp, k, ih2, g.omega * g.omega * m);
    } else if (yp == yq && (xp - xq == 1 || xq - xp == 1)) {
        v = c3x(g.tab, b, min(xp, xq), yp, k, ih2);
    } else if (xp == xq && (yp - yq == 1 || yq - yp == 1)) {
        v = c3y(g.tab, b, xp, min(yp, yq), k, ih2);
    }
    const size_t SS = (size_t)S * S;
    if (it.below >= 0) {   // coupling of planes k-1 and k
        const c128 cp = c3z(g.tab, b, xp, yp, k - 1, ih2), cq = c3z(g.tab, b, xq, yq, k - 1, ih2);
        v = v - cp * a.G[s.g_off + (size_t)it.below * SS + (size_t)q * S + p] * cq;
    }
    if (it.above >= 0) {   // coupling of planes k and k+1
        const c128 cp = c3z(g.tab, b, xp, yp, k, ih2), cq = c3z(g.tab, b, xq, yq, k, ih2);
        v = v - cp * a.G[s.g_off + (size_t)it.above * SS + (size_t)q * S + p] * cq;
    }
    A[idx] = v;
}

// 2D line blocks (App. A 5-point operator restricted to grid line k of the window, x fastest):
// S_k = D_k - C_{k-1} G_below C_{k-1} - C_k G_above C_k with C the diagonal couplings between
// neighbouring lines, the same elimination as in 3D with lines for planes.
__device__ inline c128 l2x(const c128* tab, const SubDesc& s, int a, int k, double ih2) {
    return -ih2 * (tab[s.tx + s.W + a + 1] * tab[s.ty + k]);      // (a, k)-(a+1, k)
}
__device__ inline c128 l2y(const c128* tab, const SubDesc& s, int a, int k, double ih2) {
    return -ih2 * (tab[s.ty + s.H + k + 1] * tab[s.tx + a]);      // (a, k)-(a, k+1)
}

__global__ void k_f2_build(Fact3Args a) {
    const Fact3Item it = a.items[blockIdx.y];
    const SubDesc s = a.subs[it.sub];
    const int n = a.n, W = s.W;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int p = (int)(idx % n), q = (int)(idx / n);
    c128* A = a.ws + (size_t)blockIdx.y * n * n;
    if (p >= W || q >= W) {
        A[idx] = mk(p == q ? 1.0 : 0.0, 0.0);
        return;
    }
    const Geometry& g = a.geo;
    const c128* tab = g.tab;
    const double ih2 = 1.0 / (g.h * g.h);
    const int k = it.k;
    c128 v = mk(0.0, 0.0);
    if (p == q) {
        const double m = g.m[(size_t)(s.wy0 + k) * g.Nx + s.wx0 + p];
        const c128 sx = tab[s.tx + W + p + 1] + tab[s.tx + W + p];
        const c128 sy = tab[s.ty + s.H + k + 1] + tab[s.ty + s.H + k];
        v = ih2 * (sx * tab[s.ty + k] + sy * tab[s.tx + p]) - (g.omega * g.omega * m) * (tab[s.tx + p] * tab[s.ty + k]);
    } else if (p - q == 1 || q - p == 1) {
        v = l2x(tab, s, min(p, q), k, ih2);
    }
    const size_t WW = (size_t)W * W;
    if (it.below >= 0) {
        const c128 cp = l2y(tab, s, p, k - 1, ih2), cq = l2y(tab, s, q, k - 1, ih2);
        v = v - cp * a.G[s.g_off + (size_t)it.below * WW + (size_t)q * W + p] * cq;
    }
    if (it.above >= 0) {
        const c128 cp = l2y(tab, s, p, k, ih2), cq = l2y(tab, s, q, k, ih2);
        v = v - cp * a.G[s.g_off + (size_t)it.above * WW + (size_t)q * W + p] * cq;
    }
    A[idx] = v;
}

// Gauss-Jordan on columns [p0, p0 + b) of every matrix (b <= 32): for each column j, choose the
// pivot in rows >= j, interchange rows j and the pivot row within the panel, scale the pivot row,
// eliminate the column from every other row.  One workgroup of 1024 lanes per matrix; lane t owns
// rows t + 1024 r (r < RPT).  The panel is processed in sub-panels of 4 columns held in registers:
// their pivot steps touch only registers and the pivot rows of the other panel columns, and the
// other panel columns then receive the 4 steps at once as a rank-4 update (A[:, c] += (X - E) A[J, c],
// X the sub-panel after elimination, J its pivot rows), so the panel is read and written once per
// sub-panel instead of once per column.  The interchanges reach the columns outside the panel
// afterwards (k_f3_laswp), and those columns the whole panel's transformation as one rank-b update.
template <int RPT>
__global__ __launch_bounds__(1024) void k_f3_panel(Fact3Args a, int p0, int b) {
    constexpr int NT = 1024, SB = 4;
    __shared__ double wbest[NT / 64];
    __shared__ int wbi[NT / 64];
    __shared__ c128 rowx[2][SB];       // the sub-panel entries of the two rows being interchanged
    __shared__ c128 prow[SB];          // the scaled pivot row over the sub-panel
    __shared__ c128 trow[SB][32];      // the sub-panel's pivot rows over the other panel columns
    __shared__ int sh_piv, sh_sing;
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    c128* A = a.ws + (size_t)blockIdx.x * n * n;
    int* perm = a.perm + (size_t)blockIdx.x * n;
    if (tid == 0) sh_sing = 0;
    for (int s0 = 0; s0 < b; s0 += SB) {
        const int sb = min(SB, b - s0), cs = p0 + s0;   // sub-panel columns [cs, cs + sb)
        c128 x[RPT][SB];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + NT * r;
#pragma unroll
            for (int c = 0; c < SB; ++c) x[r][c] = (i < n && c < sb) ? A[i + (size_t)(cs + c) * n] : mk(0.0, 0.0);
        }
#pragma unroll
        for (int c = 0; c < SB; ++c) {   // unrolled: the register sub-panel is indexed by constants
            if (c >= sb) break;           // (sb is the same for the whole workgroup)
            const int j = cs + c;
            double best = -1.0;
            int bi = j;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + NT * r;
                const double v = abs2(x[r][c]);
                if (i >= j && i < n && v > best) {
                    best = v;
                    bi = i;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off);
                const int oi = __shfl_xor(bi, off);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (lane == 0) {
                wbest[wv] = best;
                wbi[wv] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                double bb = wbest[0];
                int ii = wbi[0];
                for (int w = 1; w < NT / 64; ++w)
                    if (wbest[w] > bb || (wbest[w] == bb && wbi[w] < ii)) {
                        bb = wbest[w];
                        ii = wbi[w];
                    }
                sh_piv = ii;
                perm[j] = ii;
                if (!(bb > 0.0)) sh_sing = 1;
            }
            __syncthreads();
            const int pr = sh_piv;
            // rows j and pr: their sub-panel entries through LDS, the other panel columns in place
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + NT * r;
                if (i == j || i == pr)
#pragma unroll
                    for (int cc = 0; cc < SB; ++cc) rowx[i == j ? 0 : 1][cc] = x[r][cc];
            }
            if (pr != j && tid < b && (tid < s0 || tid >= s0 + sb)) {
                c128* e1 = A + j + (size_t)(p0 + tid) * n;
                c128* e2 = A + pr + (size_t)(p0 + tid) * n;
                const c128 t = *e1;
                *e1 = *e2;
                *e2 = t;
            }
            __syncthreads();
            // after the interchange row j holds what row pr held
            const c128 piv = rowx[pr != j ? 1 : 0][c];
            const c128 inv = abs2(piv) > 0.0 ? cinv(piv) : mk(0.0, 0.0);
            if (tid < SB) prow[tid] = tid == c ? inv : rowx[pr != j ? 1 : 0][tid] * inv;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + NT * r;
                if (pr != j && i == pr)
#pragma unroll
                    for (int cc = 0; cc < SB; ++cc) x[r][cc] = rowx[0][cc];   // row pr takes row j's old entries
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + NT * r;
                if (i == j) {
#pragma unroll
                    for (int cc = 0; cc < SB; ++cc) x[r][cc] = prow[cc];
                } else {
                    const c128 f = x[r][c];
#pragma unroll
                    for (int cc = 0; cc < SB; ++cc) x[r][cc] = cc == c ? -(f * inv) : x[r][cc] - f * prow[cc];
                }
            }
            __syncthreads();   // rowx / prow are rewritten by the next pivot step
        }
        // write the sub-panel back; the other panel columns (before and after it) take its
        // transformation X: A[i, c] += X[i, :] T[:, c] for the rows i outside [cs, cs + sb) and
        // A[i, c] = X[i, :] T[:, c] for those inside, T = rows [cs, cs + sb) of those columns (never
        // X - E: with pivots far from 1, 1/pivot - 1 would cancel the pivot rows' digits)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + NT * r;
            if (i < n)
#pragma unroll
                for (int c = 0; c < SB; ++c)
                    if (c < sb) A[i + (size_t)(cs + c) * n] = x[r][c];
        }
        for (int e = tid; e < SB * 32; e += NT) {
            const int cc = e / 32, col = e % 32;
            trow[cc][col] = (cc < sb && col < b && (col < s0 || col >= s0 + sb)) ? A[cs + cc + (size_t)(p0 + col) * n]
                                                                                  : mk(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + NT * r;
            if (i >= n) continue;
            const bool pivot_row = i >= cs && i < cs + sb;
            for (int col = 0; col < b; ++col) {
                if (col >= s0 && col < s0 + sb) continue;
                c128* e = A + i + (size_t)(p0 + col) * n;
                c128 v = pivot_row ? mk(0.0, 0.0) : *e;
#pragma unroll
                for (int cc = 0; cc < SB; ++cc) v = cmac(v, x[r][cc], trow[cc][col]);
                *e = v;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && sh_sing) a.status[a.items[blockIdx.x].sub] = 1;
}

// The same panel elimination for n <= 256 (2D line blocks): the whole n x b panel lives in LDS
// (128 KB at n = 256, b = 32), so every pivot step is an LDS pass between barriers.
__global__ __launch_bounds__(1024) void k_f3_panel_lds(Fact3Args a, int p0, int b) {
    constexpr int NT = 1024;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    c128* sp = reinterpret_cast<c128*>(smem);   // [b][n] column-major panel
    c128* colf = sp + (size_t)b * n;            // the multipliers of the current pivot column
    __shared__ double wbest[NT / 64];
    __shared__ int wbi[NT / 64];
    __shared__ int sh_piv, sh_sing;
    c128* A = a.ws + (size_t)blockIdx.x * n * n;
    int* perm = a.perm + (size_t)blockIdx.x * n;
    if (tid == 0) sh_sing = 0;
    for (int e = tid; e < n * b; e += NT) {
        const int c = e / n, i = e - c * n;
        sp[e] = A[i + (size_t)(p0 + c) * n];
    }
    __syncthreads();
    for (int jj = 0; jj < b; ++jj) {
        const int j = p0 + jj;
        double best = -1.0;
        int bi = j;
        if (tid >= j && tid < n) {
            best = abs2(sp[jj * n + tid]);
            bi = tid;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (lane == 0) {
            wbest[wv] = best;
            wbi[wv] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double bb = wbest[0];
            int ii = wbi[0];
            for (int w = 1; w < NT / 64; ++w)
                if (wbest[w] > bb || (wbest[w] == bb && wbi[w] < ii)) {
                    bb = wbest[w];
                    ii = wbi[w];
                }
            sh_piv = ii;
            perm[j] = ii;
            if (!(bb > 0.0)) sh_sing = 1;
        }
        __syncthreads();
        const int pr = sh_piv;
        if (pr != j && tid < b) {
            const c128 t = sp[tid * n + j];
            sp[tid * n + j] = sp[tid * n + pr];
            sp[tid * n + pr] = t;
        }
        __syncthreads();
        const c128 piv = sp[jj * n + j];
        const c128 inv = abs2(piv) > 0.0 ? cinv(piv) : mk(0.0, 0.0);
        if (tid < n) colf[tid] = sp[jj * n + tid];
        __syncthreads();
        if (tid < b) sp[tid * n + j] = tid == jj ? inv : sp[tid * n + j] * inv;
        __syncthreads();
        for (int e = tid; e < n * b; e += NT) {
            const int c = e / n, i = e - c * n;
            if (i == j) continue;
            const c128 f = colf[i];
            sp[e] = c == jj ? -(f * inv) : sp[e] - f * sp[c * n + j];
        }
        __syncthreads();
    }
    for (int e = tid; e < n * b; e += NT) {
        const int c = e / n, i = e - c * n;
        A[i + (size_t)(p0 + c) * n] = sp[e];
    }
    if (tid == 0 && sh_sing) a.status[a.items[blockIdx.x].sub] = 1;
}

// The row interchanges of panel [p0, p0 + b), in order, applied to every column outside the panel
// (one lane per column).
__global__ void k_f3_laswp(Fact3Args a, int p0, int b) {
    const int n = a.n;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || (c >= p0 && c < p0 + b)) return;
    c128* col = a.ws + (size_t)blockIdx.y * n * n + (size_t)c * n;
    const int* perm = a.perm + (size_t)blockIdx.y * n;
    for (int j = p0; j < p0 + b; ++j) {
        const int r = perm[j];
        if (r != j) {
            const c128 t = col[j];
            col[j] = col[r];
            col[r] = t;
        }
    }
}

__global__ void k_f3_prep(Fact3Args a, int p0, int b, c128* Pbar, c128* T) {
    const int n = a.n;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * b) return;
    const c128* A = a.ws + (size_t)blockIdx.y * n * n;
    c128* P = Pbar + (size_t)blockIdx.y * n * b;
    c128* Tb = T + (size_t)blockIdx.y * n * b;
    {   // P[i, cc] = A[i, p0 + cc]: the panel's transformation, column cc
        const int i = (int)(idx % n), cc = (int)(idx / n);
        P[idx] = A[i + (size_t)(p0 + cc) * n];
    }
    {   // T[cc, c] = A[p0 + cc, c]
        const int cc = (int)(idx % b), c = (int)(idx / b);
        Tb[idx] = A[p0 + cc + (size_t)c * n];
    }
}

// The rank-b update of a blocked Gauss-Jordan step on matrix cores: for every matrix of the batch
// and c in [0, m), W[i, c0 + c] += P[i, :] T[:, c0 + c] for the rows i outside the panel's pivot rows
// [j0, j0 + b) and W[i, c0 + c] = P[i, :] T[:, c0 + c] for those inside (P = the panel's
// transformation, n x b column-major, ld n; T = its pivot rows of all columns, b x n, ld b).  The
// pivot rows are overwritten, not updated by (P - E) T: the diagonal of P holds 1/pivot, and
// 1/pivot - 1 would cancel their digits when the pivots are far from 1.  One workgroup of four waves owns a 64 x 64 tile
// of W; each wave a 32 x 32 quarter as 2 x 2 blocks of 16 x 16 accumulated by
// v_mfma_f64_16x16x4f64 over k in steps of 4.  A complex block product is four real ones,
// Re += Pr Tr + (-Pi) Ti, Im += Pr Ti + Pi Tr.  Lane l holds P[16-row block row l % 16][k0 + l / 16]
// and T[k0 + l / 16][16-column block column l % 16], and accumulator entry v of lane l is row
// l / 16 + 4 v, column l % 16 of its block (the
// operand and result layout of the FP64 16x16x4 instruction; the FP32 one places rows 4 (l / 16) + v).
// The tile of W is read once into the accumulators and written once.
typedef double mfd4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_f3_update(const c128* __restrict__ P, const c128* __restrict__ T,
                                                   c128* __restrict__ Wm, int n, int b, int j0, int c0, int m) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // Workgroup L runs on XCD L mod 8.  Each XCD takes a contiguous range of the tiles (matrix
    // slowest, then column tile, then row tile), so the workgroups that read the same matrix's P and
    // T share one XCD's L2.
    const uint32_t total = gridDim.x, L = blockIdx.x;
    const uint32_t per = total / 8, extra = total % 8, xcd = L % 8;
    const uint32_t t = xcd * per + min(xcd, extra) + L / 8;
    const uint32_t nrt = (uint32_t)(n + 63) / 64, nct = (uint32_t)(m + 63) / 64;
    const int r0 = (int)(t % nrt) * 64 + 32 * (wv & 1);
    const int q0 = (int)((t / nrt) % nct) * 64 + 32 * (wv >> 1);   // column offset within [0, m)
    const size_t z = t / (nrt * nct);
    const c128* Pz = P + z * (size_t)n * b;
    const c128* Tz = T + z * (size_t)n * b;
    c128* Wz = Wm + z * (size_t)n * n;
    mfd4 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int col = q0 + 16 * bj + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + 16 * bi + lk + 4 * v;
                c128 w = mk(0.0, 0.0);
                if (row < n && col < m && (row < j0 || row >= j0 + b)) w = Wz[row + (size_t)(c0 + col) * n];
                acc_re[bi][bj][v] = w.re;
                acc_im[bi][bj][v] = w.im;
            }
        }
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4) {
        if (k0 >= b) break;
        const int k = k0 + lk;
        double ar[2], ai[2], an[2], br[2], bim[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
            const int row = r0 + 16 * bi + li;
            c128 v = mk(0.0, 0.0);
            if (k < b && row < n) v = Pz[row + (size_t)k * n];
            ar[bi] = v.re;
            ai[bi] = v.im;
            an[bi] = -v.im;
        }
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int col = q0 + 16 * bj + li;
            c128 v = mk(0.0, 0.0);
            if (k < b && col < m) v = Tz[k + (size_t)(c0 + col) * b];
            br[bj] = v.re;
            bim[bj] = v.im;
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                acc_re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[bi], br[bj], acc_re[bi][bj], 0, 0, 0);
                acc_re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(an[bi], bim[bj], acc_re[bi][bj], 0, 0, 0);
                acc_im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[bi], bim[bj], acc_im[bi][bj], 0, 0, 0);
                acc_im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[bi], br[bj], acc_im[bi][bj], 0, 0, 0);
            }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int col = q0 + 16 * bj + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + 16 * bi + lk + 4 * v;
                if (row < n && col < m) Wz[row + (size_t)(c0 + col) * n] = mk(acc_re[bi][bj][v], acc_im[bi][bj][v]);
            }
        }
}

// The row interchanges undone as column interchanges, in reverse order, composed into one column
// permutation per matrix: column q of the inverse is column src[q] of the eliminated matrix.
__global__ void k_f3_perm(Fact3Args a, int* src) {
    if (threadIdx.x != 0) return;
    const int n = a.n;
    const int* perm = a.perm + (size_t)blockIdx.x * n;
    int* sq = src + (size_t)blockIdx.x * n;
    for (int q = 0; q < n; ++q) sq[q] = q;
    for (int j = n - 1; j >= 0; --j) {
        const int r = perm[j];
        if (r != j) {
            const int t = sq[j];
            sq[j] = sq[r];
            sq[r] = t;
        }
    }
}

// G_k = the s x s inverse (column-major), gathered through the column permutation
__global__ void k_f3_finish(Fact3Args a, const int* src) {
    const Fact3Item it = a.items[blockIdx.y];
    const SubDesc s = a.subs[it.sub];
    const int n = a.n, S = a.line ? s.W : s.W * s.H;
    const c128* A = a.ws + (size_t)blockIdx.y * n * n;
    const int* sq = src + (size_t)blockIdx.y * n;
    c128* G = a.G + s.g_off + (size_t)it.k * S * S;   // S = W (2D lines) or W H (3D planes)
    const size_t SS = (size_t)S * S;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < SS; idx += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(idx % S), q = (int)(idx / S);
        G[idx] = A[p + (size_t)sq[q] * n];
    }
}

// ------------------------------------------------------------------ sweeps
template <typename T>
__device__ inline bool chi3(int kind, const SubDesc& s, int y, int x) {
    switch (kind) {
        case KIND_B: return y >= s.r0;
        case KIND_T: return y < s.r1;
        case KIND_L: return x >= s.c0;
        case KIND_R: return x < s.c1;
        case KIND_BL: return y >= s.r0 && x >= s.c0;
        case KIND_TR: return y < s.r1 && x < s.c1;
        case KIND_BR: return y >= s.r0 && x < s.c1;
        case KIND_TL: return y < s.r1 && x >= s.c0;
        default: return false;
    }
}

// incoming trace value at (x, y) of plane z: trace arrays are [line][z][along the side];
// L legs are restricted to the receiving quadrant and the horizontal leg is used on the point
// both legs share
template <typename T>
__device__ inline cx<T> utilde3(int kind, const SubDesc& s, int Nz, const cx<T>* in_h, const cx<T>* in_v, int y,
                                int x, int z) {
    const bool corner = kind >= KIND_BL;
    const bool hB = (kind == KIND_B || kind == KIND_BL || kind == KIND_BR);
    const bool hT = (kind == KIND_T || kind == KIND_TR || kind == KIND_TL);
    const bool vL = (kind == KIND_L || kind == KIND_BL || kind == KIND_TL);
    const bool vR = (kind == KIND_R || kind == KIND_TR || kind == KIND_BR);
    if (hB || hT) {
        const int l0 = hB ? s.r0 - 1 : s.r1 - 1;
        const bool in_cols = !corner || (vL ? x >= s.c0 : x < s.c1);
        if ((y == l0 || y == l0 + 1) && in_cols) return in_h[((size_t)(y - l0) * Nz + z) * s.W + x];
    }
    if (vL || vR) {
        const int l0 = vL ? s.c0 - 1 : s.c1 - 1;
        const bool in_rows = !corner || (hB ? y >= s.r0 : y < s.r1);
        if ((x == l0 || x == l0 + 1) && in_rows) return in_v[((size_t)(x - l0) * Nz + z) * s.H + y];
    }
    return cx<T>{T(0), T(0)};
}

// eq. DiscPol2 at (x, y, z): sum over the in-plane neighbours q across the boundary of chi of
// A_pq (chi_q - chi_p) u~_q (the z neighbours share chi)
template <typename T>
__device__ inline c128 polar3(int kind, const SubDesc& s, const Geometry& g, const Box3& b, const cx<T>* in_h,
                              const cx<T>* in_v, int y, int x, int z) {
    const bool cp = chi3<T>(kind, s, y, x);
    const double ih2 = 1.0 / (g.h * g.h);
    c128 acc = mk(0.0, 0.0);
    auto add = [&](c128 A, cx<T> u) {
        const c128 t = A * cvt<double>(u);
        acc = cp ? acc - t : acc + t;
    };
    if (x > 0 && chi3<T>(kind, s, y, x - 1) != cp)
        add(c3x(g.tab, b, x - 1, y, z, ih2), utilde3<T>(kind, s, g.Nz, in_h, in_v, y, x - 1, z));
    if (x + 1 < s.W && chi3<T>(kind, s, y, x + 1) != cp)
        add(c3x(g.tab, b, x, y, z, ih2), utilde3<T>(kind, s, g.Nz, in_h, in_v, y, x + 1, z));
    if (y > 0 && chi3<T>(kind, s, y - 1, x) != cp)
        add(c3y(g.tab, b, x, y - 1, z, ih2), utilde3<T>(kind, s, g.Nz, in_h, in_v, y - 1, x, z));
    if (y + 1 < s.H && chi3<T>(kind, s, y + 1, x) != cp)
        add(c3y(g.tab, b, x, y, z, ih2), utilde3<T>(kind, s, g.Nz, in_h, in_v, y + 1, x, z));
    return acc;
}

template <typename T>
__global__ void k_rhs3(Chain3Args a, int smax) {
    const SolveDesc& d = a.descs[blockIdx.y];
    const SubDesc s = a.subs[d.sub];
    const Geometry& g = a.geo;
    const int rhs = blockIdx.z, S = s.W * s.H;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)g.Nz * smax) return;
    const int z = (int)(idx / smax), p = (int)(idx % smax);
    cx<T>* out = reinterpret_cast<cx<T>*>(a.rhs) + ((size_t)rhs * a.nslots + blockIdx.y) * a.slot_stride;
    c128 v = mk(0.0, 0.0);
    if (p < S) {
        const int y = p / s.W, x = p - y * s.W;
        if (d.kind == KIND_STAGE1) {
            if (y >= s.r0 && y < s.r1 && x >= s.c0 && x < s.c1) {
                const size_t N = (size_t)g.Nx * g.Ny * g.Nz;
                v = a.r[(size_t)rhs * N + ((size_t)z * g.Ny + s.wy0 + y) * g.Nx + s.wx0 + x];
            }
        } else {
            const cx<T>* tr = reinterpret_cast<const cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
            v = polar3<T>(d.kind, s, g, window_box(s, g), d.in_h >= 0 ? tr + d.in_h : nullptr,
                          d.in_v >= 0 ? tr + d.in_v : nullptr, y, x, z);
        }
    }
    out[idx] = cvt<T>(v);
}

// The plane of one half at step (phase, t) of the twisted substitution (planes k < m eliminated
// from below, k > m from above, m last) and the planes whose results enter its input:
//   phase 0, half 0: y_k = G_k (g_k - C_{k-1} y_{k-1}), k = t
//   phase 0, half 1: y_k = G_k (g_k - C_k y_{k+1}),     k = Nz-1-t
//   phase 1:         x_m = G_m (g_m - C_{m-1} y_{m-1} - C_m y_{m+1})
//   phase 2, half 0: x_k = y_k - G_k C_k x_{k+1},       k = m-1-t
//   phase 2, half 1: x_k = y_k - G_k C_{k-1} x_{k-1},   k = m+1+t
// prev/prev2 are the planes read (-1: none), cpl/cpl2 the coupling planes.  False: no plane.
struct StepPlane {
    int k, prev, prev2, cpl, cpl2;
};
__device__ inline bool step_plane(int phase, int t, int half, int Nz, int m, StepPlane& sp) {
    sp.prev = sp.prev2 = -1;
    sp.cpl = sp.cpl2 = 0;
    if (phase == 0) {
        if (half == 0) {
            if (t >= m) return false;
            sp.k = t;
            if (t > 0) sp.prev = sp.cpl = sp.k - 1;
        } else {
            if (t >= Nz - 1 - m) return false;
            sp.k = Nz - 1 - t;
            if (t > 0) { sp.prev = sp.k + 1; sp.cpl = sp.k; }
        }
    } else if (phase == 1) {
        if (half == 1) return false;
        sp.k = m;
        if (m >= 1) sp.prev = sp.cpl = m - 1;
        if (m + 1 <= Nz - 1) { sp.prev2 = m + 1; sp.cpl2 = m; }
    } else {
        if (half == 0) {
            if (t >= m) return false;
            sp.k = m - 1 - t;
            sp.prev = sp.k + 1;
            sp.cpl = sp.k;
        } else {
            if (t >= Nz - 1 - m) return false;
            sp.k = m + 1 + t;
            sp.prev = sp.cpl = sp.k - 1;
        }
    }
    return true;
}

// entry c of the vector the plane block multiplies: g_k - couplings * neighbours (phases 0, 1),
// or C x_prev (phase 2)
template <typename T>
__device__ inline cx<T> step_input(int phase, const StepPlane& sp, const SubDesc& s, const Geometry& g, const Box3& b,
                                   double ih2, const cx<T>* R, const cx<T>* Y, int smax, int c) {
    const int y = c / s.W, x = c - y * s.W;
    if (phase == 2) return cvt<T>(c3z(g.tab, b, x, y, sp.cpl, ih2)) * Y[(size_t)sp.prev * smax + c];
    cx<T> val = R[(size_t)sp.k * smax + c];
    if (sp.prev >= 0) val = val - cvt<T>(c3z(g.tab, b, x, y, sp.cpl, ih2)) * Y[(size_t)sp.prev * smax + c];
    if (sp.prev2 >= 0) val = val - cvt<T>(c3z(g.tab, b, x, y, sp.cpl2, ih2)) * Y[(size_t)sp.prev2 * smax + c];
    return val;
}

// One step of the twisted substitution on the full plane blocks, for every (solve, half) of a
// front: workgroup (chunk, 2*slot + half) forms v in LDS and computes rows [64*chunk, 64*chunk + 64)
// of G_k v, one row per lane, the 16 waves splitting the columns of the column-major block.
template <typename T>
__global__ __launch_bounds__(1024) void k_step3(Chain3Args a, int smax, int phase, int t) {
    constexpr int NT = 1024, NW = NT / 64, KB = sizeof(T) == 4 ? 16 : 8;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* v = reinterpret_cast<cx<T>*>(smem);   // [S]
    __shared__ cx<T> part[NW][64];
    const int slot = blockIdx.y >> 1, half = blockIdx.y & 1, rhs = blockIdx.z;
    const SolveDesc& d = a.descs[slot];
    const SubDesc s = a.subs[d.sub];
    const Geometry& g = a.geo;
    const int S = s.W * s.H;
    const int row0 = blockIdx.x * 64;
    if (row0 >= S) return;
    StepPlane sp;
    if (!step_plane(phase, t, half, g.Nz, s.mid, sp)) return;
    const int k = sp.k;
    const Box3 b = window_box(s, g);
    const double ih2 = 1.0 / (g.h * g.h);
    const cx<T>* R = reinterpret_cast<const cx<T>*>(a.rhs) + ((size_t)rhs * a.nslots + slot) * a.slot_stride;
    cx<T>* Y = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)rhs * a.nslots + slot) * a.slot_stride;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int c = tid; c < S; c += NT) v[c] = step_input<T>(phase, sp, s, g, b, ih2, R, Y, smax, c);
    __syncthreads();
    const cx<T>* Gk = reinterpret_cast<const cx<T>*>(a.G) + s.g_off + (size_t)k * S * S;
    const __amdgpu_buffer_rsrc_t gr = rsrc3(Gk, (uint32_t)((size_t)S * S * sizeof(cx<T>)));
    const int row = row0 + lane;
    const bool valid = row < S;
    const int per = (S + NW - 1) / NW;
    const int c0 = wv * per, c1 = min(S, c0 + per);
    cx<T> acc{T(0), T(0)};
    for (int base = c0; base < c1; base += KB) {
        cx<T> q[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int c = base + u;
            q[u] = bload3<T>(gr, (valid && c < c1) ? (uint32_t)((size_t)c * S + row) * (uint32_t)sizeof(cx<T>) : kOob3);
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (base + u < c1) acc = acc + q[u] * v[base + u];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && valid) {
        cx<T> y = part[0][lane];
#pragma unroll
        for (int w = 1; w < NW; ++w) y = y + part[w][lane];
        cx<T>* out = Y + (size_t)k * smax + row;
        *out = (phase == 2) ? *out - y : y;
    }
}

// ------------------------------------------------------------------ packed symmetric plane blocks
// lane-to-lane moves inside rows of 16 lanes (DPP): quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror; every lane of a row ends with the row's sum
template <int CTRL>
__device__ inline float dpp3(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp3(double v) {
    const long long bits = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ inline T row16_sum(T x) {
    x += dpp3<0xB1>(x);
    x += dpp3<0x4E>(x);
    x += dpp3<0x141>(x);
    x += dpp3<0x140>(x);
    return x;
}

__device__ inline void tile3_ij(int tau, int nb, int& I, int& J) {
    int i = 0, rem = tau;
    while (rem >= nb - i) {
        rem -= nb - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

// Tile part of a packed step: workgroup (tau, 2*slot + half) multiplies tile (I, J) of G_k by v_J
// (rows of block I) and, off the diagonal, its transpose by v_I (rows of block J).  Lane l owns a
// 4 x 4 sub-block: row sums over the 16 lanes of a tile row by DPP, column sums through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_tile3(Chain3Args a, int smax, int phase, int t) {
    __shared__ cx<T> vJ[64], vI[64];
    __shared__ cx<T> cs[16][68];
    const int slot = blockIdx.y >> 1, half = blockIdx.y & 1, rhs = blockIdx.z;
    const SolveDesc& d = a.descs[slot];
    const SubDesc s = a.subs[d.sub];
    const Geometry& g = a.geo;
    const int S = s.W * s.H, nb = plane3_nb(S), ntl = nb * (nb + 1) / 2;
    const int tau = blockIdx.x;
    if (tau >= ntl) return;
    StepPlane sp;
    if (!step_plane(phase, t, half, g.Nz, s.mid, sp)) return;
    int I, J;
    tile3_ij(tau, nb, I, J);
    const int tid = threadIdx.x;
    // the tile: 8 contiguous runs of 512 entries, two per lane in each
    const cx<T>* Gt = reinterpret_cast<const cx<T>*>(a.G) + s.gs_off + ((size_t)sp.k * ntl + tau) * 4096 + 2 * tid;
    cx<T> e[16];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        e[2 * u] = Gt[u * 512];
        e[2 * u + 1] = Gt[u * 512 + 1];
    }
    if (tid < 128) {
        const int blk = tid < 64 ? J : I, c = blk * 64 + (tid & 63);
        cx<T> val{T(0), T(0)};
        if (c < S) {
            const Box3 b = window_box(s, g);
            const double ih2 = 1.0 / (g.h * g.h);
            const cx<T>* R = reinterpret_cast<const cx<T>*>(a.rhs) + ((size_t)rhs * a.nslots + slot) * a.slot_stride;
            const cx<T>* Y = reinterpret_cast<const cx<T>*>(a.Y) + ((size_t)rhs * a.nslots + slot) * a.slot_stride;
            val = step_input<T>(phase, sp, s, g, b, ih2, R, Y, smax, c);
        }
        if (tid < 64) vJ[tid] = val;
        else vI[tid - 64] = val;
    }
    __syncthreads();
    const int i4 = tid >> 4, j4 = tid & 15;
    cx<T>* P = reinterpret_cast<cx<T>*>(a.P3) +
               ((((size_t)rhs * a.nslots + slot) * 2 + half) * a.ptiles + tau) * 128;
    cx<T> rp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        cx<T> acc{T(0), T(0)};
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = acc + e[4 * r + c] * vJ[4 * j4 + c];
        acc.re = row16_sum(acc.re);
        acc.im = row16_sum(acc.im);
        rp[r] = acc;
    }
    if (j4 == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) P[4 * i4 + r] = rp[r];
    }
    if (I != J) {   // uniform over the workgroup
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cx<T> acc{T(0), T(0)};
#pragma unroll
            for (int r = 0; r < 4; ++r) acc = acc + e[4 * r + c] * vI[4 * i4 + r];
            cs[i4][4 * j4 + c] = acc;
        }
        __syncthreads();
        if (tid < 64) {
            cx<T> acc = cs[0][tid];
#pragma unroll
            for (int r = 1; r < 16; ++r) acc = acc + cs[r][tid];
            P[64 + tid] = acc;
        }
    }
}

// Reduction part of a packed step: workgroup (block b, 2*slot + half) adds, for the 64 rows of
// block b, its nb partials: entry e < nb - b is the row partial of tile (b, b + e), entry
// e >= nb - b the column partial of tile (e - (nb - b), b).  Wave w takes the entries e = w mod 4
// (loads issued together), then wave 0 adds the four sums in order.
template <typename T>
__global__ __launch_bounds__(256) void k_red3(Chain3Args a, int smax, int phase, int t) {
    constexpr int EPW = 8;   // entries per wave and pass
    __shared__ cx<T> part[4][64];
    const int slot = blockIdx.y >> 1, half = blockIdx.y & 1, rhs = blockIdx.z;
    const SolveDesc& d = a.descs[slot];
    const SubDesc s = a.subs[d.sub];
    const Geometry& g = a.geo;
    const int S = s.W * s.H, nb = plane3_nb(S), bI = blockIdx.x;
    if (bI >= nb) return;
    StepPlane sp;
    if (!step_plane(phase, t, half, g.Nz, s.mid, sp)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const cx<T>* P = reinterpret_cast<const cx<T>*>(a.P3) + (((size_t)rhs * a.nslots + slot) * 2 + half) * a.ptiles * 128;
    const int nrow = nb - bI, diag = bI * nb - bI * (bI - 1) / 2;   // tau of tile (b, b)
    cx<T> acc{T(0), T(0)};
    for (int e0 = w; e0 < nb; e0 += 4 * EPW) {
        cx<T> v[EPW];
        // every load is unconditional, so all EPW are in flight together (guarded loads compile to
        // one branch and one wait each): an entry past nb reads the first one and is scaled by 0
#pragma unroll
        for (int u = 0; u < EPW; ++u) {
            const int e = e0 + 4 * u, I = e - nrow;
            const size_t off = e < nrow ? (size_t)(diag + e) * 128 + lane
                               : e < nb ? (size_t)(I * nb - I * (I - 1) / 2 + (bI - I)) * 128 + 64 + lane
                                        : (size_t)diag * 128 + lane;
            const T f = e < nb ? T(1) : T(0);
            const cx<T> x = P[off];
            v[u] = cx<T>{x.re * f, x.im * f};
        }
#pragma unroll
        for (int u = 0; u < EPW; ++u) acc = acc + v[u];
    }
    part[w][lane] = acc;
    __syncthreads();
    const int row = bI * 64 + lane;
    if (w == 0 && row < S) {
        const cx<T> y = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        cx<T>* out = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)rhs * a.nslots + slot) * a.slot_stride +
                     (size_t)sp.k * smax + row;
        *out = (phase == 2) ? *out - y : y;
    }
}

// Packing: entry o of subdomain blockIdx.y's packed pool from its full FP64 plane blocks.
template <typename T>
__global__ void k_pack3(const SubDesc* subs, int Nz, const c128* G, cx<T>* Gs) {
    const SubDesc s = subs[blockIdx.y];
    const int S = s.W * s.H, nb = plane3_nb(S), ntl = nb * (nb + 1) / 2;
    const size_t per_plane = (size_t)ntl * 4096;
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= per_plane * Nz) return;
    const size_t k = o / per_plane, rem = o - k * per_plane;
    const int tau = (int)(rem >> 12), e = (int)(rem & 4095);
    const int u = e >> 9, w = e & 511, l = w >> 1, q = 2 * u + (w & 1);
    int I, J;
    tile3_ij(tau, nb, I, J);
    const int row = I * 64 + 4 * (l >> 4) + (q >> 2), col = J * 64 + 4 * (l & 15) + (q & 3);
    c128 v = mk(0.0, 0.0);
    if (row < S && col < S) {
        const c128* Gk = G + s.g_off + k * (size_t)S * S;   // column-major
        const c128 x = Gk[(size_t)col * S + row], y = Gk[(size_t)row * S + col];
        v = mk(0.5 * (x.re + y.re), 0.5 * (x.im + y.im));
    }
    Gs[s.gs_off + o] = cvt<T>(v);
}

template <typename T>
__global__ void k_epi3(Chain3Args a, int smax) {
    const SolveDesc& d = a.descs[blockIdx.y];
    const SubDesc s = a.subs[d.sub];
    const Geometry& g = a.geo;
    const int rhs = blockIdx.z, S = s.W * s.H, Nz = g.Nz;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)Nz * smax) return;
    const int z = (int)(idx / smax), p = (int)(idx % smax);
    if (p >= S) return;
    const int y = p / s.W, x = p - y * s.W;
    const cx<T> val = reinterpret_cast<const cx<T>*>(a.Y)[((size_t)rhs * a.nslots + blockIdx.y) * a.slot_stride + idx];
    if (d.zpart >= 0 && y >= s.r0 && y < s.r1 && x >= s.c0 && x < s.c1) {
        cx<T>* zp = reinterpret_cast<cx<T>*>(a.zpart) + (size_t)d.zpart * a.zpart_stride;
        const size_t N = (size_t)g.Nx * g.Ny * Nz;
        zp[(size_t)rhs * N + ((size_t)z * g.Ny + s.wy0 + y) * g.Nx + s.wx0 + x] = val;
    }
    cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
    for (int o = 0; o < d.nout; ++o) {
        const int side = d.out_side[o];
        long long e = -1;
        if (side == SIDE_B || side == SIDE_T) {
            const int l0 = side == SIDE_B ? s.r0 - 1 : s.r1 - 1;
            if (y == l0 || y == l0 + 1) e = ((long long)(y - l0) * Nz + z) * s.W + x;
        } else {
            const int l0 = side == SIDE_L ? s.c0 - 1 : s.c1 - 1;
            if (x == l0 || x == l0 + 1) e = ((long long)(x - l0) * Nz + z) * s.H + y;
        }
        if (e < 0) continue;
        cx<T>* out = tr + d.out_off[o] + e;
        *out = d.out_acc[o] ? *out + val : val;
    }
}

template <typename T>
__global__ void k_zsum3(const cx<T>* zpart, size_t stride, c128* z, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    c128 acc = mk(0.0, 0.0);
    for (int k = 0; k < 9; ++k) acc = acc + cvt<double>(zpart[(size_t)k * stride + i]);
    z[i] = acc;
}

__global__ void k_matvec3(Geometry g, const c128* X, c128* Y, const c128* B) {
    const size_t N = (size_t)g.Nx * g.Ny * g.Nz;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int rhs = blockIdx.y;
    const int x = (int)(p % g.Nx), y = (int)((p / g.Nx) % g.Ny), z = (int)(p / ((size_t)g.Nx * g.Ny));
    const double ih2 = 1.0 / (g.h * g.h);
    const Box3 b{g.gtx, g.Nx, g.gty, g.Ny, g.gtz, g.Nz};
    const c128* Xr = X + (size_t)rhs * N;
    const size_t sy = g.Nx, sz = (size_t)g.Nx * g.Ny;
    c128 acc = d3(g.tab, b, x, y, z, ih2, g.omega * g.omega * g.m[p]) * Xr[p];
    if (x > 0) acc = acc + c3x(g.tab, b, x - 1, y, z, ih2) * Xr[p - 1];
    if (x + 1 < g.Nx) acc = acc + c3x(g.tab, b, x, y, z, ih2) * Xr[p + 1];
    if (y > 0) acc = acc + c3y(g.tab, b, x, y - 1, z, ih2) * Xr[p - sy];
    if (y + 1 < g.Ny) acc = acc + c3y(g.tab, b, x, y, z, ih2) * Xr[p + sy];
    if (z > 0) acc = acc + c3z(g.tab, b, x, y, z - 1, ih2) * Xr[p - sz];
    if (z + 1 < g.Nz) acc = acc + c3z(g.tab, b, x, y, z, ih2) * Xr[p + sz];
    Y[(size_t)rhs * N + p] = B ? B[(size_t)rhs * N + p] - acc : acc;
}

inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_fact3_build(const Fact3Args& a, int nbatch, hipStream_t st) {
    k_f3_build<<<dim3(nblk((size_t)a.n * a.n, 256), nbatch), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_fact2_build(const Fact3Args& a, int nbatch, hipStream_t st) {
    k_f2_build<<<dim3(nblk((size_t)a.n * a.n, 256), nbatch), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_fact3_panel(const Fact3Args& a, int nbatch, int p0, int b, hipStream_t st) {
    if (b > 32 || a.n > 4096) return hipErrorInvalidValue;
    if (a.n <= 256) {
        const size_t lds = sizeof(c128) * (size_t)(b + 1) * a.n;
        hipError_t e = hipFuncSetAttribute((const void*)k_f3_panel_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        k_f3_panel_lds<<<nbatch, 1024, lds, st>>>(a, p0, b);
    } else if (a.n <= 1024) k_f3_panel<1><<<nbatch, 1024, 0, st>>>(a, p0, b);
    else if (a.n <= 2048) k_f3_panel<2><<<nbatch, 1024, 0, st>>>(a, p0, b);
    else k_f3_panel<4><<<nbatch, 1024, 0, st>>>(a, p0, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_f3_laswp<<<dim3((a.n + 255) / 256, nbatch), 256, 0, st>>>(a, p0, b);
    return hipGetLastError();
}

hipError_t launch_fact3_prep(const Fact3Args& a, int nbatch, int p0, int b, c128* Pbar, c128* T, hipStream_t st) {
    k_f3_prep<<<dim3(nblk((size_t)a.n * b, 256), nbatch), 256, 0, st>>>(a, p0, b, Pbar, T);
    return hipGetLastError();
}

hipError_t launch_fact3_update(const c128* P, const c128* T, c128* W, int n, int b, int j0, int c0, int m,
                               int nbatch, hipStream_t st) {
    if (m <= 0 || b <= 0) return hipSuccess;
    if (b > 32) return hipErrorInvalidValue;   // one pass of at most 32 columns of k
    const size_t tiles = (size_t)((n + 63) / 64) * ((m + 63) / 64) * nbatch;
    if (tiles > 0x7fffffffu) return hipErrorInvalidValue;
    k_f3_update<<<(unsigned)tiles, 256, 0, st>>>(P, T, W, n, b, j0, c0, m);
    return hipGetLastError();
}

hipError_t launch_fact3_finish(const Fact3Args& a, int nbatch, int* src, hipStream_t st) {
    k_f3_perm<<<nbatch, 64, 0, st>>>(a, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)std::min<size_t>(1024, ((size_t)a.n * a.n + 255) / 256);
    k_f3_finish<<<dim3(blocks, nbatch), 256, 0, st>>>(a, src);
    return hipGetLastError();
}

hipError_t launch_rhs3(const Chain3Args& a, int smax, int nrhs, bool f32, hipStream_t st) {
    dim3 grid(nblk((size_t)a.geo.Nz * smax, 256), a.nslots, nrhs);
    if (f32) k_rhs3<float><<<grid, 256, 0, st>>>(a, smax);
    else k_rhs3<double><<<grid, 256, 0, st>>>(a, smax);
    return hipGetLastError();
}

hipError_t launch_step3(const Chain3Args& a, int smax, int nrhs, int phase, int t, bool f32, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
    dim3 grid(nblk((size_t)smax, 64), 2 * a.nslots, nrhs);
    const size_t lds = (f32 ? sizeof(c64) : sizeof(c128)) * (size_t)smax;
    hipError_t e = hipFuncSetAttribute(f32 ? (const void*)k_step3<float> : (const void*)k_step3<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (e0 && (e = hipEventRecord(e0, st)) != hipSuccess) return e;
    if (f32) k_step3<float><<<grid, 1024, lds, st>>>(a, smax, phase, t);
    else k_step3<double><<<grid, 1024, lds, st>>>(a, smax, phase, t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (e1 && (e = hipEventRecord(e1, st)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_step3_packed(const Chain3Args& a, int smax, int nrhs, int phase, int t, bool f32, hipStream_t st,
                               hipEvent_t e0, hipEvent_t e1) {
    const dim3 tg(a.ptiles, 2 * a.nslots, nrhs), rg(plane3_nb(smax), 2 * a.nslots, nrhs);
    hipError_t e;
    if (e0 && (e = hipEventRecord(e0, st)) != hipSuccess) return e;
    if (f32) k_tile3<float><<<tg, 256, 0, st>>>(a, smax, phase, t);
    else k_tile3<double><<<tg, 256, 0, st>>>(a, smax, phase, t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (e1 && (e = hipEventRecord(e1, st)) != hipSuccess) return e;
    if (f32) k_red3<float><<<rg, 256, 0, st>>>(a, smax, phase, t);
    else k_red3<double><<<rg, 256, 0, st>>>(a, smax, phase, t);
    return hipGetLastError();
}

hipError_t launch_pack3(const SubDesc* subs, int nsub, int Nz, const c128* G, void* Gs, size_t maxper, bool f32,
                        hipStream_t st) {
    const dim3 grid(nblk(maxper, 256), nsub);
    if (f32) k_pack3<float><<<grid, 256, 0, st>>>(subs, Nz, G, reinterpret_cast<c64*>(Gs));
    else k_pack3<double><<<grid, 256, 0, st>>>(subs, Nz, G, reinterpret_cast<c128*>(Gs));
    return hipGetLastError();
}

hipError_t launch_epi3(const Chain3Args& a, int smax, int nrhs, bool f32, hipStream_t st) {
    dim3 grid(nblk((size_t)a.geo.Nz * smax, 256), a.nslots, nrhs);
    if (f32) k_epi3<float><<<grid, 256, 0, st>>>(a, smax);
    else k_epi3<double><<<grid, 256, 0, st>>>(a, smax);
    return hipGetLastError();
}

hipError_t launch_zsum3(const void* zpart, size_t stride, c128* z, size_t n, bool f32, hipStream_t st) {
    if (f32) k_zsum3<float><<<nblk(n, 256), 256, 0, st>>>(reinterpret_cast<const c64*>(zpart), stride, z, n);
    else k_zsum3<double><<<nblk(n, 256), 256, 0, st>>>(reinterpret_cast<const c128*>(zpart), stride, z, n);
    return hipGetLastError();
}

hipError_t launch_matvec3(const Geometry& g, const c128* x, c128* y, const c128* b, int nrhs, hipStream_t st) {
    const size_t N = (size_t)g.Nx * g.Ny * g.Nz;
    k_matvec3<<<dim3(nblk(N, 256), nrhs), 256, 0, st>>>(g, x, y, b);
    return hipGetLastError();
}

}  // namespace lsw
