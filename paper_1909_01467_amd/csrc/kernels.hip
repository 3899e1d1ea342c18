// HIP kernels of the L-sweeps library (gfx950).
//
//  k_factor   batched block-tridiagonal LU of every local problem (Phase 2, Sec. 3):
//             S_0 = D_0, G_k = S_k^-1, S_{k+1} = D_{k+1} - C_k G_k C_k, one workgroup per
//             subdomain, the W x W block held in LDS and inverted by Gauss-Jordan with
//             partial pivoting in FP64; G_k stored column-major in complex64/complex128.
//  k_sweep    one sweep front: a batch of independent local solves A_ij U = g.  The
//             right-hand side g = A(chi u~) - chi(A u~) of eq. DiscPol2 is formed on the
//             fly from the incoming traces (fused prologue), the block forward/back
//             substitution streams G_k from HBM, and the epilogue writes U on Omega_ij to
//             the sweep's accumulator and the outgoing 2-line traces (fused epilogue).
//  k_zsum     z on Omega_ij = sum of the per-sweep contributions (end of Alg. Scenario3).
//  k_matvec   y = A x, FP64, 5-point stencil with coefficients evaluated from the 1-D
//             PML tables (App. A).
//  Krylov     batched dot products, AXPY-type updates and norms for FGMRES (FP64).
#include "launch.h"

namespace lsw {

// ------------------------------------------------------------------ coefficients
// Couplings of the 5-point symmetric PML operator on a box whose x table starts at tx
// (Px points) and y table at ty (Py points); see the table layout in common.h.
__device__ inline c128 coup_x(const c128* tab, int tx, int Px, int ty, int a, int b, double ih2) {
    // -(s1 at (a+1/2, b))/h^2 ;  s1 = alpha_x(half) / alpha_y(int)
    return -ih2 * (tab[tx + Px + a + 1] * tab[ty + b]);
}
__device__ inline c128 coup_y(const c128* tab, int tx, int ty, int Py, int a, int b, double ih2) {
    // -(s2 at (a, b+1/2))/h^2 ;  s2 = alpha_y(half) / alpha_x(int)
    return -ih2 * (tab[ty + Py + b + 1] * tab[tx + a]);
}
__device__ inline c128 diag_coef(const c128* tab, int tx, int Px, int ty, int Py, int a, int b,
                                 double ih2, double om2m) {
    c128 sx = tab[tx + Px + a + 1] + tab[tx + Px + a];
    c128 sy = tab[ty + Py + b + 1] + tab[ty + Py + b];
    c128 d = ih2 * (sx * tab[ty + b] + sy * tab[tx + a]);
    return d - om2m * (tab[tx + a] * tab[ty + b]);
}

// ------------------------------------------------------------------ K3: factorisation
template <int NT, bool kLds, typename TG>
__global__ __launch_bounds__(NT) void k_factor(FactorArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ c128 colp[kMaxWindow];
    __shared__ int perm[kMaxWindow];
    __shared__ int sh_piv, sh_sing;
    const SubDesc s = a.subs[blockIdx.x];
    const int W = s.W, H = s.H, tid = threadIdx.x;
    constexpr int NTX = 32, NTY = NT / 32;
    const int tx = tid % NTX, ty = tid / NTX;
    c128* S = kLds ? reinterpret_cast<c128*>(smem) : a.work + (size_t)blockIdx.x * a.work_stride;
    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h), om2 = a.geo.omega * a.geo.omega;
    TG* G = reinterpret_cast<TG*>(a.G) + s.g_off;
    if (tid == 0) sh_sing = 0;

    for (int k = 0; k < H; ++k) {
        // couplings to the previous block row, C_{k-1} (diagonal)
        if (k > 0)
            for (int x = tid; x < W; x += NT) colp[x] = coup_y(tab, s.tx, s.ty, H, x, k - 1, ih2);
        __syncthreads();
        // S_k = D_k - C_{k-1} G_{k-1} C_{k-1}; G_{k-1} is the current content of S
        const double* mrow = a.geo.m + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0;
        for (int r = ty; r < W; r += NTY) {
            for (int c = tx; c < W; c += NTX) {
                c128 val = mk(0.0, 0.0);
                if (r == c) val = diag_coef(tab, s.tx, W, s.ty, H, c, k, ih2, om2 * mrow[c]);
                else if (c == r + 1) val = coup_x(tab, s.tx, W, s.ty, r, k, ih2);
                else if (r == c + 1) val = coup_x(tab, s.tx, W, s.ty, c, k, ih2);
                if (k > 0) val = val - colp[r] * S[r * W + c] * colp[c];
                S[r * W + c] = val;
            }
        }
        __syncthreads();
        // in-place Gauss-Jordan inversion with row pivoting
        for (int p = 0; p < W; ++p) {
            if (tid < 64) {
                double best = -1.0;
                int bi = p;
                for (int r = p + tid; r < W; r += 64) {
                    double v = abs2(S[r * W + p]);
                    if (v > best) { best = v; bi = r; }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    double ob = __shfl_xor(best, off);
                    int oi = __shfl_xor(bi, off);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (tid == 0) {
                    sh_piv = bi;
                    perm[p] = bi;
                    if (!(best > 0.0)) sh_sing = 1;
                }
            }
            __syncthreads();
            const int piv = sh_piv;
            if (piv != p)
                for (int c = tid; c < W; c += NT) {
                    c128 t = S[p * W + c];
                    S[p * W + c] = S[piv * W + c];
                    S[piv * W + c] = t;
                }
            __syncthreads();
            const c128 inv = cinv(S[p * W + p]);
            for (int r = tid; r < W; r += NT) colp[r] = S[r * W + p];
            __syncthreads();
            for (int c = tid; c < W; c += NT) S[p * W + c] = (c == p) ? inv : S[p * W + c] * inv;
            __syncthreads();
            for (int r = ty; r < W; r += NTY) {
                if (r == p) continue;
                const c128 f = colp[r];
                for (int c = tx; c < W; c += NTX) {
                    if (c == p) S[r * W + c] = -(f * inv);
                    else S[r * W + c] = S[r * W + c] - f * S[p * W + c];
                }
            }
            __syncthreads();
        }
        // undo the row interchanges as column interchanges, in reverse order
        for (int p = W - 1; p >= 0; --p) {
            const int pv = perm[p];
            if (pv != p)
                for (int r = tid; r < W; r += NT) {
                    c128 t = S[r * W + p];
                    S[r * W + p] = S[r * W + pv];
                    S[r * W + pv] = t;
                }
            __syncthreads();
        }
        // G_k, column-major: G[c*W + t] = (S_k^-1)[t][c]
        TG* Gk = G + (size_t)k * W * W;
        for (int c = ty; c < W; c += NTY)
            for (int t = tx; t < W; t += NTX) {
                c128 v = S[t * W + c];
                Gk[(size_t)c * W + t] = TG{static_cast<decltype(TG::re)>(v.re),
                                           static_cast<decltype(TG::re)>(v.im)};
            }
        __syncthreads();
    }
    if (tid == 0 && sh_sing) a.status[blockIdx.x] = 1;
}

// ------------------------------------------------------------------ K4/K5: one sweep front
template <typename T>
struct Local {
    const SubDesc& s;
    const SolveDesc& d;
    const c128* tab;
    const cx<T>* in_h;
    const cx<T>* in_v;
    double ih2;
};

__device__ inline bool chi_of(int kind, int k, int c, const SubDesc& s) {
    switch (kind) {
        case KIND_B: return k >= s.r0;
        case KIND_T: return k < s.r1;
        case KIND_L: return c >= s.c0;
        case KIND_R: return c < s.c1;
        case KIND_BL: return k >= s.r0 && c >= s.c0;
        case KIND_TR: return k < s.r1 && c < s.c1;
        case KIND_BR: return k >= s.r0 && c < s.c1;
        case KIND_TL: return k < s.r1 && c >= s.c0;
        default: return false;
    }
}

// incoming trace value u~ at window point (k, c); 0 off the legs
template <typename T>
__device__ inline cx<T> utilde(const Local<T>& L, int k, int c) {
    const SubDesc& s = L.s;
    const int kind = L.d.kind;
    const bool corner = kind >= KIND_BL;
    const bool hB = (kind == KIND_B || kind == KIND_BL || kind == KIND_BR);
    const bool hT = (kind == KIND_T || kind == KIND_TR || kind == KIND_TL);
    const bool vL = (kind == KIND_L || kind == KIND_BL || kind == KIND_TL);
    const bool vR = (kind == KIND_R || kind == KIND_TR || kind == KIND_BR);
    if (hB || hT) {
        const int l0 = hB ? s.r0 - 1 : s.r1 - 1;
        const bool in_cols = !corner || (vL ? c >= s.c0 : c < s.c1);
        if ((k == l0 || k == l0 + 1) && in_cols) return L.in_h[(k - l0) * s.W + c];
    }
    if (vL || vR) {
        const int l0 = vL ? s.c0 - 1 : s.c1 - 1;
        const bool in_rows = !corner || (hB ? k >= s.r0 : k < s.r1);
        if ((c == l0 || c == l0 + 1) && in_rows) return L.in_v[(c - l0) * s.H + k];
    }
    return cx<T>{T(0), T(0)};
}

// g at (k, c): sum over the 4 neighbours q across the boundary of chi of A_pq (chi_q - chi_p) u~_q
template <typename T>
__device__ inline cx<T> g_polarized(const Local<T>& L, int k, int c) {
    const SubDesc& s = L.s;
    const int kind = L.d.kind;
    const bool has_v = !(kind == KIND_B || kind == KIND_T);
    if (!has_v) {  // straight horizontal interface: only its two lines carry g
        const int l0 = (kind == KIND_B) ? s.r0 - 1 : s.r1 - 1;
        if (k != l0 && k != l0 + 1) return cx<T>{T(0), T(0)};
    }
    const bool cp = chi_of(kind, k, c, s);
    c128 g = mk(0.0, 0.0);
    const int W = s.W, H = s.H;
    if (c > 0 && chi_of(kind, k, c - 1, s) != cp) {
        c128 A = coup_x(L.tab, s.tx, W, s.ty, c - 1, k, L.ih2);
        c128 u = cvt<double>(utilde(L, k, c - 1));
        g = cp ? g - A * u : g + A * u;
    }
    if (c + 1 < W && chi_of(kind, k, c + 1, s) != cp) {
        c128 A = coup_x(L.tab, s.tx, W, s.ty, c, k, L.ih2);
        c128 u = cvt<double>(utilde(L, k, c + 1));
        g = cp ? g - A * u : g + A * u;
    }
    if (k > 0 && chi_of(kind, k - 1, c, s) != cp) {
        c128 A = coup_y(L.tab, s.tx, s.ty, H, c, k - 1, L.ih2);
        c128 u = cvt<double>(utilde(L, k - 1, c));
        g = cp ? g - A * u : g + A * u;
    }
    if (k + 1 < H && chi_of(kind, k + 1, c, s) != cp) {
        c128 A = coup_y(L.tab, s.tx, s.ty, H, c, k, L.ih2);
        c128 u = cvt<double>(utilde(L, k + 1, c));
        g = cp ? g - A * u : g + A * u;
    }
    return cvt<T>(g);
}

template <typename T, int RC>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
    constexpr int NT = 256, NW = NT / 64, WM = 64 * RC;
    const SolveDesc d = a.descs[blockIdx.x];
    const SubDesc s = a.subs[d.sub];
    const int rhs = blockIdx.y;
    const int W = s.W, H = s.H, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ cx<T> v[WM], xk[WM];
    __shared__ cx<T> part[NW][WM];

    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    const cx<T>* Gs = reinterpret_cast<const cx<T>*>(a.G) + s.g_off;
    cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
    cx<T>* Y = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * a.Y_stride;
    cx<T>* z = reinterpret_cast<cx<T>*>(a.zpart) + (size_t)d.zpart * a.zpart_stride +
               (size_t)rhs * a.geo.Nx * a.geo.Ny;
    const c128* rin = a.r + (size_t)rhs * a.geo.Nx * a.geo.Ny;
    Local<T> L{s, d, tab, d.in_h >= 0 ? tr + d.in_h : nullptr, d.in_v >= 0 ? tr + d.in_v : nullptr, ih2};

    // ---- forward substitution: y_k = G_k (g_k - C_{k-1} y_{k-1})
    for (int k = d.kf0; k < H; ++k) {
        for (int c = tid; c < W; c += NT) {
            cx<T> g;
            if (d.kind == KIND_STAGE1) {
                const bool in = (k >= s.r0 && k < s.r1 && c >= s.c0 && c < s.c1);
                g = in ? cvt<T>(rin[(size_t)(s.wy0 + k) * a.geo.Nx + s.wx0 + c]) : cx<T>{T(0), T(0)};
            } else {
                g = g_polarized(L, k, c);
            }
            if (k > d.kf0) g = g - cvt<T>(coup_y(tab, s.tx, s.ty, H, c, k - 1, ih2)) * xk[c];
            v[c] = g;
        }
        __syncthreads();
        const cx<T>* Gk = Gs + (size_t)k * W * W;
        cx<T> acc[RC];
#pragma unroll
        for (int q = 0; q < RC; ++q) acc[q] = cx<T>{T(0), T(0)};
#pragma unroll 4
        for (int c = wv; c < W; c += NW) {
            const cx<T> vc = v[c];
            const cx<T>* col = Gk + (size_t)c * W;
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int t = lane + 64 * q;
                if (t < W) acc[q] = fma(acc[q], col[t], vc);
            }
        }
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int t = lane + 64 * q;
            if (t < W) part[wv][t] = acc[q];
        }
        __syncthreads();
        for (int t = tid; t < W; t += NT) {
            cx<T> y = part[0][t];
#pragma unroll
            for (int w = 1; w < NW; ++w) y = y + part[w][t];
            xk[t] = y;
            Y[(size_t)k * W + t] = y;
        }
        __syncthreads();
    }

    // ---- backward substitution: x_k = y_k - G_k C_k x_{k+1}; xk holds x_{H-1} = y_{H-1}
    for (int k = H - 1; k >= d.kb0; --k) {
        if (k < H - 1) {
            for (int c = tid; c < W; c += NT) v[c] = cvt<T>(coup_y(tab, s.tx, s.ty, H, c, k, ih2)) * xk[c];
            __syncthreads();
            const cx<T>* Gk = Gs + (size_t)k * W * W;
            cx<T> acc[RC];
#pragma unroll
            for (int q = 0; q < RC; ++q) acc[q] = cx<T>{T(0), T(0)};
#pragma unroll 4
            for (int c = wv; c < W; c += NW) {
                const cx<T> vc = v[c];
                const cx<T>* col = Gk + (size_t)c * W;
#pragma unroll
                for (int q = 0; q < RC; ++q) {
                    const int t = lane + 64 * q;
                    if (t < W) acc[q] = fma(acc[q], col[t], vc);
                }
            }
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int t = lane + 64 * q;
                if (t < W) part[wv][t] = acc[q];
            }
            __syncthreads();
            for (int t = tid; t < W; t += NT) {
                cx<T> y = (k >= d.kf0) ? Y[(size_t)k * W + t] : cx<T>{T(0), T(0)};
#pragma unroll
                for (int w = 0; w < NW; ++w) y = y - part[w][t];
                xk[t] = y;
            }
            __syncthreads();
        }
        // ---- epilogue for block row k
        if (k >= s.r0 && k < s.r1) {
            cx<T>* zrow = z + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0;
            for (int c = s.c0 + tid; c < s.c1; c += NT) zrow[c] = xk[c];
        }
        for (int o = 0; o < d.nout; ++o) {
            const int side = d.out_side[o];
            cx<T>* out = tr + d.out_off[o];
            const bool acc = d.out_acc[o] != 0;
            if (side == SIDE_B || side == SIDE_T) {
                const int l0 = (side == SIDE_B) ? s.r0 - 1 : s.r1 - 1;
                if (k == l0 || k == l0 + 1) {
                    cx<T>* line = out + (size_t)(k - l0) * W;
                    for (int c = tid; c < W; c += NT) line[c] = acc ? line[c] + xk[c] : xk[c];
                }
            } else {
                const int l0 = (side == SIDE_L) ? s.c0 - 1 : s.c1 - 1;
                if (tid < 2) {
                    cx<T>* p = out + (size_t)tid * H + k;
                    *p = acc ? *p + xk[l0 + tid] : xk[l0 + tid];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ z assembly
template <typename T>
__global__ void k_zsum(ZsumArgs a) {
    const size_t N = (size_t)a.Nx * a.Ny;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int rhs = blockIdx.y;
    const int x = (int)(p % a.Nx), y = (int)(p / a.Nx);
    const int j = a.xgroup[x], i = a.ygroup[y];
    const int q = a.q, r = a.r;
    const bool vis[9] = {true,   i >= 1,         i <= q - 2,         j >= 1,         j <= r - 2,
                         i >= 1 && j >= 1, i <= q - 2 && j <= r - 2, i >= 1 && j <= r - 2,
                         i <= q - 2 && j >= 1};
    const cx<T>* zp = reinterpret_cast<const cx<T>*>(a.zpart) + (size_t)rhs * N + p;
    c128 acc = mk(0.0, 0.0);
#pragma unroll
    for (int sw = 0; sw < 9; ++sw)
        if (vis[sw]) acc = acc + cvt<double>(zp[(size_t)sw * a.zpart_stride]);
    a.z[(size_t)rhs * N + p] = acc;
}

// ------------------------------------------------------------------ K6: y = A x (FP64)
__global__ void k_matvec(MatvecArgs a) {
    const Geometry& g = a.geo;
    const size_t N = (size_t)g.Nx * g.Ny;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int rhs = blockIdx.y;
    const int x = (int)(p % g.Nx), y = (int)(p / g.Nx);
    const double ih2 = 1.0 / (g.h * g.h);
    const c128* X = a.x + (size_t)rhs * N;
    const c128* tab = g.tab;
    c128 acc = diag_coef(tab, g.gtx, g.Nx, g.gty, g.Ny, x, y, ih2, g.omega * g.omega * g.m[p]) * X[p];
    if (x > 0) acc = acc + coup_x(tab, g.gtx, g.Nx, g.gty, x - 1, y, ih2) * X[p - 1];
    if (x + 1 < g.Nx) acc = acc + coup_x(tab, g.gtx, g.Nx, g.gty, x, y, ih2) * X[p + 1];
    if (y > 0) acc = acc + coup_y(tab, g.gtx, g.gty, g.Ny, x, y - 1, ih2) * X[p - g.Nx];
    if (y + 1 < g.Ny) acc = acc + coup_y(tab, g.gtx, g.gty, g.Ny, x, y, ih2) * X[p + g.Nx];
    c128 out = acc;
    if (a.b) out = a.b[(size_t)rhs * N + p] - acc;   // residual mode: r = b - A x
    a.y[(size_t)rhs * N + p] = out;
}

// ------------------------------------------------------------------ K7: Krylov BLAS (FP64)
// partial[(rhs * nv + l) * nblk + blk] = sum over the block's points of conj(V_l) w
__global__ void k_dots_partial(DotsArgs a) {
    __shared__ c128 red[256];
    const int blk = blockIdx.x, l = blockIdx.y, rhs = blockIdx.z;
    const c128* V = a.V + ((size_t)l * a.vstride_l + (size_t)rhs * a.vstride_rhs);
    const c128* w = a.w + (size_t)rhs * a.wstride;
    c128 acc = mk(0.0, 0.0);
    for (size_t p = (size_t)blk * blockDim.x + threadIdx.x; p < a.N; p += (size_t)gridDim.x * blockDim.x)
        acc = acc + conj(V[p]) * w[p];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[((size_t)rhs * a.nv + l) * gridDim.x + blk] = red[0];
}

// out[rhs * ostride + l] (+)= sum_blk partial ; one thread per (l, rhs)
__global__ void k_dots_finish(const c128* partial, int nblk, int nv, int nrhs, c128* out, int ostride,
                              int accumulate) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nv * nrhs) return;
    const int rhs = idx / nv, l = idx % nv;
    c128 acc = mk(0.0, 0.0);
    const c128* pp = partial + ((size_t)rhs * nv + l) * nblk;
    for (int b = 0; b < nblk; ++b) acc = acc + pp[b];
    c128* o = out + (size_t)rhs * ostride + l;
    *o = accumulate ? *o + acc : acc;
}

// w -= sum_l V_l c_l   (c = coefficients on the device, [rhs * cstride + l]); masked rhs skipped
__global__ void k_gs_update(GsArgs a) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (p >= a.N || (a.active && !a.active[rhs])) return;
    const c128* cf = a.coef + (size_t)rhs * a.cstride;
    c128 acc = mk(0.0, 0.0);
    for (int l = 0; l < a.nv; ++l)
        acc = acc + a.V[(size_t)l * a.vstride_l + (size_t)rhs * a.vstride_rhs + p] * cf[l];
    c128* w = a.w + (size_t)rhs * a.wstride + p;
    *w = a.sign > 0 ? *w + acc : *w - acc;
}

// dst = src * scale[rhs]  (scale = 1/norm, computed on the host), masked rhs skipped
__global__ void k_scale(const c128* src, c128* dst, const double* scale, const int* active, size_t N,
                        size_t sstride, size_t dstride) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (p >= N || (active && !active[rhs])) return;
    const double s = scale[rhs];
    const c128 v = src[(size_t)rhs * sstride + p];
    dst[(size_t)rhs * dstride + p] = mk(s * v.re, s * v.im);
}

__global__ void k_conj(const c128* src, c128* dst, size_t n) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[p] = conj(src[p]);
}

__global__ void k_mass_gradient(const c128* lam, const c128* u, int nrhs, Geometry g, double* grad) {
    const size_t N = (size_t)g.Nx * g.Ny;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int x = (int)(p % g.Nx), y = (int)(p / g.Nx);
    const c128 w = g.tab[g.gtx + x] * g.tab[g.gty + y];   // 1/(alpha_x alpha_y)
    double acc = 0.0;
    for (int s = 0; s < nrhs; ++s) {
        const c128 t = lam[(size_t)s * N + p] * w * u[(size_t)s * N + p];
        acc += t.re;
    }
    grad[p] += g.omega * g.omega * acc;
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_factor(const FactorArgs& a, int nsub, int Wmax, bool use_lds, size_t lds_bytes,
                         bool store_c64, hipStream_t st) {
    constexpr int NT = 1024;
    if (use_lds) {
        hipError_t e;
        if (store_c64) {
            e = hipFuncSetAttribute((const void*)k_factor<NT, true, c64>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e != hipSuccess) return e;
            k_factor<NT, true, c64><<<nsub, NT, lds_bytes, st>>>(a);
        } else {
            e = hipFuncSetAttribute((const void*)k_factor<NT, true, c128>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e != hipSuccess) return e;
            k_factor<NT, true, c128><<<nsub, NT, lds_bytes, st>>>(a);
        }
    } else {
        if (store_c64) k_factor<NT, false, c64><<<nsub, NT, 0, st>>>(a);
        else k_factor<NT, false, c128><<<nsub, NT, 0, st>>>(a);
    }
    (void)Wmax;
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_sweep_t(const SweepArgs& a, int nsolves, int nrhs, int Wmax, hipStream_t st) {
    dim3 grid(nsolves, nrhs);
    if (Wmax <= 64) k_sweep<T, 1><<<grid, 256, 0, st>>>(a);
    else if (Wmax <= 128) k_sweep<T, 2><<<grid, 256, 0, st>>>(a);
    else if (Wmax <= 192) k_sweep<T, 3><<<grid, 256, 0, st>>>(a);
    else k_sweep<T, 4><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& a, int nsolves, int nrhs, int Wmax, bool c64mode, hipStream_t st) {
    return c64mode ? launch_sweep_t<float>(a, nsolves, nrhs, Wmax, st)
                   : launch_sweep_t<double>(a, nsolves, nrhs, Wmax, st);
}

hipError_t launch_zsum(const ZsumArgs& a, int nrhs, bool c64mode, hipStream_t st) {
    const size_t N = (size_t)a.Nx * a.Ny;
    dim3 grid(blocks_for(N, 256), nrhs);
    if (c64mode) k_zsum<float><<<grid, 256, 0, st>>>(a);
    else k_zsum<double><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_matvec(const MatvecArgs& a, int nrhs, hipStream_t st) {
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    dim3 grid(blocks_for(N, 256), nrhs);
    k_matvec<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_dots(const DotsArgs& a, int nrhs, c128* out, int ostride, int accumulate, hipStream_t st) {
    dim3 grid(a.nblk, a.nv, nrhs);
    k_dots_partial<<<grid, 256, 0, st>>>(a);
    const int n = a.nv * nrhs;
    k_dots_finish<<<blocks_for(n, 64), 64, 0, st>>>(a.partial, a.nblk, a.nv, nrhs, out, ostride, accumulate);
    return hipGetLastError();
}

hipError_t launch_gs_update(const GsArgs& a, int nrhs, hipStream_t st) {
    dim3 grid(blocks_for(a.N, 256), nrhs);
    k_gs_update<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_scale(const c128* src, c128* dst, const double* scale, const int* active, size_t N,
                        size_t sstride, size_t dstride, int nrhs, hipStream_t st) {
    dim3 grid(blocks_for(N, 256), nrhs);
    k_scale<<<grid, 256, 0, st>>>(src, dst, scale, active, N, sstride, dstride);
    return hipGetLastError();
}

hipError_t launch_conj(const c128* src, c128* dst, size_t n, hipStream_t st) {
    k_conj<<<blocks_for(n, 256), 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_mass_gradient(const c128* lam, const c128* u, int nrhs, const Geometry& g, double* grad,
                                hipStream_t st) {
    const size_t N = (size_t)g.Nx * g.Ny;
    k_mass_gradient<<<blocks_for(N, 256), 256, 0, st>>>(lam, u, nrhs, g, grad);
    return hipGetLastError();
}

}  // namespace lsw
