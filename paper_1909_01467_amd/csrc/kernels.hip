// HIP kernels of the L-sweeps library (gfx950).
//
//  k_factor   batched block-tridiagonal LU of every local problem (Phase 2, Sec. 3):
//             S_0 = D_0, G_k = S_k^-1, S_{k+1} = D_{k+1} - C_k G_k C_k, one workgroup per
//             subdomain, the W x W block held in LDS and inverted by Gauss-Jordan with
//             partial pivoting in FP64; G_k stored column-major in complex64/complex128.
//  k_chain    a batch of independent local solves A_ij U = g by block forward/back
//             substitution streaming G_k from HBM (stage 1, the final z solve, the unit
//             solves that build Q, and every front of the chained sweep mode).  The
//             right-hand side (restricted residual, eq. DiscPol2 polarized source, or the
//             accumulated sweep sources) is formed on the fly and the epilogue writes the
//             outgoing 2-line traces, z, or a column of Q.
//  k_gemv     one sweep front in trace-compressed form: the outgoing traces of each solve
//             are Q[out lines, in slots] * g with Q = A_ij^-1 restricted to the 8 trace
//             lines, so the front is one fully parallel batched GEMV.
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
// Geometry and incoming traces of one polarized local solve, held by value so that the
// compiler keeps everything in registers.
template <typename T>
struct Local {
    int kind, W, H, r0, r1, c0, c1, tx, ty;
    const c128* tab;
    const cx<T>* in_h;
    const cx<T>* in_v;
    double ih2;
};

template <typename T>
__device__ inline Local<T> make_local(const SubDesc& s, int kind, const c128* tab, const cx<T>* in_h,
                                      const cx<T>* in_v, double ih2) {
    return Local<T>{kind, s.W, s.H, s.r0, s.r1, s.c0, s.c1, s.tx, s.ty, tab, in_h, in_v, ih2};
}

template <typename T>
__device__ inline bool chi_of(const Local<T>& L, int k, int c) {
    switch (L.kind) {
        case KIND_B: return k >= L.r0;
        case KIND_T: return k < L.r1;
        case KIND_L: return c >= L.c0;
        case KIND_R: return c < L.c1;
        case KIND_BL: return k >= L.r0 && c >= L.c0;
        case KIND_TR: return k < L.r1 && c < L.c1;
        case KIND_BR: return k >= L.r0 && c < L.c1;
        case KIND_TL: return k < L.r1 && c >= L.c0;
        default: return false;
    }
}

// incoming trace value u~ at window point (k, c); 0 off the legs.  The legs of an L-shaped
// interface are restricted to the receiving quadrant and the horizontal leg is used on the
// point they share.
template <typename T>
__device__ inline cx<T> utilde(const Local<T>& L, int k, int c) {
    const int kind = L.kind;
    const bool corner = kind >= KIND_BL;
    const bool hB = (kind == KIND_B || kind == KIND_BL || kind == KIND_BR);
    const bool hT = (kind == KIND_T || kind == KIND_TR || kind == KIND_TL);
    const bool vL = (kind == KIND_L || kind == KIND_BL || kind == KIND_TL);
    const bool vR = (kind == KIND_R || kind == KIND_TR || kind == KIND_BR);
    if (hB || hT) {
        const int l0 = hB ? L.r0 - 1 : L.r1 - 1;
        const bool in_cols = !corner || (vL ? c >= L.c0 : c < L.c1);
        if ((k == l0 || k == l0 + 1) && in_cols) return L.in_h[(k - l0) * L.W + c];
    }
    if (vL || vR) {
        const int l0 = vL ? L.c0 - 1 : L.c1 - 1;
        const bool in_rows = !corner || (hB ? k >= L.r0 : k < L.r1);
        if ((c == l0 || c == l0 + 1) && in_rows) return L.in_v[(c - l0) * L.H + k];
    }
    return cx<T>{T(0), T(0)};
}

// g at (k, c) = (A(chi u~) - chi (A u~))(k, c): sum over the 4 neighbours q across the
// boundary of chi of A_pq (chi_q - chi_p) u~_q (eq. DiscPol2)
template <typename T>
__device__ inline cx<T> g_polarized(const Local<T>& L, int k, int c) {
    const int kind = L.kind;
    const bool has_v = !(kind == KIND_B || kind == KIND_T);
    if (!has_v) {  // straight horizontal interface: only its two lines carry g
        const int l0 = (kind == KIND_B) ? L.r0 - 1 : L.r1 - 1;
        if (k != l0 && k != l0 + 1) return cx<T>{T(0), T(0)};
    }
    const bool cp = chi_of(L, k, c);
    c128 g = mk(0.0, 0.0);
    const int W = L.W, H = L.H;
    if (c > 0 && chi_of(L, k, c - 1) != cp) {
        c128 A = coup_x(L.tab, L.tx, W, L.ty, c - 1, k, L.ih2);
        c128 u = cvt<double>(utilde(L, k, c - 1));
        g = cp ? g - A * u : g + A * u;
    }
    if (c + 1 < W && chi_of(L, k, c + 1) != cp) {
        c128 A = coup_x(L.tab, L.tx, W, L.ty, c, k, L.ih2);
        c128 u = cvt<double>(utilde(L, k, c + 1));
        g = cp ? g - A * u : g + A * u;
    }
    if (k > 0 && chi_of(L, k - 1, c) != cp) {
        c128 A = coup_y(L.tab, L.tx, L.ty, H, c, k - 1, L.ih2);
        c128 u = cvt<double>(utilde(L, k - 1, c));
        g = cp ? g - A * u : g + A * u;
    }
    if (k + 1 < H && chi_of(L, k + 1, c) != cp) {
        c128 A = coup_y(L.tab, L.tx, L.ty, H, c, k, L.ih2);
        c128 u = cvt<double>(utilde(L, k + 1, c));
        g = cp ? g - A * u : g + A * u;
    }
    return cvt<T>(g);
}

// right-hand side of a block row element (k, c) for the kinds that are not polarized
template <typename T>
__device__ inline cx<T> rhs_plain(const ChainArgs& a, const SolveDesc& d, const SubDesc& s, int rhs, int k, int c) {
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    if (d.kind == KIND_UNIT) return (k == d.unit_k && c == d.unit_c) ? cx<T>{T(1), T(0)} : cx<T>{T(0), T(0)};
    c128 g = mk(0.0, 0.0);
    if (k >= s.r0 && k < s.r1 && c >= s.c0 && c < s.c1)
        g = a.r[(size_t)rhs * N + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0 + c];
    cx<T> out = cvt<T>(g);
    if (d.kind == KIND_FINAL) {
        // sum of the sweeps' right-hand sides g_s (each supported on the trace-line slots)
        const int W = s.W, H = s.H;
        const cx<T>* gp = reinterpret_cast<const cx<T>*>(a.gparts) + (size_t)rhs * 8 * a.LT + s.gp_off;
        for (int sw = 0; sw < 8; ++sw, gp += a.LT) {
            if (k == s.r0 - 1) out = out + gp[c];
            if (k == s.r0) out = out + gp[W + c];
            if (k == s.r1 - 1) out = out + gp[2 * W + c];
            if (k == s.r1 && k < H) out = out + gp[3 * W + c];
            if (c == s.c0 - 1) out = out + gp[4 * W + k];
            if (c == s.c0) out = out + gp[4 * W + H + k];
            if (c == s.c1 - 1) out = out + gp[4 * W + 2 * H + k];
            if (c == s.c1 && c < W) out = out + gp[4 * W + 3 * H + k];
        }
    }
    return out;
}

// Batched block forward/back substitution, one workgroup per (local solve, rhs).
// Thread tid < NA = floor(1024/W)*W owns block row t = tid % W and the columns
// c = tid / W + NG*j (j < ept) of every W x W block G_k: its elements sit at the flat
// offsets tid + NA*j of the column-major block, so the loads are fully coalesced.  A ring
// of PD+1 register buffers keeps PD blocks in flight ahead of the current one.
template <typename T, int EPT, int PD, bool POLAR>
__global__ __launch_bounds__(1024) void k_chain(ChainArgs a) {
    constexpr int NT = 1024;
    const SolveDesc& d = a.descs[blockIdx.x];
    const SubDesc s = a.subs[d.sub];
    const int rhs = blockIdx.y;
    const int W = s.W, H = s.H, tid = threadIdx.x;
    const int NG = NT / W, NA = NG * W;
    const bool act = tid < NA;
    const int cg = act ? tid / W : 0;
    const int ept = (W + NG - 1) / NG;
    const int WW = W * W;
    __shared__ cx<T> v[kMaxWindow], xk[kMaxWindow];
    __shared__ cx<T> part[NT];

    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    const cx<T>* Gs = reinterpret_cast<const cx<T>*>(a.G) + s.g_off;
    cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
    cx<T>* Y = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * a.Y_stride;
    const bool polar = d.kind >= KIND_B && d.kind <= KIND_TL;
    const Local<T> L = make_local<T>(s, d.kind, tab, d.in_h >= 0 ? tr + d.in_h : nullptr,
                                     d.in_v >= 0 ? tr + d.in_v : nullptr, ih2);
    const cx<T> zero{T(0), T(0)};

    auto load = [&](int k, cx<T>* buf) {
        const cx<T>* Gk = Gs + (size_t)k * WW;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + NA * j;
            buf[j] = (act && j < ept && e < WW) ? Gk[e] : zero;
        }
    };
    // part[tid] = sum_j G_k[c_j][t] vin[c_j]
    auto gemv = [&](const cx<T>* buf) {
        cx<T> acc = zero;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int c = cg + NG * j;
            if (j < ept && c < W) acc = fma(acc, buf[j], v[c]);
        }
        if (act) part[tid] = acc;
    };
    auto reduce = [&](int t) {
        cx<T> y = part[t];
        for (int g = 1; g < NG; ++g) y = y + part[g * W + t];
        return y;
    };

    cx<T> ring[PD + 1][EPT];
    // ---- forward substitution: y_k = G_k (g_k - C_{k-1} y_{k-1})
    auto fwd = [&](int k, const cx<T>* buf) {
        if (tid < W) {
            cx<T> g;
            if constexpr (POLAR) g = polar ? g_polarized(L, k, tid) : rhs_plain<T>(a, d, s, rhs, k, tid);
            else g = rhs_plain<T>(a, d, s, rhs, k, tid);
            if (k > d.kf0) g = g - cvt<T>(coup_y(tab, s.tx, s.ty, H, tid, k - 1, ih2)) * xk[tid];
            v[tid] = g;
        }
        __syncthreads();
        gemv(buf);
        __syncthreads();
        if (tid < W) {
            const cx<T> y = reduce(tid);
            xk[tid] = y;
            Y[(size_t)k * W + tid] = y;
        }
        __syncthreads();
    };
#pragma unroll
    for (int p = 0; p < PD; ++p)
        if (d.kf0 + p < H) load(d.kf0 + p, ring[p]);
    for (int k0 = d.kf0; k0 < H; k0 += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            const int k = k0 + u;
            if (k < H) {
                if (k + PD < H) load(k + PD, ring[(u + PD) % (PD + 1)]);
                fwd(k, ring[u]);
            }
        }
    }

    // ---- epilogue of one block row (x_k in xk)
    auto emit = [&](int k) {
        if (d.kind == KIND_FINAL) {
            if (k >= s.r0 && k < s.r1) {
                c128* zrow = a.z + (size_t)rhs * a.geo.Nx * a.geo.Ny + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0;
                for (int c = s.c0 + tid; c < s.c1; c += NT) zrow[c] = cvt<double>(xk[c]);
            }
        } else if (d.kind == KIND_UNIT) {
            cx<T>* col = reinterpret_cast<cx<T>*>(a.Q) + d.q_col;
            const int hb = (s.sides >> SIDE_B) & 1, ht = (s.sides >> SIDE_T) & 1;
            const int hl = (s.sides >> SIDE_L) & 1, hr = (s.sides >> SIDE_R) & 1;
            int off = -1;
            if (hb && k == s.r0 - 1) off = 0;
            if (hb && k == s.r0) off = W;
            if (ht && k == s.r1 - 1) off = 2 * W;
            if (ht && k == s.r1) off = 3 * W;
            if (off >= 0)
                for (int c = tid; c < W; c += NT) col[off + c] = xk[c];
            if (tid == 0 && hl) { col[4 * W + k] = xk[s.c0 - 1]; col[4 * W + H + k] = xk[s.c0]; }
            if (tid == 1 && hr) { col[4 * W + 2 * H + k] = xk[s.c1 - 1]; col[4 * W + 3 * H + k] = xk[s.c1]; }
        } else if (d.zpart >= 0 && k >= s.r0 && k < s.r1) {
            cx<T>* zrow = reinterpret_cast<cx<T>*>(a.zpart) + (size_t)d.zpart * a.zpart_stride +
                          (size_t)rhs * a.geo.Nx * a.geo.Ny + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0;
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
    };

    // ---- backward substitution: x_k = y_k - G_k C_k x_{k+1}; xk holds x_{H-1} = y_{H-1}
    emit(H - 1);
    auto bwd = [&](int k, const cx<T>* buf) {
        if (tid < W) v[tid] = cvt<T>(coup_y(tab, s.tx, s.ty, H, tid, k, ih2)) * xk[tid];
        __syncthreads();
        gemv(buf);
        __syncthreads();
        if (tid < W) {
            const cx<T> y = (k >= d.kf0) ? Y[(size_t)k * W + tid] : zero;
            xk[tid] = y - reduce(tid);
        }
        __syncthreads();
        emit(k);
    };
    const int kstart = H - 2;
#pragma unroll
    for (int p = 0; p < PD; ++p)
        if (kstart - p >= d.kb0) load(kstart - p, ring[p]);
    for (int k0 = kstart; k0 >= d.kb0; k0 -= PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            const int k = k0 - u;
            if (k >= d.kb0) {
                if (k - PD >= d.kb0) load(k - PD, ring[(u + PD) % (PD + 1)]);
                bwd(k, ring[u]);
            }
        }
    }
}

// slot -> window point of the trace-line layout (see common.h)
__device__ inline void slot_point(const SubDesc& s, int sl, int& k, int& c) {
    const int W = s.W, H = s.H;
    if (sl < 4 * W) {
        const int line = sl / W;
        c = sl - line * W;
        k = (line == 0) ? s.r0 - 1 : (line == 1) ? s.r0 : (line == 2) ? s.r1 - 1 : s.r1;
    } else {
        const int v = sl - 4 * W, line = v / H;
        k = v - line * H;
        c = (line == 0) ? s.c0 - 1 : (line == 1) ? s.c0 : (line == 2) ? s.c1 - 1 : s.c1;
    }
}

// Trace-compressed sweep front: out = Q[out side, in slots] g[in slots].
template <typename T>
__global__ __launch_bounds__(256) void k_gemv(GemvArgs a) {
    constexpr int NT = 256, NW = 4;
    const GemvItem it = a.items[blockIdx.x];
    const GemvSolve& d = a.solves[it.solve];
    const SubDesc s = a.subs[d.sub];
    const int rhs = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ cx<T> gv[4 * kMaxWindow];
    __shared__ int slot[4 * kMaxWindow];
    __shared__ cx<T> part[NW][64];
    cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    const Local<T> L = make_local<T>(s, d.kind, a.geo.tab, d.in_h >= 0 ? tr + d.in_h : nullptr,
                                     d.in_v >= 0 ? tr + d.in_v : nullptr, ih2);
    int total = 0;
    for (int r = 0; r < d.nin; ++r) total += d.in_len[r];
    cx<T>* gp = reinterpret_cast<cx<T>*>(a.gparts) + ((size_t)rhs * 8 + (d.sweep - 1)) * a.LT + s.gp_off;
    for (int idx = tid; idx < total; idx += NT) {
        int r = 0, off = idx;
        while (off >= d.in_len[r]) { off -= d.in_len[r]; ++r; }
        const int sl = d.in_start[r] + off;
        int k, c;
        slot_point(s, sl, k, c);
        const cx<T> g = g_polarized(L, k, c);
        slot[idx] = sl;
        gv[idx] = g;
        if (it.first) gp[sl] = g;
    }
    __syncthreads();
    if (it.out < 0) return;   // a solve without outgoing traces only stores its g
    const int side = d.out_side[it.out];
    const int sb = (side == SIDE_B) ? 0 : (side == SIDE_T) ? 2 * s.W : (side == SIDE_L) ? 4 * s.W : 4 * s.W + 2 * s.H;
    const int len = (side == SIDE_B || side == SIDE_T) ? 2 * s.W : 2 * s.H;
    const int o = it.chunk * 64 + lane;
    const cx<T>* Qs = reinterpret_cast<const cx<T>*>(a.Q) + s.q_off + sb + o;
    cx<T> acc{T(0), T(0)};
    if (o < len) {
        int idx = wv;
        for (; idx + 3 * NW < total; idx += 4 * NW) {
            const cx<T> q0 = Qs[(size_t)slot[idx] * s.L];
            const cx<T> q1 = Qs[(size_t)slot[idx + NW] * s.L];
            const cx<T> q2 = Qs[(size_t)slot[idx + 2 * NW] * s.L];
            const cx<T> q3 = Qs[(size_t)slot[idx + 3 * NW] * s.L];
            acc = fma(acc, q0, gv[idx]);
            acc = fma(acc, q1, gv[idx + NW]);
            acc = fma(acc, q2, gv[idx + 2 * NW]);
            acc = fma(acc, q3, gv[idx + 3 * NW]);
        }
        for (; idx < total; idx += NW) acc = fma(acc, Qs[(size_t)slot[idx] * s.L], gv[idx]);
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && o < len) {
        const cx<T> val = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
        cx<T>* p = tr + d.out_off[it.out] + o;
        *p = d.out_acc[it.out] ? *p + val : val;
    }
}

__global__ void k_cast(const c128* src, c64* dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = c64{static_cast<float>(src[i].re), static_cast<float>(src[i].im)};
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

// out[rhs * ostride + l] (+)= sum_blk partial ; one workgroup per (l, rhs), fixed order
__global__ void k_dots_finish(const c128* partial, int nblk, int nv, int nrhs, c128* out, int ostride,
                              int accumulate) {
    __shared__ c128 red[256];
    const int l = blockIdx.x, rhs = blockIdx.y;
    const c128* pp = partial + ((size_t)rhs * nv + l) * nblk;
    c128 acc = mk(0.0, 0.0);
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc = acc + pp[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c128* o = out + (size_t)rhs * ostride + l;
        *o = accumulate ? *o + red[0] : red[0];
    }
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

// prefetch depth: as many blocks in flight as the 128-VGPR budget of a 1024-thread
// workgroup allows (complex64: 2 floats, complex128: 4 per element)
template <typename T, bool POLAR>
static void launch_chain_p(const ChainArgs& a, dim3 grid, int ept, hipStream_t st) {
    constexpr bool dbl = sizeof(T) == 8;
    if (ept <= 4) k_chain<T, 4, 2, POLAR><<<grid, 1024, 0, st>>>(a);
    else if (ept <= 8) k_chain<T, 8, dbl ? 1 : 2, POLAR><<<grid, 1024, 0, st>>>(a);
    else if (ept <= 16) k_chain<T, 16, dbl ? 0 : 1, POLAR><<<grid, 1024, 0, st>>>(a);
    else if (ept <= 32) k_chain<T, 32, 0, POLAR><<<grid, 1024, 0, st>>>(a);
    else k_chain<T, 64, 0, POLAR><<<grid, 1024, 0, st>>>(a);
}

hipError_t launch_chain(const ChainArgs& a, int nsolves, int nrhs, int ept, bool c64mode, bool polar,
                        hipStream_t st) {
    dim3 grid(nsolves, nrhs);
    if (c64mode) {
        if (polar) launch_chain_p<float, true>(a, grid, ept, st);
        else launch_chain_p<float, false>(a, grid, ept, st);
    } else {
        if (polar) launch_chain_p<double, true>(a, grid, ept, st);
        else launch_chain_p<double, false>(a, grid, ept, st);
    }
    return hipGetLastError();
}

hipError_t launch_gemv(const GemvArgs& a, int nitems, int nrhs, bool c64mode, hipStream_t st) {
    dim3 grid(nitems, nrhs);
    if (c64mode) k_gemv<float><<<grid, 256, 0, st>>>(a);
    else k_gemv<double><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_cast(const c128* src, c64* dst, size_t n, hipStream_t st) {
    k_cast<<<2048, 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
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
    k_dots_finish<<<dim3(a.nv, nrhs), 256, 0, st>>>(a.partial, a.nblk, a.nv, nrhs, out, ostride, accumulate);
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
