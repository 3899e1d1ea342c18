// HIP kernels of the L-sweeps library (gfx950).
//
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

// ------------------------------------------------------------------ buffer loads
// Raw buffer loads: 128-bit resource in SGPRs (base, byte size), 32-bit byte offset per lane.
// The whole offset goes in the per-lane operand, which the range check covers: offsets past
// the size (kOob for a lane that must read nothing) return zero without a memory access.
constexpr uint32_t kOob = 0x80000000u;
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ inline cx<T> bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline cx<float> bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ inline cx<double> bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

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

// Which right-hand sides and outputs one instantiation of k_chain handles.
enum ChainSet : int { CS_STAGE1 = 0, CS_FINAL = 1, CS_UNIT = 2, CS_POLAR = 3 };

// Batched block substitution with the twisted factorisation, two workgroups per
// (local solve, rhs): half 0 owns block rows below the middle row m, half 1 those above.
//   phase 0: forward elimination of each half towards m,
//            half 0: y_k = G_k (g_k - C_{k-1} y_{k-1}),  half 1: y_k = G_k (g_k - C_k y_{k+1});
//   phase 1: x_m = G_m (g_m - C_{m-1} y_{m-1} - C_m y_{m+1}) (computed by both halves), then
//            half 0: x_k = y_k - G_k C_k x_{k+1} downwards,  half 1: x_k = y_k - G_k C_{k-1} x_{k-1} upwards.
// Thread tid < NA = floor(1024/W)*W owns block row t = tid % W and the columns
// c = tid / W + NG*j (c < W) of every W x W block G_k: its elements sit at the flat
// offsets tid + NA*j of the column-major block, so the loads are fully coalesced.
// A register ring keeps PD blocks of G (and the right-hand-side / y values) in flight ahead
// of the block in use; every load in the loop is unconditional (zero past the buffer, and
// columns past W meet a zero entry of v) and nothing is stored to global memory inside the
// loop (the half's y or x
// live in Ybuf, LDS when it fits), so waiting for a block never waits for the younger
// prefetches.  Thread t < W carries its y/x entry in a register: two barriers per block.
template <typename T, int EPT, int PD, int CS, bool YLDS, int PH>
__global__ __launch_bounds__(1024) void k_chain(ChainArgs a) {
    constexpr int NT = 1024;
    extern __shared__ __align__(16) unsigned char dyn[];
    const int sidx = blockIdx.x >> 1, h = blockIdx.x & 1, nsol = gridDim.x >> 1;
    const SolveDesc& dref = a.descs[sidx];
    const int sub = dref.sub, kind = dref.kind;
    const int kf0 = dref.kf0, kf1 = dref.kf1, kb0 = dref.kb0, kb1 = dref.kb1;
    const SubDesc s = a.subs[sub];
    const int rhs = blockIdx.y;
    const int W = s.W, H = s.H, m = s.mid, tid = threadIdx.x;
    const int NG = NT / W, NA = NG * W;
    const bool act = tid < NA;
    const bool mine = tid < W;
    const int tc = mine ? tid : W - 1;          // clamped column for address arithmetic
    const int cg = act ? tid / W : 0;
    const int WW = W * W;
    __shared__ cx<T> v[kMaxWindow + 1];   // v[kMaxWindow] stays zero: the slot of masked columns
    __shared__ cx<T> part[NT];
    __shared__ c128 a2h[kMaxWindow + 1];

    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    for (int k = tid; k <= H; k += NT) a2h[k] = tab[s.ty + H + k];   // alpha_y at the half points
    if (tid == 0) v[kMaxWindow] = cx<T>{T(0), T(0)};
    const c128 ia_c = tab[s.tx + tc];                                  // 1/alpha_x of my column
    const cx<T>* Gs = reinterpret_cast<const cx<T>*>(a.G) + s.g_off;
    cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
    // y of both halves (written in phase 0, read in phase 1); x goes to Ybuf
    cx<T>* Yg = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)blockIdx.y * nsol + sidx) * a.Y_stride;
    cx<T>* Ybuf = YLDS ? reinterpret_cast<cx<T>*>(dyn) : Yg + (PH == 1 ? (size_t)H * W : 0);
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    // a prvalue zero: a named zero in a conditional with an array element makes the
    // compiler select between addresses and move the register rings to scratch
    auto zero = []() { return cx<T>{T(0), T(0)}; };
    // coupling of block rows l and l+1 at my column (diagonal of C_l)
    auto cy = [&](int l) { return cvt<T>(-ih2 * (a2h[l + 1] * ia_c)); };

    // right-hand side sources (one unconditional load per block row and thread)
    const bool from_r = CS == CS_STAGE1 || CS == CS_POLAR;
    const c128* rptr = from_r ? a.r + (size_t)rhs * N : a.fw + (size_t)rhs * a.fw_stride + s.fw_off;
    const __amdgpu_buffer_rsrc_t rsrc =
        make_rsrc(rptr, CS == CS_UNIT ? 0u : (uint32_t)((from_r ? N : (size_t)H * W) * sizeof(c128)));
    const uint32_t rbase = (uint32_t)((from_r ? (size_t)s.wy0 * a.geo.Nx + s.wx0 + tc : (size_t)tc) * sizeof(c128));
    const uint32_t rstep = (uint32_t)((from_r ? (size_t)a.geo.Nx : (size_t)W) * sizeof(c128));
    const __amdgpu_buffer_rsrc_t grsrc = make_rsrc(Gs, (uint32_t)((size_t)H * WW * sizeof(cx<T>)));
    const __amdgpu_buffer_rsrc_t yrsrc = make_rsrc(Yg, (uint32_t)((size_t)H * W * sizeof(cx<T>)));
    const bool in_cols = mine && tid >= s.c0 && tid < s.c1;
    const int unit_k = dref.unit_k, unit_c = dref.unit_c;
    Local<T> L = make_local<T>(s, kind, tab, nullptr, nullptr, ih2);
    if constexpr (CS == CS_POLAR) {
        L.in_h = dref.in_h >= 0 ? tr + dref.in_h : nullptr;
        L.in_v = dref.in_v >= 0 ? tr + dref.in_v : nullptr;
    }
    // value of g_k at my column from the raw loaded value
    auto rhs_use = [&](int k, c128 raw) -> cx<T> {
        if (k < kf0 || k > kf1) return zero();
        if constexpr (CS == CS_UNIT) return (k == unit_k && tid == unit_c) ? cx<T>{T(1), T(0)} : zero();
        if constexpr (CS == CS_FINAL) return mine ? cvt<T>(raw) : zero();
        if constexpr (CS == CS_POLAR)
            if (kind != KIND_STAGE1) return mine ? g_polarized(L, k, tid) : zero();
        return (in_cols && k >= s.r0 && k < s.r1) ? cvt<T>(raw) : zero();
    };
    auto rhs_load = [&](int k) -> c128 {
        if constexpr (CS == CS_UNIT) return mk(0.0, 0.0);
        else return bload<double>(rsrc, rbase + (uint32_t)k * rstep);
    };
    auto yload = [&](int k) -> cx<T> { return bload<T>(yrsrc, (uint32_t)(k * W + tc) * (uint32_t)sizeof(cx<T>)); };
    // G_k elements of this thread; lanes past the last block read zeros from the buffer
    auto load = [&](int k, cx<T>* buf) {
        const uint32_t kb = (uint32_t)k * (uint32_t)WW * (uint32_t)sizeof(cx<T>);
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            buf[j] = bload<T>(grsrc, kb + (uint32_t)(tid + NA * j) * (uint32_t)sizeof(cx<T>));
    };
    // part[tid] = sum_j G_k[c_j][t] v[c_j].  With up to 8 complex64 values per thread all v
    // reads are issued before the first product (one LDS round trip per block instead of one
    // per column; columns past W, and the lanes past NA, read the zero slot).  Larger or
    // complex128 blocks leave no registers for that and take one read per product.
    auto gemv = [&](const cx<T>* buf) {
        cx<T> acc = zero();
        if constexpr (sizeof(T) == 4 && EPT <= 8) {
            cx<T> vv[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int c = cg + NG * j;
                vv[j] = v[(act && c < W) ? c : kMaxWindow];
            }
#pragma unroll
            for (int j = 0; j < EPT; ++j) acc = acc + buf[j] * vv[j];
        } else {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int c = cg + NG * j;
                const bool ok = act && c < W;
                const cx<T> t = buf[j] * v[ok ? c : 0];
                if (ok) acc = acc + t;
            }
        }
        part[tid] = acc;
    };
    auto reduce = [&](int t) {
        cx<T> y = part[t];
        for (int g = 1; g < NG; ++g) y = y + part[g * W + t];
        return y;
    };

    cx<T> ring[PD + 1][EPT];
    c128 rr[PD + 1];
    cx<T> yr[PD + 1];
    cx<T> yv = zero();   // the y (phase 0) or x (phase 1) entry of my column at the previous block row
    __syncthreads();   // a2h

    if constexpr (PH == 0) {
        // ---- forward elimination of this half towards the middle row
        const int kstart = h == 0 ? kf0 : kf1;
        const int dir = h == 0 ? 1 : -1;
        const int n = h == 0 ? m - kf0 : kf1 - m;   // block rows m-1..kf0 or kf1..m+1
        auto kat = [&](int i) { return kstart + dir * min(i, n - 1); };
#pragma unroll
        for (int p = 0; p < PD; ++p)
            if (n > 0) {
                rr[p] = rhs_load(kat(p));
                load(kat(p), ring[p]);
            }
        auto fstep = [&](int i, int u) __attribute__((always_inline)) {
            const int k = kstart + dir * i;
            rr[(u + PD) % (PD + 1)] = rhs_load(kat(i + PD));
            load(kat(i + PD), ring[(u + PD) % (PD + 1)]);
            if (mine) {
                cx<T> g = rhs_use(k, rr[u]);
                if (i > 0) g = g - cy(h == 0 ? k - 1 : k) * yv;
                v[tid] = g;
            }
            __syncthreads();
            gemv(ring[u]);
            __syncthreads();
            if (mine) {
                yv = reduce(tid);
                Ybuf[(size_t)k * W + tid] = yv;
            }
        };
        // whole groups of PD + 1 steps carry no guard, so every path through the loop
        // consumes the ring in order and the waits stay partial; then the tail
        int i0 = 0;
        for (; i0 + PD < n; i0 += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) fstep(i0 + u, u);
        }
#pragma unroll
        for (int u = 0; u < PD; ++u)
            if (i0 + u < n) fstep(i0 + u, u);
        if constexpr (YLDS) {
            __syncthreads();
            const int lo = h == 0 ? kf0 : m + 1, hi = h == 0 ? m - 1 : kf1;
            for (int idx = tid; idx < (hi - lo + 1) * W; idx += NT) Yg[(size_t)lo * W + idx] = Ybuf[(size_t)lo * W + idx];
        }
        return;
    }

    // ---- phase 1: middle row, then back substitution of this half away from it
    {
        cx<T> gm[EPT];
        load(m, gm);
        const c128 rm = rhs_load(m);
        const cx<T> ylo = (kf0 <= m - 1) ? yload(m - 1) : zero();
        const cx<T> yhi = (kf1 >= m + 1) ? yload(m + 1) : zero();
        if (mine) {
            cx<T> g = rhs_use(m, rm);
            if (m >= 1) g = g - cy(m - 1) * ylo;
            if (m + 1 <= H - 1) g = g - cy(m) * yhi;
            v[tid] = g;
        }
        __syncthreads();
        gemv(gm);
        __syncthreads();
        if (mine) {
            yv = reduce(tid);
            Ybuf[(size_t)m * W + tid] = yv;
        }
    }
    {
        const int kstart = h == 0 ? m - 1 : m + 1;
        const int dir = h == 0 ? -1 : 1;
        const int n = h == 0 ? m - kb0 : kb1 - m;   // block rows m-1..kb0 or m+1..kb1
        auto kat = [&](int i) { return kstart + dir * min(i, n - 1); };
#pragma unroll
        for (int p = 0; p < PD; ++p)
            if (n > 0) {
                yr[p] = yload(kat(p));
                load(kat(p), ring[p]);
            }
        auto bstep = [&](int i, int u) __attribute__((always_inline)) {
            const int k = kstart + dir * i;
            yr[(u + PD) % (PD + 1)] = yload(kat(i + PD));
            load(kat(i + PD), ring[(u + PD) % (PD + 1)]);
            if (mine) v[tid] = cy(h == 0 ? k : k - 1) * yv;
            __syncthreads();
            gemv(ring[u]);
            __syncthreads();
            if (mine) {
                // y of the bottom half is zero below kf0, that of the top half above kf1
                const cx<T> y = (h == 0 ? k >= kf0 : k <= kf1) ? yr[u] : zero();
                yv = y - reduce(tid);
                Ybuf[(size_t)k * W + tid] = yv;
            }
        };
        int i0 = 0;
        for (; i0 + PD < n; i0 += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) bstep(i0 + u, u);
        }
#pragma unroll
        for (int u = 0; u < PD; ++u)
            if (i0 + u < n) bstep(i0 + u, u);
    }
    __syncthreads();

    // ---- outputs of the block rows this half owns, from Ybuf
    const cx<T>* X = Ybuf;
    const int olo = h == 0 ? kb0 : max(kb0, m + 1);
    const int ohi = h == 0 ? min(kb1, m) : kb1;
    auto own = [&](int k) { return k >= olo && k <= ohi; };
    if constexpr (CS == CS_FINAL) {
        const int r0 = max(s.r0, olo), r1 = min(s.r1, ohi + 1);
        const int nc = s.c1 - s.c0, n = max(0, r1 - r0) * nc;
        c128* z = a.z + (size_t)rhs * N + (size_t)(s.wy0 + r0) * a.geo.Nx + s.wx0 + s.c0;
        for (int idx = tid; idx < n; idx += NT) {
            const int rr0 = idx / nc, cc = idx - rr0 * nc;
            z[(size_t)rr0 * a.geo.Nx + cc] = cvt<double>(X[(size_t)(r0 + rr0) * W + s.c0 + cc]);
        }
    } else if constexpr (CS == CS_UNIT) {
        cx<T>* col = reinterpret_cast<cx<T>*>(a.Q) + dref.q_col;
        const int L8 = 4 * W + 4 * H;
        for (int sl = tid; sl < L8; sl += NT) {
            int k, c, side;
            if (sl < 4 * W) {
                const int line = sl / W;
                c = sl - line * W;
                side = line < 2 ? SIDE_B : SIDE_T;
                k = line == 0 ? s.r0 - 1 : line == 1 ? s.r0 : line == 2 ? s.r1 - 1 : s.r1;
            } else {
                const int q = sl - 4 * W, line = q / H;
                k = q - line * H;
                side = line < 2 ? SIDE_L : SIDE_R;
                c = line == 0 ? s.c0 - 1 : line == 1 ? s.c0 : line == 2 ? s.c1 - 1 : s.c1;
            }
            if (((s.sides >> side) & 1) && own(k)) col[sl] = X[(size_t)k * W + c];
        }
    } else {
        if (dref.zpart >= 0) {
            const int r0 = max(s.r0, olo), r1 = min(s.r1, ohi + 1);
            const int nc = s.c1 - s.c0, n = max(0, r1 - r0) * nc;
            cx<T>* z = reinterpret_cast<cx<T>*>(a.zpart) + (size_t)dref.zpart * a.zpart_stride + (size_t)rhs * N +
                       (size_t)(s.wy0 + r0) * a.geo.Nx + s.wx0 + s.c0;
            for (int idx = tid; idx < n; idx += NT) {
                const int rr0 = idx / nc, cc = idx - rr0 * nc;
                z[(size_t)rr0 * a.geo.Nx + cc] = X[(size_t)(r0 + rr0) * W + s.c0 + cc];
            }
        }
        const int nout = dref.nout;
        for (int o = 0; o < nout; ++o) {
            const int side = dref.out_side[o];
            cx<T>* out = tr + dref.out_off[o];
            const bool acc = dref.out_acc[o] != 0;
            if (side == SIDE_B || side == SIDE_T) {
                const int l0 = (side == SIDE_B) ? s.r0 - 1 : s.r1 - 1;
                for (int idx = tid; idx < 2 * W; idx += NT) {
                    const int line = idx / W, c = idx - line * W;
                    if (!own(l0 + line)) continue;
                    const cx<T> xv = X[(size_t)(l0 + line) * W + c];
                    out[idx] = acc ? out[idx] + xv : xv;
                }
            } else {
                const int l0 = (side == SIDE_L) ? s.c0 - 1 : s.c1 - 1;
                for (int idx = tid; idx < 2 * H; idx += NT) {
                    const int line = idx / H, k = idx - line * H;
                    if (!own(k)) continue;
                    const cx<T> xv = X[(size_t)k * W + l0 + line];
                    out[idx] = acc ? out[idx] + xv : xv;
                }
            }
        }
    }
}

// The same twisted block substitution for R right-hand sides per workgroup (stage 1 and the
// final z solves): every G_k element is loaded once and applied to the R vectors of the
// group, so a batch of sources reads the factors nrhs/R times instead of nrhs times.  y and
// x live in global memory (phase 0 writes y at [0, H W) of each right-hand side's slab,
// phase 1 writes x at [H W, 2 H W)).
template <typename T, int EPT, int PD, int CS, int R, int PH>
__global__ __launch_bounds__(1024) void k_chain_mr(ChainArgs a) {
    static_assert(CS == CS_STAGE1 || CS == CS_FINAL, "stage 1 and final solves only");
    constexpr int NT = 1024;
    const int sidx = blockIdx.x >> 1, h = blockIdx.x & 1, nsol = gridDim.x >> 1;
    const SolveDesc& dref = a.descs[sidx];
    const int sub = dref.sub;
    const int kf0 = dref.kf0, kf1 = dref.kf1, kb0 = dref.kb0, kb1 = dref.kb1;
    const SubDesc s = a.subs[sub];
    const int rhs0 = blockIdx.y * R;
    const int nr = min(R, a.nrhs - rhs0);   // right-hand sides of this group (the rest only reads zeros)
    const int W = s.W, H = s.H, m = s.mid, tid = threadIdx.x;
    const int NG = NT / W, NA = NG * W;
    const bool act = tid < NA;
    const bool mine = tid < W;
    const int tc = mine ? tid : W - 1;
    const int cg = act ? tid / W : 0;
    const int WW = W * W;
    __shared__ cx<T> v[R][kMaxWindow + 1];   // v[r][kMaxWindow] stays zero
    __shared__ cx<T> part[R][NT];
    __shared__ c128 a2h[kMaxWindow + 1];

    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    for (int k = tid; k <= H; k += NT) a2h[k] = tab[s.ty + H + k];
    if (tid < R) v[tid][kMaxWindow] = cx<T>{T(0), T(0)};
    const c128 ia_c = tab[s.tx + tc];
    const cx<T>* Gs = reinterpret_cast<const cx<T>*>(a.G) + s.g_off;
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    auto zero = []() { return cx<T>{T(0), T(0)}; };
    auto cy = [&](int l) { return cvt<T>(-ih2 * (a2h[l + 1] * ia_c)); };
    constexpr bool from_r = CS == CS_STAGE1;
    // per right-hand side: its sources, its y/x slab (empty ranges for a short last group)
    __amdgpu_buffer_rsrc_t rsrc[R], yrsrc[R];
    cx<T>* Yg[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int rhs = rhs0 + r;
        const bool ok = rhs < a.nrhs;
        const int rr = ok ? rhs : rhs0;
        const c128* rptr = from_r ? a.r + (size_t)rr * N : a.fw + (size_t)rr * a.fw_stride + s.fw_off;
        rsrc[r] = make_rsrc(rptr, ok ? (uint32_t)((from_r ? N : (size_t)H * W) * sizeof(c128)) : 0u);
        Yg[r] = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)rr * nsol + sidx) * a.Y_stride;
        yrsrc[r] = make_rsrc(Yg[r], ok ? (uint32_t)((size_t)H * W * sizeof(cx<T>)) : 0u);
    }
    const uint32_t rbase = (uint32_t)((from_r ? (size_t)s.wy0 * a.geo.Nx + s.wx0 + tc : (size_t)tc) * sizeof(c128));
    const uint32_t rstep = (uint32_t)((from_r ? (size_t)a.geo.Nx : (size_t)W) * sizeof(c128));
    const __amdgpu_buffer_rsrc_t grsrc = make_rsrc(Gs, (uint32_t)((size_t)H * WW * sizeof(cx<T>)));
    const bool in_cols = mine && tid >= s.c0 && tid < s.c1;
    auto rhs_use = [&](int k, cx<T> raw) -> cx<T> {
        if (k < kf0 || k > kf1) return zero();
        if constexpr (CS == CS_FINAL) return mine ? raw : zero();
        return (in_cols && k >= s.r0 && k < s.r1) ? raw : zero();
    };
    auto rhs_load = [&](int r, int k) -> cx<T> { return cvt<T>(bload<double>(rsrc[r], rbase + (uint32_t)k * rstep)); };
    auto yload = [&](int r, int k) -> cx<T> {
        return bload<T>(yrsrc[r], (uint32_t)(k * W + tc) * (uint32_t)sizeof(cx<T>));
    };
    auto load = [&](int k, cx<T>* buf) {
        const uint32_t kb = (uint32_t)k * (uint32_t)WW * (uint32_t)sizeof(cx<T>);
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            buf[j] = bload<T>(grsrc, kb + (uint32_t)(tid + NA * j) * (uint32_t)sizeof(cx<T>));
    };
    // part[r][tid] = sum_j G_k[c_j][t] v[r][c_j]
    auto gemv = [&](const cx<T>* buf) {
        cx<T> acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = zero();
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int c = cg + NG * j;
            const bool ok = act && c < W;
            const int cc = ok ? c : 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const cx<T> t = buf[j] * v[r][cc];
                if (ok) acc[r] = acc[r] + t;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) part[r][tid] = acc[r];
    };
    auto reduce = [&](int r, int t) {
        cx<T> y = part[r][t];
        for (int g = 1; g < NG; ++g) y = y + part[r][g * W + t];
        return y;
    };

    cx<T> ring[PD + 1][EPT];
    cx<T> rr[PD + 1][R];
    cx<T> yv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) yv[r] = zero();
    __syncthreads();

    if constexpr (PH == 0) {
        const int kstart = h == 0 ? kf0 : kf1;
        const int dir = h == 0 ? 1 : -1;
        const int n = h == 0 ? m - kf0 : kf1 - m;
        auto kat = [&](int i) { return kstart + dir * min(i, n - 1); };
#pragma unroll
        for (int p = 0; p < PD; ++p)
            if (n > 0) {
#pragma unroll
                for (int r = 0; r < R; ++r) rr[p][r] = rhs_load(r, kat(p));
                load(kat(p), ring[p]);
            }
        for (int i0 = 0; i0 < n; i0 += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) {
                const int i = i0 + u;
                if (i < n) {
                    const int k = kstart + dir * i;
#pragma unroll
                    for (int r = 0; r < R; ++r) rr[(u + PD) % (PD + 1)][r] = rhs_load(r, kat(i + PD));
                    load(kat(i + PD), ring[(u + PD) % (PD + 1)]);
                    if (mine) {
                        const cx<T> c = cy(h == 0 ? k - 1 : k);
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            cx<T> g = rhs_use(k, rr[u][r]);
                            if (i > 0) g = g - c * yv[r];
                            v[r][tid] = g;
                        }
                    }
                    __syncthreads();
                    gemv(ring[u]);
                    __syncthreads();
                    if (mine) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            yv[r] = reduce(r, tid);
                            if (r < nr) Yg[r][(size_t)k * W + tid] = yv[r];
                        }
                    }
                }
            }
        }
        return;
    }

    // ---- phase 1: middle row, then back substitution of this half away from it
    {
        cx<T> gm[EPT];
        load(m, gm);
        cx<T> rm[R], ylo[R], yhi[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            rm[r] = rhs_load(r, m);
            ylo[r] = (kf0 <= m - 1) ? yload(r, m - 1) : zero();
            yhi[r] = (kf1 >= m + 1) ? yload(r, m + 1) : zero();
        }
        if (mine) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cx<T> g = rhs_use(m, rm[r]);
                if (m >= 1) g = g - cy(m - 1) * ylo[r];
                if (m + 1 <= H - 1) g = g - cy(m) * yhi[r];
                v[r][tid] = g;
            }
        }
        __syncthreads();
        gemv(gm);
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                yv[r] = reduce(r, tid);
                if (r < nr) Yg[r][(size_t)H * W + (size_t)m * W + tid] = yv[r];
            }
        }
    }
    {
        const int kstart = h == 0 ? m - 1 : m + 1;
        const int dir = h == 0 ? -1 : 1;
        const int n = h == 0 ? m - kb0 : kb1 - m;
        auto kat = [&](int i) { return kstart + dir * min(i, n - 1); };
#pragma unroll
        for (int p = 0; p < PD; ++p)
            if (n > 0) {
#pragma unroll
                for (int r = 0; r < R; ++r) rr[p][r] = yload(r, kat(p));
                load(kat(p), ring[p]);
            }
        for (int i0 = 0; i0 < n; i0 += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) {
                const int i = i0 + u;
                if (i < n) {
                    const int k = kstart + dir * i;
#pragma unroll
                    for (int r = 0; r < R; ++r) rr[(u + PD) % (PD + 1)][r] = yload(r, kat(i + PD));
                    load(kat(i + PD), ring[(u + PD) % (PD + 1)]);
                    if (mine) {
                        const cx<T> c = cy(h == 0 ? k : k - 1);
#pragma unroll
                        for (int r = 0; r < R; ++r) v[r][tid] = c * yv[r];
                    }
                    __syncthreads();
                    gemv(ring[u]);
                    __syncthreads();
                    if (mine) {
                        const bool has_y = h == 0 ? k >= kf0 : k <= kf1;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const cx<T> y = has_y ? rr[u][r] : zero();
                            yv[r] = y - reduce(r, tid);
                            if (r < nr) Yg[r][(size_t)H * W + (size_t)k * W + tid] = yv[r];
                        }
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- outputs of the block rows this half owns
    const int olo = h == 0 ? kb0 : max(kb0, m + 1);
    const int ohi = h == 0 ? min(kb1, m) : kb1;
    for (int r = 0; r < R; ++r) {
        const int rhs = rhs0 + r;
        if (rhs >= a.nrhs) break;
        const cx<T>* X = Yg[r] + (size_t)H * W;
        if constexpr (CS == CS_FINAL) {
            const int r0 = max(s.r0, olo), r1 = min(s.r1, ohi + 1);
            const int nc = s.c1 - s.c0, n = max(0, r1 - r0) * nc;
            c128* z = a.z + (size_t)rhs * N + (size_t)(s.wy0 + r0) * a.geo.Nx + s.wx0 + s.c0;
            for (int idx = tid; idx < n; idx += NT) {
                const int rr0 = idx / nc, cc = idx - rr0 * nc;
                z[(size_t)rr0 * a.geo.Nx + cc] = cvt<double>(X[(size_t)(r0 + rr0) * W + s.c0 + cc]);
            }
        } else {
            cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
            auto own = [&](int k) { return k >= olo && k <= ohi; };
            for (int o = 0; o < dref.nout; ++o) {
                const int side = dref.out_side[o];
                cx<T>* out = tr + dref.out_off[o];
                const bool acc = dref.out_acc[o] != 0;
                if (side == SIDE_B || side == SIDE_T) {
                    const int l0 = (side == SIDE_B) ? s.r0 - 1 : s.r1 - 1;
                    for (int idx = tid; idx < 2 * W; idx += NT) {
                        const int line = idx / W, c = idx - line * W;
                        if (!own(l0 + line)) continue;
                        const cx<T> xv = X[(size_t)(l0 + line) * W + c];
                        out[idx] = acc ? out[idx] + xv : xv;
                    }
                } else {
                    const int l0 = (side == SIDE_L) ? s.c0 - 1 : s.c1 - 1;
                    for (int idx = tid; idx < 2 * H; idx += NT) {
                        const int line = idx / H, k = idx - line * H;
                        if (!own(k)) continue;
                        const cx<T> xv = X[(size_t)k * W + l0 + line];
                        out[idx] = acc ? out[idx] + xv : xv;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ K4 on packed symmetric factors
// Two consecutive complex values (entries t and t+1 of a packed row) in one load.
template <typename T>
struct Pair {
    cx<T> a, b;
};
template <typename T>
__device__ inline Pair<T> bload2(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline Pair<float> bload2<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(Pair<float>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <>
__device__ inline Pair<double> bload2<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return Pair<double>{bload<double>(r, off), bload<double>(r, off + 16u)};
}
// the same with a uniform part of the offset in the scalar operand: voff alone past the buffer
// size reads zeros whether or not the range check adds soff
template <typename T>
__device__ inline Pair<T> bload2s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline Pair<float> bload2s<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(Pair<float>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <>
__device__ inline Pair<double> bload2s<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return Pair<double>{__builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0)),
                        __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + 16u, 0))};
}

// Sum over groups of RS = 1, 2 or 4 neighbouring lanes (RS uniform), by DPP quad permutations.
__device__ inline float lane_sum(float x, int RS) {
    if (RS >= 2) x += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
    if (RS >= 4) x += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x4E, 0xF, 0xF, false));
    return x;
}
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double lane_sum(double x, int RS) {
    if (RS >= 2) x += dpp_f64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    if (RS >= 4) x += dpp_f64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    return x;
}

// The twisted block substitution of k_chain (stage 1 and final solves, one right-hand side per
// workgroup) on the factors in the packed symmetric tile layout (tile_nt / sym_block): about
// half the bytes of the full blocks.  NT lanes; lane l holds the tiles tau = l + NT m (m < TPL).
// For its tile (I, J) it forms the row sums A v_J (into c[J][4I..4I+3]) and, off the diagonal,
// the column sums A^T v_I (into c[I][4J..4J+3]), so every entry read from HBM is used twice from
// registers.  c (LDS, [nt][4 nt]) is then summed over J by RS lanes per row (unrolled LDS reads
// into two accumulators, then DPP).  A register ring keeps PD blocks in flight; scheduling
// barriers keep the issue order of the loads, so each wait covers only the block in use.  The
// shapes (NT, TPL, PD, RS) a window width allows are listed in kSymCfgs and timed at setup.
template <typename T, int NT, int TPL, int PD, int RS, int CS, int PH>
__global__ __launch_bounds__(NT) void k_chain_sym(ChainArgs a) {
    static_assert(CS == CS_STAGE1 || CS == CS_FINAL, "stage 1 and final solves only");
    static_assert(RS == 1 || RS == 2 || RS == 4, "1, 2 or 4 lanes per row");
    extern __shared__ __align__(16) unsigned char dyn[];
    cx<T>* cs = reinterpret_cast<cx<T>*>(dyn);   // c[J][r] at J * Wp + r, J <= nt (row nt zero)
    const int sidx = blockIdx.x >> 1, h = blockIdx.x & 1, nsol = gridDim.x >> 1;
    const SolveDesc& dref = a.descs[sidx];
    const int kf0 = dref.kf0, kf1 = dref.kf1, kb0 = dref.kb0, kb1 = dref.kb1;
    const SubDesc s = a.subs[dref.sub];
    const int rhs = blockIdx.y;
    const int W = s.W, H = s.H, m = s.mid, tid = threadIdx.x;
    // c rows are Wp apart, Wp = 10 (mod 16) entries (80 bytes mod 128 in complex64): the 16-byte
    // row-sum writes of eight consecutive tiles (J, J+1, ...) cover all LDS banks, and the RS lanes
    // of a row read rows of c 80 bytes apart in the reduction
    const int nt = tile_nt(W), Wp = sym_cstride(W), NTL = tile_count(W);
    const uint32_t BSb = (uint32_t)sym_block(W) * (uint32_t)sizeof(cx<T>);   // bytes per block
    // the reduction of row t: lanes RS t .. RS t + RS-1; the first of them owns the row
    const int tr = min(tid / RS, W - 1), rq = tid % RS;
    const bool mine = rq == 0 && tid / RS < W;
    __shared__ __align__(16) cx<T> v[kMaxWindow + 4];   // zero past W
    __shared__ cx<T> ay[kMaxWindow];                      // -alpha_y(l + 1/2) / h^2, l < H - 1
    __shared__ cx<T> ax[kMaxWindow];                      // 1/alpha_x at the points

    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    for (int l = tid; l < H - 1; l += NT) ay[l] = cvt<T>(-ih2 * tab[s.ty + H + l + 1]);
    for (int c = tid; c < W; c += NT) ax[c] = cvt<T>(tab[s.tx + c]);
    for (int c = W + tid; c < 4 * nt; c += NT) v[c] = cx<T>{T(0), T(0)};
    const cx<T>* Gs = reinterpret_cast<const cx<T>*>(a.G) + s.gs_off;
    cx<T>* Yg = reinterpret_cast<cx<T>*>(a.Y) + ((size_t)rhs * nsol + sidx) * a.Y_stride;
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    auto zero = []() { return cx<T>{T(0), T(0)}; };
    // coupling of block rows l and l+1 at my row (iax: after the first barrier)
    cx<T> iax = zero();
    auto cy = [&](int l) { return ay[l] * iax; };

    constexpr bool from_r = CS == CS_STAGE1;
    const c128* rptr = from_r ? a.r + (size_t)rhs * N : a.fw + (size_t)rhs * a.fw_stride + s.fw_off;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(rptr, (uint32_t)((from_r ? N : (size_t)H * W) * sizeof(c128)));
    // only the row owners read right-hand sides and y (the other lanes read nothing)
    const uint32_t rbase = mine ? (uint32_t)((from_r ? (size_t)s.wy0 * a.geo.Nx + s.wx0 + tr : (size_t)tr) * sizeof(c128))
                                : kOob;
    const uint32_t rstep = mine ? (uint32_t)((from_r ? (size_t)a.geo.Nx : (size_t)W) * sizeof(c128)) : 0u;
    const __amdgpu_buffer_rsrc_t grsrc = make_rsrc(Gs, (uint32_t)H * BSb);
    const __amdgpu_buffer_rsrc_t yrsrc = make_rsrc(Yg, (uint32_t)((size_t)H * W * sizeof(cx<T>)));
    const bool in_cols = mine && tr >= s.c0 && tr < s.c1;
    auto rhs_use = [&](int k, c128 raw) -> cx<T> {
        if (k < kf0 || k > kf1) return zero();
        if constexpr (CS == CS_FINAL) return mine ? cvt<T>(raw) : zero();
        return (in_cols && k >= s.r0 && k < s.r1) ? cvt<T>(raw) : zero();
    };
    auto rhs_load = [&](int k) -> c128 { return bload<double>(rsrc, rbase + (uint32_t)k * rstep); };
    auto yload = [&](int k) -> cx<T> {
        return bload<T>(yrsrc, mine ? (uint32_t)(k * W + tr) * (uint32_t)sizeof(cx<T>) : kOob);
    };

    // my tiles: (I, J) and the byte offset of entry pair 0 in a block (kOob past the last tile)
    int tI[TPL], tJ[TPL];
    uint32_t toff[TPL];
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
        const int tau = tid + NT * q;
        int I = 0, start = 0;
        while (I < nt - 1 && start + (nt - I) <= tau) {
            start += nt - I;
            ++I;
        }
        tI[q] = I;
        tJ[q] = I + (tau - start);
        // an idle lane's offsets lie past the buffer (every block and pair), so its loads read zeros
        toff[q] = tau < NTL ? (uint32_t)(2 * tau) * (uint32_t)sizeof(cx<T>) : (uint32_t)H * BSb;
    }
    const uint32_t ustep = (uint32_t)(2 * NTL) * (uint32_t)sizeof(cx<T>);   // bytes between entry pairs
    struct Slot {
        Pair<T> A[TPL][8];
    };
    auto load = [&](int k, Slot& sl) {
        const uint32_t kb = (uint32_t)k * BSb;
#pragma unroll
        for (int q = 0; q < TPL; ++q)
#pragma unroll
            for (int u = 0; u < 8; ++u)
                sl.A[q][u] = bload2s<T>(grsrc, toff[q], kb + (uint32_t)u * ustep);
    };
    // c[J][4I+i] and c[I][4J+j] of my tiles (after the first barrier: v ready)
    auto gemv = [&](const Slot& sl) {
#pragma unroll
        for (int q = 0; q < TPL; ++q) {
            if (tid + NT * q >= NTL) continue;
            const int I = tI[q], J = tJ[q];
            cx<T> vI[4], vJ[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                vI[i] = v[4 * I + i];
                vJ[i] = v[4 * J + i];
            }
            // entry q = 4i + j is sl.A[q][q / 2].a (q even) or .b (q odd)
            auto e = [&](int i, int j) -> cx<T> {
                const Pair<T>& p = sl.A[q][(4 * i + j) >> 1];
                return ((4 * i + j) & 1) ? p.b : p.a;
            };
            cx<T> row[4], col[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                row[i] = zero();
                col[i] = zero();
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    row[i] = cmac(row[i], e(i, j), vJ[j]);
                    col[j] = cmac(col[j], e(i, j), vI[i]);
                }
#pragma unroll
            for (int i = 0; i < 4; ++i) cs[J * Wp + 4 * I + i] = row[i];
            if (I < J)
#pragma unroll
                for (int j = 0; j < 4; ++j) cs[I * Wp + 4 * J + j] = col[j];
        }
    };
    // (G_k v)_t for the row owners (every lane takes part: the group sums are lane exchanges)
    // every lane's share of the reduction is at most NRED partial sums (nt <= sym_nt_max(NT TPL))
    constexpr int NRED = (sym_nt_max(NT * TPL) + RS - 1) / RS;
    // Every read and add is unconditional: a row index past nt reads row nt of c, which is zero, so all
    // NRED reads are issued before the first wait (guarded reads compile to one branch and one LDS
    // round trip each).
    auto reduce = [&]() {
        cx<T> y0 = zero(), y1 = zero();
#pragma unroll
        for (int it = 0; it < NRED; it += 2) {
            const int J0 = rq + RS * it, J1 = J0 + RS;
            y0 = y0 + cs[min(J0, nt) * Wp + tr];
            if (it + 1 < NRED) y1 = y1 + cs[min(J1, nt) * Wp + tr];
        }
        cx<T> y = y0 + y1;
        y.re = lane_sum(y.re, RS);
        y.im = lane_sum(y.im, RS);
        return y;
    };

    Slot ring[PD + 1];
    c128 rr[PD + 1];
    cx<T> yr[PD + 1];
    cx<T> yv = zero();   // y (phase 0) or x (phase 1) of my row at the previous block row
    for (int c = tid; c < Wp; c += NT) cs[nt * Wp + c] = zero();   // row nt of c: the reduction's padding
    __syncthreads();     // ay, ax, zero tail of v, zero row of c
    iax = ax[tr];        // from LDS: no global load older than the ring is left for the loop to wait on

    if constexpr (PH == 0) {
        // ---- forward elimination of this half towards the middle row
        const int kstart = h == 0 ? kf0 : kf1;
        const int dir = h == 0 ? 1 : -1;
        const int n = h == 0 ? m - kf0 : kf1 - m;
        auto kat = [&](int i) { return kstart + dir * min(i, n - 1); };
        if (n > 0) {
#pragma unroll
            for (int p = 0; p < PD; ++p) {
                rr[p] = rhs_load(kat(p));
                load(kat(p), ring[p]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        cx<T> gnext = zero();   // v of the next step (owners)
        if (n > 0 && mine) gnext = rhs_use(kstart, rr[0]);
        auto fstep = [&](int i, int u) __attribute__((always_inline)) {
            const int k = kstart + dir * i;
            rr[(u + PD) % (PD + 1)] = rhs_load(kat(i + PD));
            load(kat(i + PD), ring[(u + PD) % (PD + 1)]);
            __builtin_amdgcn_sched_barrier(0);
            if (mine) v[tr] = gnext;
            __syncthreads();
            gemv(ring[u]);
            // the next step's coupling and right-hand side while the others finish
            const cx<T> cn = mine ? cy(h == 0 ? k : k - 1) : zero();
            const cx<T> rn = (mine && i + 1 < n) ? rhs_use(k + dir, rr[(u + 1) % (PD + 1)]) : zero();
            __syncthreads();
            const cx<T> y = reduce();
            if (mine) {
                yv = y;
                Yg[(size_t)k * W + tr] = y;
                gnext = rn - cn * y;
            }
        };
        int i0 = 0;
        for (; i0 + PD < n; i0 += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) fstep(i0 + u, u);
        }
#pragma unroll
        for (int u = 0; u < PD; ++u)
            if (i0 + u < n) fstep(i0 + u, u);
        return;
    }

    // ---- phase 1: middle row, then back substitution of this half away from it
    {
        Slot gm;
        load(m, gm);
        const c128 rm = rhs_load(m);
        const cx<T> ylo = (kf0 <= m - 1) ? yload(m - 1) : zero();
        const cx<T> yhi = (kf1 >= m + 1) ? yload(m + 1) : zero();
        if (mine) {
            cx<T> g = rhs_use(m, rm);
            if (m >= 1) g = g - cy(m - 1) * ylo;
            if (m + 1 <= H - 1) g = g - cy(m) * yhi;
            v[tr] = g;
        }
        __syncthreads();
        gemv(gm);
        __syncthreads();
        const cx<T> y = reduce();
        if (mine) {
            yv = y;
            Yg[(size_t)H * W + (size_t)m * W + tr] = y;
        }
    }
    {
        const int kstart = h == 0 ? m - 1 : m + 1;
        const int dir = h == 0 ? -1 : 1;
        const int n = h == 0 ? m - kb0 : kb1 - m;
        auto kat = [&](int i) { return kstart + dir * min(i, n - 1); };
        __syncthreads();   // every reduce of the middle row has read c
        __builtin_amdgcn_sched_barrier(0);
        if (n > 0) {
#pragma unroll
            for (int p = 0; p < PD; ++p) {
                yr[p] = yload(kat(p));
                load(kat(p), ring[p]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        cx<T> vnext = zero();
        if (n > 0 && mine) vnext = cy(h == 0 ? kstart : kstart - 1) * yv;
        auto bstep = [&](int i, int u) __attribute__((always_inline)) {
            const int k = kstart + dir * i;
            yr[(u + PD) % (PD + 1)] = yload(kat(i + PD));
            load(kat(i + PD), ring[(u + PD) % (PD + 1)]);
            __builtin_amdgcn_sched_barrier(0);
            if (mine) v[tr] = vnext;
            __syncthreads();
            gemv(ring[u]);
            const int kn = k + dir;
            const cx<T> cn = mine ? cy(h == 0 ? kn : kn - 1) : zero();
            // y of the bottom half is zero below kf0, that of the top half above kf1
            const cx<T> yk = (mine && (h == 0 ? k >= kf0 : k <= kf1)) ? yr[u] : zero();
            __syncthreads();
            const cx<T> x = reduce();
            if (mine) {
                yv = yk - x;
                Yg[(size_t)H * W + (size_t)k * W + tr] = yv;
                vnext = cn * yv;
            }
        };
        int i0 = 0;
        for (; i0 + PD < n; i0 += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) bstep(i0 + u, u);
        }
#pragma unroll
        for (int u = 0; u < PD; ++u)
            if (i0 + u < n) bstep(i0 + u, u);
    }
    __syncthreads();

    // ---- outputs of the block rows this half owns
    const int olo = h == 0 ? kb0 : max(kb0, m + 1);
    const int ohi = h == 0 ? min(kb1, m) : kb1;
    const cx<T>* X = Yg + (size_t)H * W;
    if constexpr (CS == CS_FINAL) {
        const int r0 = max(s.r0, olo), r1 = min(s.r1, ohi + 1);
        const int nc = s.c1 - s.c0, n = max(0, r1 - r0) * nc;
        c128* z = a.z + (size_t)rhs * N + (size_t)(s.wy0 + r0) * a.geo.Nx + s.wx0 + s.c0;
        for (int idx = tid; idx < n; idx += NT) {
            const int rr0 = idx / nc, cc = idx - rr0 * nc;
            z[(size_t)rr0 * a.geo.Nx + cc] = cvt<double>(X[(size_t)(r0 + rr0) * W + s.c0 + cc]);
        }
    } else {
        cx<T>* trp = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
        auto own = [&](int k) { return k >= olo && k <= ohi; };
        for (int o = 0; o < dref.nout; ++o) {
            const int side = dref.out_side[o];
            cx<T>* out = trp + dref.out_off[o];
            const bool acc = dref.out_acc[o] != 0;
            if (side == SIDE_B || side == SIDE_T) {
                const int l0 = (side == SIDE_B) ? s.r0 - 1 : s.r1 - 1;
                for (int idx = tid; idx < 2 * W; idx += NT) {
                    const int line = idx / W, c = idx - line * W;
                    if (!own(l0 + line)) continue;
                    const cx<T> xv = X[(size_t)(l0 + line) * W + c];
                    out[idx] = acc ? out[idx] + xv : xv;
                }
            } else {
                const int l0 = (side == SIDE_L) ? s.c0 - 1 : s.c1 - 1;
                for (int idx = tid; idx < 2 * H; idx += NT) {
                    const int line = idx / H, k = idx - line * H;
                    if (!own(k)) continue;
                    const cx<T> xv = X[(size_t)k * W + l0 + line];
                    out[idx] = acc ? out[idx] + xv : xv;
                }
            }
        }
    }
}

// Packed symmetric copy of the FP64 factor pool, rounded to T (tile layout of tile_nt): entry
// (r, c) is the mean of G_k[r][c] and G_k[c][r] (the computed inverse is symmetric up to
// rounding; the mean is the nearest symmetric matrix).
template <typename T>
__global__ void k_pack_sym(const SubDesc* subs, const c128* G, cx<T>* Gp) {
    const SubDesc s = subs[blockIdx.y];
    const int W = s.W, H = s.H, nt = tile_nt(W), NTL = tile_count(W);
    const long long per = sym_block(W), total = per * H;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(e / per);
        const int rem = (int)(e - (long long)k * per);
        const int u = rem / (2 * NTL), w = rem - u * 2 * NTL;
        const int tau = w >> 1, q = 2 * u + (w & 1);
        int I = 0, start = 0;
        while (I < nt - 1 && start + (nt - I) <= tau) {
            start += nt - I;
            ++I;
        }
        const int J = I + (tau - start);
        const int r = 4 * I + (q >> 2), c = 4 * J + (q & 3);
        c128 g = mk(0.0, 0.0);
        if (r < W && c < W) {
            const c128* Gk = G + s.g_off + (size_t)k * W * W;   // column-major: (row r, col c) at c*W + r
            g = 0.5 * (Gk[(size_t)c * W + r] + Gk[(size_t)r * W + c]);
        }
        Gp[s.gs_off + e] = cvt<T>(g);
    }
}

// Right-hand side of the final z solve of each window: r on Omega_ij plus the polarized
// sources g_s of all its sweep solves.  Every incoming trace keeps, after the application, the
// value its sweep solve read (each is written before it is consumed and never after), so the
// g_s are rebuilt here from the trace pool with the polarization maps tabulated at setup.
template <typename T>
__global__ void k_final_rhs(ChainArgs a) {
    const SubDesc s = a.subs[blockIdx.x];
    const int rhs = blockIdx.y;
    const int W = s.W, H = s.H;
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    const cx<T>* tr = reinterpret_cast<const cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
    const int* rp = a.frp + s.fw_off + blockIdx.x;
    c128* out = a.fw + (size_t)rhs * a.fw_stride + s.fw_off;
    // gridDim.z workgroups share a window
    const int chunk = (H * W + gridDim.z - 1) / gridDim.z;
    const int e0 = blockIdx.z * chunk, e1 = min(H * W, e0 + chunk);
    for (int idx = e0 + threadIdx.x; idx < e1; idx += blockDim.x) {
        const int k = idx / W, c = idx - k * W;
        c128 val = mk(0.0, 0.0);
        if (k >= s.r0 && k < s.r1 && c >= s.c0 && c < s.c1)
            val = a.r[(size_t)rhs * N + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0 + c];
        const int j1 = rp[idx + 1];
        for (int j = rp[idx]; j < j1; ++j) val = val + a.fcoef[j] * cvt<double>(tr[a.fpool[j]]);
        out[idx] = val;
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

// slot of window point (k, c) among the in-slot ranges of a sweep solve, -1 if none; a point on
// both a horizontal and a vertical trace line is looked up on the horizontal one first
__device__ inline int in_slot(const GemvSolve& d, const SubDesc& s, int k, int c) {
    const int kind = d.kind, W = s.W, H = s.H;
    const bool hB = kind == KIND_B || kind == KIND_BL || kind == KIND_BR;
    const bool hT = kind == KIND_T || kind == KIND_TR || kind == KIND_TL;
    const bool vL = kind == KIND_L || kind == KIND_BL || kind == KIND_TL;
    const bool vR = kind == KIND_R || kind == KIND_TR || kind == KIND_BR;
    auto member = [&](int sl) {
        for (int r = 0; r < d.nin; ++r)
            if (sl >= d.in_start[r] && sl < d.in_start[r] + d.in_len[r]) return true;
        return false;
    };
    if (hB || hT) {
        const int l0 = hB ? s.r0 - 1 : s.r1 - 1;
        if (k == l0 || k == l0 + 1) {
            const int sl = (hB ? 0 : 2 * W) + (k - l0) * W + c;
            if (member(sl)) return sl;
        }
    }
    if (vL || vR) {
        const int l0 = vL ? s.c0 - 1 : s.c1 - 1;
        if (c == l0 || c == l0 + 1) {
            const int sl = (vL ? 4 * W : 4 * W + 2 * H) + (c - l0) * H + k;
            if (member(sl)) return sl;
        }
    }
    return -1;
}

// Column e of the polarization map P_s of a sweep solve.  The polarized source (eq. DiscPol2)
// is linear in the incoming trace values: g_p = sum_q A_pq (chi_q - chi_p) u~_q over the
// neighbours q of p.  Column e is u~ at the point q of in-slot e (the in-slot set and the
// support of u~ coincide); its nonzeros are the neighbours p of q across the boundary of chi.
struct PolColumn {
    int np;
    int slot[4], point[4];
    c128 coef[4];
    long long pool;   // trace-pool offset of u~_q (relative to the right-hand side's pool)
};

__device__ inline PolColumn pol_column(const GemvSolve& d, const SubDesc& s, const Geometry& geo, int e) {
    PolColumn col;
    col.np = 0;
    int r = 0, off = e;
    while (off >= d.in_len[r]) { off -= d.in_len[r]; ++r; }
    const int sq = d.in_start[r] + off;
    const int W = s.W, H = s.H;
    if (sq < 4 * W) col.pool = d.in_h + (sq < 2 * W ? sq : sq - 2 * W);
    else col.pool = d.in_v + (sq < 4 * W + 2 * H ? sq - 4 * W : sq - 4 * W - 2 * H);
    int kq, cq;
    slot_point(s, sq, kq, cq);
    const double ih2 = 1.0 / (geo.h * geo.h);
    const Local<double> L = make_local<double>(s, d.kind, geo.tab, nullptr, nullptr, ih2);
    const bool chq = chi_of(L, kq, cq);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int kp = kq + (n == 2 ? -1 : n == 3 ? 1 : 0), cp = cq + (n == 0 ? -1 : n == 1 ? 1 : 0);
        if (kp < 0 || kp >= H || cp < 0 || cp >= W) continue;
        if (chi_of(L, kp, cp) == chq) continue;
        const int sl = in_slot(d, s, kp, cp);
        if (sl < 0) continue;
        const c128 A = n < 2 ? coup_x(geo.tab, s.tx, W, s.ty, min(cp, cq), kq, ih2)
                             : coup_y(geo.tab, s.tx, s.ty, H, cq, min(kp, kq), ih2);
        col.slot[col.np] = sl;
        col.point[col.np] = kp * W + cp;
        col.coef[col.np] = chq ? A : -A;   // A_pq (chi_q - chi_p)
        ++col.np;
    }
    return col;
}

// Q'_s[:, e] = sum over p of Q[out slots, slot(p)] P_s[p, e]: the trace-to-trace map of a sweep
// solve (its outgoing traces from its incoming ones), complex128.
__global__ void k_qprime(const GemvSolve* gsv, const SubDesc* subs, Geometry geo, const c128* Q, c128* Qp) {
    const GemvSolve& d = gsv[blockIdx.x];
    const SubDesc s = subs[d.sub];
    const int e = blockIdx.y;
    int total = 0;
    for (int r = 0; r < d.nin; ++r) total += d.in_len[r];
    if (e >= total) return;
    const PolColumn col = pol_column(d, s, geo, e);
    const c128* Qs = Q + s.q_off;
    // column pairs: entry (t, e) at (e / 2) * 2 ld + 2 t + e % 2, so that a lane loads the entries
    // of two columns at its row in one 16-byte access (complex64)
    c128* out = Qp + d.qp_off + (size_t)(e >> 1) * 2 * d.ld + (e & 1);
    for (int t = threadIdx.x; t < d.ld; t += blockDim.x) {
        if (t >= d.rows) {   // alignment padding
            out[2 * t] = mk(0.0, 0.0);
            continue;
        }
        int o = 0;
        while (o + 1 < d.nout && t >= d.row_base[o + 1]) ++o;
        const int side = d.out_side[o];
        const int sb = (side == SIDE_B) ? 0 : (side == SIDE_T) ? 2 * s.W : (side == SIDE_L) ? 4 * s.W : 4 * s.W + 2 * s.H;
        const int os = sb + t - d.row_base[o];
        c128 v = mk(0.0, 0.0);
        for (int j = 0; j < col.np; ++j) v = v + Qs[(size_t)col.slot[j] * s.L + os] * col.coef[j];
        out[2 * t] = v;
    }
}

// the polarization maps as terms (window point, trace-pool offset, coefficient)
__global__ void k_pmap(const GemvSolve* gsv, int max_nin, const SubDesc* subs, Geometry geo, PEntry* out) {
    const GemvSolve& d = gsv[blockIdx.x];
    const int e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= max_nin) return;
    PEntry* o = out + ((size_t)blockIdx.x * max_nin + e) * 4;
    int total = 0;
    for (int r = 0; r < d.nin; ++r) total += d.in_len[r];
    int np = 0;
    if (e < total) {
        const SubDesc s = subs[d.sub];
        const PolColumn col = pol_column(d, s, geo, e);
        np = col.np;
        for (int j = 0; j < np; ++j) {
            o[j].coef = col.coef[j];
            o[j].pool = col.pool;
            o[j].sub = d.sub;
            o[j].point = col.point[j];
        }
    }
    for (int j = np; j < 4; ++j) {
        o[j].coef = mk(0.0, 0.0);
        o[j].pool = 0;
        o[j].sub = -1;
        o[j].point = 0;
    }
}

// One dependency level of the trace-compressed sweeps (Alg. Scenario3 after stage 1): every
// work item of the level is one workgroup computing up to 64 outgoing trace values
// out = Q'_s[rows, :] u~ (one per lane, the waves splitting the input entries) for every
// right-hand side.  Levels are separate launches, so every trace an item reads or updates was
// completed by an earlier launch.  The first chunk's gather of u~ and the Q' loads depend only
// on the work item and are all issued at once, the gather first.  Right-hand sides go in chunks of four through every
// loaded Q' batch, and the Q' share of a wave stays in registers across the chunks when it
// fits, so a batch of sources reads Q' about nrhs/4 times.
template <typename T, int RC>   // RC: right-hand sides per pass over Q'
__global__ __launch_bounds__(512) void k_gemv(GemvArgs a) {
    constexpr int NT = 512, NW = NT / 64, KB = sizeof(T) == 4 ? 16 : 8, KP = KB / 2;
    __shared__ cx<T> gv[RC][4 * kMaxWindow + KB * NW];
    __shared__ cx<T> part[NW][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const GemvItem& it = a.items[blockIdx.x];
    const int nin = it.nin, ld = it.ld;
    const bool valid = lane < it.nrow;
    const cx<T>* Qb = reinterpret_cast<const cx<T>*>(a.Q) + it.qoff;
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(Qb, (uint32_t)((size_t)it.qlen * sizeof(cx<T>)));
    // the waves split the input entries in even-sized shares (column pairs of Q')
    const int per = (((nin + NW - 1) / NW) + 1) & ~1;
    const int i0 = wv * per, i1 = min(nin, i0 + per);
    const bool resident = per <= KB;   // the whole share of Q' stays in registers across rhs chunks
    const uint32_t lo = (uint32_t)lane * 2u * (uint32_t)sizeof(cx<T>);
    const uint32_t cs = (uint32_t)ld * 2u * (uint32_t)sizeof(cx<T>);
    // columns c, c + 1 (c even) of this wave's share at my row, or nothing (no overlap with the
    // next wave's share, no rows past the chunk)
    auto qoff = [&](int c) { return (valid && c < i1) ? lo + (uint32_t)(c >> 1) * cs : kOob; };
    // Gather of u~ (and of the outputs' old values when they are accumulated) for right-hand sides
    // rc0 .. rc0 + RC - 1, as buffer loads from the trace pool of each: input idx lies in range rg
    // when it is past the first rg ranges, at rng_off[rg] + idx - (lengths of ranges < rg) (unused
    // ranges have length 0); an input past nin or a right-hand side past the batch reads zero (kOob).
    // No load is guarded, so all of them are in flight together.
    constexpr int GI = (4 * kMaxWindow + KB * NW + NT - 1) / NT;   // gather loads per lane
    const int c1 = it.rng_len[0], c2 = c1 + it.rng_len[1], c3 = c2 + it.rng_len[2];
    const long long d0 = it.rng_off[0], d1 = it.rng_off[1] - c1, d2 = it.rng_off[2] - c2, d3 = it.rng_off[3] - c3;
    const uint32_t tbytes = (uint32_t)(a.trace_stride * sizeof(cx<T>));
    cx<T> gl[RC][GI], old[RC];
    auto gather = [&](int rc0) {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const bool live = rc0 + r < a.nrhs;
            const __amdgpu_buffer_rsrc_t tr =
                make_rsrc(reinterpret_cast<cx<T>*>(a.traces) + (size_t)(live ? rc0 + r : 0) * a.trace_stride, tbytes);
#pragma unroll
            for (int j = 0; j < GI; ++j) {
                const int idx = tid + NT * j;
                const long long e = (idx < c1 ? d0 : idx < c2 ? d1 : idx < c3 ? d2 : d3) + idx;
                gl[r][j] = bload<T>(tr, (live && idx < nin) ? (uint32_t)(e * (long long)sizeof(cx<T>)) : kOob);
            }
            const bool acc = live && it.out_acc && wv == 0;
            old[r] = bload<T>(tr, acc ? (uint32_t)((it.out_off + (valid ? lane : 0)) * (long long)sizeof(cx<T>)) : kOob);
        }
    };
    // the first chunk's gather before the Q' loads: waiting for it leaves those in flight
    gather(0);
    Pair<T> q[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) q[u] = bload2<T>(qr, qoff(i0 + 2 * u));
    // one chunk of right-hand sides, its gather already issued; the first chunk is peeled off the loop
    // so that the wait for its gather counts only the loads issued before the Q' loads
    auto chunk = [&](int rc0) __attribute__((always_inline)) {
        const int nrc = min(RC, a.nrhs - rc0);
        // (zero past nin, so that the tail of a wave's share adds nothing)
#pragma unroll
        for (int r = 0; r < RC; ++r)
#pragma unroll
            for (int j = 0; j < GI; ++j) {
                const int idx = tid + NT * j;
                if (idx < per * NW) gv[r][idx] = gl[r][j];
            }
        __syncthreads();
        cx<T> acc[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[r] = cx<T>{T(0), T(0)};
        for (int base = i0;;) {
            if (base != i0 || (rc0 > 0 && !resident)) {
#pragma unroll
                for (int u = 0; u < KP; ++u) q[u] = bload2<T>(qr, qoff(base + 2 * u));
            }
#pragma unroll
            for (int u = 0; u < KP; ++u)
                if (base + 2 * u < i0 + per) {
#pragma unroll
                    for (int r = 0; r < RC; ++r)
                        if (r < nrc) {
                            acc[r] = fma(acc[r], q[u].a, gv[r][base + 2 * u]);
                            acc[r] = fma(acc[r], q[u].b, gv[r][base + 2 * u + 1]);
                        }
                }
            base += KB;
            if (base >= i1) break;
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            if (r >= nrc) break;
            part[wv][lane] = acc[r];
            __syncthreads();
            if (wv == 0 && valid) {
                cx<T> val = part[0][lane];
#pragma unroll
                for (int w = 1; w < NW; ++w) val = val + part[w][lane];
                cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)(rc0 + r) * a.trace_stride;
                tr[it.out_off + lane] = it.out_acc ? old[r] + val : val;
            }
            __syncthreads();
        }
    };
    chunk(0);
    for (int rc0 = RC; rc0 < a.nrhs; rc0 += RC) {
        gather(rc0);
        chunk(rc0);
    }
}

__global__ void k_cast(const c128* src, c64* dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = c64{static_cast<float>(src[i].re), static_cast<float>(src[i].im)};
}

// ------------------------------------------------------------------ scenario 4 windows (Sec. 2.1)
// out = phi (.) r over nrhs vectors of N points (x fastest, then y, then z in 3D); phi = A(x) B(y)
// with A = a, or 1 - a for the CDD shifted along x (kx = 1), and B = b, or 1 - b for the CDD
// shifted along y (ky = 1), the same on every z plane
__global__ void k_window(const c128* r, c128* out, const double* wx, const double* wy, int kx, int ky, int Nx,
                         int Ny, size_t N, size_t total) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t pnt = i % N;
        const int x = (int)(pnt % Nx), y = (int)((pnt / Nx) % Ny);
        const double A = kx ? 1.0 - wx[x] : wx[x];
        const double B = ky ? 1.0 - wy[y] : wy[y];
        const double f = A * B;
        out[i] = c128{f * r[i].re, f * r[i].im};
    }
}

// z = ((z + a) + b) + c, entry by entry
__global__ void k_accumulate(c128* z, const c128* a, const c128* b, const c128* c, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        z[i] = ((z[i] + a[i]) + b[i]) + c[i];
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
// Reductions are two launches: workgroup partials, then one wave per sum adds them in a fixed order
// (a device-wide completion count would need an L2 write-back per workgroup on this chip); the
// Gram-Schmidt update can instead sum its own coefficients in every workgroup, in the same order.
__device__ inline c128 block_sum(c128 acc, c128* red) {
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    return red[0];
}

// partial[(rhs * nv + l) * nblk + blk] = sum over the points blk*256 + t + k*nblk*256 of conj(V_l) w
__global__ void k_dots_partial(DotsArgs a) {
    __shared__ c128 red[256];
    const int blk = blockIdx.x, l = blockIdx.y, rhs = blockIdx.z;
    const c128* V = a.V + ((size_t)l * a.vstride_l + (size_t)rhs * a.vstride_rhs);
    const c128* w = a.w + (size_t)rhs * a.wstride;
    c128 acc = mk(0.0, 0.0);
    for (size_t p = (size_t)blk * blockDim.x + threadIdx.x; p < a.N; p += (size_t)gridDim.x * blockDim.x)
        acc = acc + conj(V[p]) * w[p];
    const c128 part = block_sum(acc, red);
    if (threadIdx.x == 0) a.partial[((size_t)rhs * a.nv + l) * gridDim.x + blk] = part;
}

// pp[0] + ... + pp[n - 1] by one whole wave in a fixed order: lane i adds pp[i], pp[i + 64], ... in
// turn (four loads issued together per pass), then an xor butterfly over the 64 lanes, after which
// every lane holds the same bits (each level adds the same two values in either order)
__device__ inline c128 wave_finish(const c128* pp, int n, int lane) {
    c128 acc = mk(0.0, 0.0);
    for (int b0 = 0; b0 < n; b0 += 256) {
        c128 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + lane + 64 * j;
            const c128 x = pp[min(b, n - 1)];
            v[j] = b < n ? x : mk(0.0, 0.0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = acc + v[j];
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        acc.re += __shfl_xor(acc.re, m);
        acc.im += __shfl_xor(acc.im, m);
    }
    return acc;
}

// out[rhs * ostride + l] (+)= sum_blk partial ; one wave per (l, rhs), the order of wave_finish
__global__ __launch_bounds__(64) void k_dots_finish(const c128* partial, int nblk, int nv, c128* out, int ostride,
                                                    int accumulate) {
    const int l = blockIdx.x, rhs = blockIdx.y;
    const c128 sum = wave_finish(partial + ((size_t)rhs * nv + l) * nblk, nblk, threadIdx.x);
    if (threadIdx.x == 0) {
        c128* o = out + (size_t)rhs * ostride + l;
        *o = accumulate ? *o + sum : sum;
    }
}

// w -= sum_l V_l c_l (c = coefficients on the device, [rhs * cstride + l]; masked rhs skipped); with
// partial, also the workgroup partials of ||w||^2 after the update, partial[rhs * nblk + blk].
// FIN: the coefficients are first summed from the dot products' workgroup partials
// (a.cpart[(rhs * nv + l) * cnblk + b]) by the waves of every workgroup, as k_dots_finish sums them,
// into LDS; workgroup 0 also stores them (a.cout[rhs * costride + l], added when caccum), so that the
// dot products need no finishing launch of their own.
template <bool FIN>
__global__ __launch_bounds__(256) void k_gs_update(GsArgs a) {
    __shared__ c128 red[256];
    __shared__ c128 cl[FIN ? kGsFinishMax : 1];
    const int rhs = blockIdx.y;
    const bool on = !(a.active && !a.active[rhs]);
    const c128* cf;
    if constexpr (FIN) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int l = wv; l < a.nv; l += 4) {
            const c128 s = wave_finish(a.cpart + ((size_t)rhs * a.nv + l) * a.cnblk, a.cnblk, lane);
            if (lane == 0) {
                cl[l] = s;
                if (blockIdx.x == 0) {
                    c128* o = a.cout + (size_t)rhs * a.costride + l;
                    *o = a.caccum ? *o + s : s;
                }
            }
        }
        __syncthreads();
        cf = cl;
    } else {
        cf = a.coef + (size_t)rhs * a.cstride;
    }
    if (!on && !a.partial) return;
    c128* w = a.w + (size_t)rhs * a.wstride;
    c128 nacc = mk(0.0, 0.0);
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.N; p += (size_t)gridDim.x * blockDim.x) {
        c128 v = w[p];
        if (on) {
            c128 acc = mk(0.0, 0.0);
            for (int l = 0; l < a.nv; ++l)
                acc = acc + a.V[(size_t)l * a.vstride_l + (size_t)rhs * a.vstride_rhs + p] * cf[l];
            v = a.sign > 0 ? v + acc : v - acc;
            w[p] = v;
        }
        nacc = nacc + conj(v) * v;
    }
    if (!a.partial) return;
    const c128 part = block_sum(nacc, red);
    if (threadIdx.x == 0) a.partial[(size_t)rhs * gridDim.x + blockIdx.x] = part;
}

// All nv <= LC dot products <V_l, w> of one right-hand side in one pass over the points: w is read
// once instead of once per column.  Points, workgroups and the partial layout are those of
// k_dots_partial (same per-thread order, same tree), so the sums are bitwise the same.
template <int LC>
__global__ __launch_bounds__(256) void k_dots_w(DotsArgs a) {
    __shared__ c128 red[256];
    const int blk = blockIdx.x, rhs = blockIdx.y, nv = a.nv;
    const c128* V = a.V + (size_t)rhs * a.vstride_rhs;
    const c128* w = a.w + (size_t)rhs * a.wstride;
    c128 acc[LC];
#pragma unroll
    for (int l = 0; l < LC; ++l) acc[l] = mk(0.0, 0.0);
    for (size_t p = (size_t)blk * blockDim.x + threadIdx.x; p < a.N; p += (size_t)gridDim.x * blockDim.x) {
        const c128 wp = w[p];
#pragma unroll
        for (int l = 0; l < LC; ++l)
            if (l < nv) acc[l] = acc[l] + conj(V[(size_t)l * a.vstride_l + p]) * wp;
    }
#pragma unroll
    for (int l = 0; l < LC; ++l) {
        if (l < nv) {   // uniform
            const c128 part = block_sum(acc[l], red);
            if (threadIdx.x == 0) a.partial[((size_t)rhs * a.nv + l) * gridDim.x + blk] = part;
            __syncthreads();   // red[0] read before the next sum overwrites it
        }
    }
}

// The first Gram-Schmidt update fused with the second pass's dot products (CGS2): per point,
// w <- w + sign V c (as k_gs_update, active right-hand sides only) and then the partials of
// <V_l, w> of the updated w, with the V_l of the point still in registers, so V is read once for
// both.  Points, workgroups and the partial layout are those of k_dots_partial (d.nblk
// workgroups per right-hand side), so the partials are bitwise those of a separate pass.
template <int LC>
__global__ __launch_bounds__(256) void k_gs_dots(GsArgs g, DotsArgs d) {
    __shared__ c128 red[256];
    const int blk = blockIdx.x, rhs = blockIdx.y, nv = d.nv;
    const bool on = !(g.active && !g.active[rhs]);
    const c128* cf = g.coef + (size_t)rhs * g.cstride;
    const c128* V = g.V + (size_t)rhs * g.vstride_rhs;
    c128* w = g.w + (size_t)rhs * g.wstride;
    c128 c[LC], acc[LC];
#pragma unroll
    for (int l = 0; l < LC; ++l) {
        c[l] = l < nv ? cf[l] : mk(0.0, 0.0);
        acc[l] = mk(0.0, 0.0);
    }
    for (size_t p = (size_t)blk * blockDim.x + threadIdx.x; p < d.N; p += (size_t)gridDim.x * blockDim.x) {
        c128 v[LC];
#pragma unroll
        for (int l = 0; l < LC; ++l) v[l] = l < nv ? V[(size_t)l * g.vstride_l + p] : mk(0.0, 0.0);
        c128 wp = w[p];
        if (on) {
            c128 s = mk(0.0, 0.0);
#pragma unroll
            for (int l = 0; l < LC; ++l)
                if (l < nv) s = s + v[l] * c[l];
            wp = g.sign > 0 ? wp + s : wp - s;
            w[p] = wp;
        }
#pragma unroll
        for (int l = 0; l < LC; ++l)
            if (l < nv) acc[l] = acc[l] + conj(v[l]) * wp;
    }
#pragma unroll
    for (int l = 0; l < LC; ++l) {
        if (l < nv) {   // uniform
            const c128 part = block_sum(acc[l], red);
            if (threadIdx.x == 0) d.partial[((size_t)rhs * nv + l) * gridDim.x + blk] = part;
            __syncthreads();
        }
    }
}

// dst = src / sqrt(nrm2[rhs * nstride].re) (0 if the norm is 0), masked rhs skipped, grid-stride over
// the points.  FIN: the squared norm is first summed from the update's workgroup partials
// npart[rhs * nnblk + b] by one wave of every workgroup, as k_dots_finish sums them; workgroup 0
// stores it to nrm2[rhs * nstride].
template <bool FIN>
__global__ __launch_bounds__(256) void k_scale(const c128* src, c128* dst, c128* nrm2, int nstride, const int* active,
                                               size_t N, size_t sstride, size_t dstride, const c128* npart,
                                               int nnblk) {
    const int rhs = blockIdx.y;
    double n2 = 0.0;
    if constexpr (FIN) {
        __shared__ double sh;
        if (threadIdx.x < 64) {   // one whole wave
            const c128 s = wave_finish(npart + (size_t)rhs * nnblk, nnblk, threadIdx.x);
            if (threadIdx.x == 0) {
                sh = s.re;
                if (blockIdx.x == 0) nrm2[(size_t)rhs * nstride] = s;
            }
        }
        __syncthreads();
        n2 = sh;
    }
    if (active && !active[rhs]) return;
    if constexpr (!FIN) n2 = nrm2[(size_t)rhs * nstride].re;
    const double nr = sqrt(fmax(0.0, n2));
    const double s = nr > 0 ? 1.0 / nr : 0.0;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (size_t)gridDim.x * blockDim.x) {
        const c128 v = src[(size_t)rhs * sstride + p];
        dst[(size_t)rhs * dstride + p] = mk(s * v.re, s * v.im);
    }
}

// zero fill of n 16-byte words (a kernel rather than a memset node, so that a captured graph
// replays it like any other launch)
__global__ void k_zero16(uint4* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_conj(const c128* src, c128* dst, size_t n) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[p] = conj(src[p]);
}

__global__ void k_mass_gradient(const c128* lam, const c128* u, int nrhs, Geometry g, double* grad) {
    const size_t N = (size_t)g.Nx * g.Ny * g.Nz;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int x = (int)(p % g.Nx), y = (int)((p / g.Nx) % g.Ny), z = (int)(p / ((size_t)g.Nx * g.Ny));
    c128 w = g.tab[g.gtx + x] * g.tab[g.gty + y];   // 1/(alpha_x alpha_y) [ / alpha_z in 3D ]
    if (g.Nz > 1) w = w * g.tab[g.gtz + z];
    double acc = 0.0;
    for (int s = 0; s < nrhs; ++s) {
        const c128 t = lam[(size_t)s * N + p] * w * u[(size_t)s * N + p];
        acc += t.re;
    }
    grad[p] += g.omega * g.omega * acc;
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// prefetch depth: as many blocks in flight as the 128-VGPR budget of a 1024-thread
// workgroup allows (complex64: 2 floats, complex128: 4 per element)
// register-ring depth of the complex64 kernel at 8 elements per thread (blocks in flight)
constexpr int kPdF8 = 3;

template <typename T, int CS, bool YLDS, int PH>
static void launch_chain_c(const ChainArgs& a, dim3 grid, int ept, size_t lds, hipStream_t st) {
    constexpr bool dbl = sizeof(T) == 8;
    if (ept <= 4) k_chain<T, 4, 2, CS, YLDS, PH><<<grid, 1024, lds, st>>>(a);
    else if (ept <= 8) k_chain<T, 8, dbl ? 1 : kPdF8, CS, YLDS, PH><<<grid, 1024, lds, st>>>(a);
    else if (ept <= 16) k_chain<T, 16, dbl ? 0 : 1, CS, YLDS, PH><<<grid, 1024, lds, st>>>(a);
    else if (ept <= 32) k_chain<T, 32, 0, CS, YLDS, PH><<<grid, 1024, lds, st>>>(a);
    else k_chain<T, 64, 0, CS, YLDS, PH><<<grid, 1024, lds, st>>>(a);
}

template <typename T, int CS, int PH>
static hipError_t set_lds_one(int ept, size_t lds) {
    // dynamic LDS beyond the default needs the attribute on every instantiation that may run
    auto one = [&](const void* f) { return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); };
    constexpr bool dbl = sizeof(T) == 8;
    if (ept <= 4) return one((const void*)k_chain<T, 4, 2, CS, true, PH>);
    if (ept <= 8) return one((const void*)k_chain<T, 8, dbl ? 1 : kPdF8, CS, true, PH>);
    if (ept <= 16) return one((const void*)k_chain<T, 16, dbl ? 0 : 1, CS, true, PH>);
    if (ept <= 32) return one((const void*)k_chain<T, 32, 0, CS, true, PH>);
    return one((const void*)k_chain<T, 64, 0, CS, true, PH>);
}

template <typename T>
static hipError_t set_lds(int cs, int ept, size_t lds) {
    hipError_t e = hipSuccess;
#define LSW_SET(CSV)                                                         \
    if (cs == CSV) {                                                         \
        e = set_lds_one<T, CSV, 0>(ept, lds);                                \
        if (e == hipSuccess) e = set_lds_one<T, CSV, 1>(ept, lds);           \
    }
    LSW_SET(CS_STAGE1)
    LSW_SET(CS_FINAL)
    LSW_SET(CS_UNIT)
    LSW_SET(CS_POLAR)
#undef LSW_SET
    return e;
}

template <typename T>
static hipError_t launch_chain_t(const ChainArgs& a0, int nsolves, int nrhs, int ept, int cs, size_t ylds,
                                 hipStream_t st) {
    dim3 grid(2 * nsolves, nrhs);
    if (ylds > 0) {
        hipError_t e = set_lds<T>(cs, ept, ylds);
        if (e != hipSuccess) return e;
    }
    // phase 0 (forward halves), then phase 1 (middle row and backward halves): the kernel
    // boundary is where the two halves of every solve meet
#define LSW_GO(CSV, PHV)                                                                    \
    if (cs == CSV) {                                                                        \
        if (ylds > 0) launch_chain_c<T, CSV, true, PHV>(a0, grid, ept, ylds, st);           \
        else launch_chain_c<T, CSV, false, PHV>(a0, grid, ept, 0, st);                      \
    }
    LSW_GO(CS_STAGE1, 0) LSW_GO(CS_FINAL, 0) LSW_GO(CS_UNIT, 0) LSW_GO(CS_POLAR, 0)
    LSW_GO(CS_STAGE1, 1) LSW_GO(CS_FINAL, 1) LSW_GO(CS_UNIT, 1) LSW_GO(CS_POLAR, 1)
#undef LSW_GO
    return hipGetLastError();
}

hipError_t launch_chain(const ChainArgs& a, int nsolves, int nrhs, int ept, bool c64mode, int cs, size_t ylds,
                        hipStream_t st) {
    return c64mode ? launch_chain_t<float>(a, nsolves, nrhs, ept, cs, ylds, st)
                   : launch_chain_t<double>(a, nsolves, nrhs, ept, cs, ylds, st);
}

template <typename T, int CS, int R, int PH>
static void launch_chain_mr_c(const ChainArgs& a, dim3 grid, int ept, hipStream_t st) {
    constexpr bool dbl = sizeof(T) == 8;
    if (ept <= 4) k_chain_mr<T, 4, 2, CS, R, PH><<<grid, 1024, 0, st>>>(a);
    else if (ept <= 8) k_chain_mr<T, 8, dbl ? 1 : 2, CS, R, PH><<<grid, 1024, 0, st>>>(a);
    else if (ept <= 16) k_chain_mr<T, 16, dbl ? 0 : 1, CS, R, PH><<<grid, 1024, 0, st>>>(a);
    else if (ept <= 32) k_chain_mr<T, 32, 0, CS, R, PH><<<grid, 1024, 0, st>>>(a);
    else k_chain_mr<T, 64, 0, CS, R, PH><<<grid, 1024, 0, st>>>(a);
}

template <typename T>
static hipError_t launch_chain_mr_t(const ChainArgs& a0, int nsolves, int nrhs, int ept, int cs, int R,
                                    hipStream_t st) {
    dim3 grid(2 * nsolves, (nrhs + R - 1) / R);
    ChainArgs a = a0;
    a.nrhs = nrhs;
#define LSW_GO(CSV, RV, PHV) if (cs == CSV && R == RV) launch_chain_mr_c<T, CSV, RV, PHV>(a, grid, ept, st);
    LSW_GO(CS_STAGE1, 2, 0) LSW_GO(CS_STAGE1, 4, 0) LSW_GO(CS_FINAL, 2, 0) LSW_GO(CS_FINAL, 4, 0)
    LSW_GO(CS_STAGE1, 2, 1) LSW_GO(CS_STAGE1, 4, 1) LSW_GO(CS_FINAL, 2, 1) LSW_GO(CS_FINAL, 4, 1)
#undef LSW_GO
    return hipGetLastError();
}

// ------------------------------------------------------------------ many right-hand sides on matrix cores
// 16 x 16 x 4 matrix-core products in the working precision.  Lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator entry v is row l / 16 + 4 v (FP64) or 4 (l / 16) + v (FP32), column
// l % 16 (established by an in-bounds probe of both instructions).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    __device__ static inline acc mac(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static inline int row(int lk, int v) { return 4 * lk + v; }
};
template <>
struct Mfma<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    __device__ static inline acc mac(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
};

// The twisted block substitution of the stage-1 and final fronts for R = 16 RB right-hand sides per
// workgroup, each block step a matrix-core product Y = G_k V of the W x W block with the W x R block of
// right-hand-side columns, so that every G_k is read once per R right-hand sides and the arithmetic is
// dense: complex products as four real ones (Re += Gr Vr + (-Gi) Vi, Im += Gr Vi + Gi Vr).  Four waves
// share the row blocks of G_k (wave w owns 16-row blocks w, w + 4, ...); V lives in LDS, one row per
// window column x, R entries per row; thread x forms row x of V from the right-hand side and the
// previous block's y or x; y (phase 0) and x (phase 1) go to each right-hand side's slab of a.Y as in
// k_chain_mr, whose phases, ranges and outputs this kernel shares.  With CS_UNIT a workgroup carries
// a group of up to R unit solves of one subdomain (the columns of Q): right-hand side r is the unit
// vector at window point (unit_k, unit_c) of the group's r-th unit descriptor.
template <typename T, int CS, int RB, int PH, int QM>
__global__ __launch_bounds__(256) void k_chain_mma(ChainArgs a) {
    static_assert(CS == CS_STAGE1 || CS == CS_FINAL || CS == CS_UNIT, "stage-1, final and unit solves");
    constexpr int NT = 256, R = 16 * RB;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    const int sidx = blockIdx.x >> 1, h = blockIdx.x & 1, nsol = gridDim.x >> 1;
    const int ufirst = CS == CS_UNIT ? a.ugroups[4 * sidx] : sidx;
    const SolveDesc& dref = a.descs[ufirst];
    const int kf0 = CS == CS_UNIT ? a.ugroups[4 * sidx + 2] : dref.kf0;
    const int kf1 = CS == CS_UNIT ? a.ugroups[4 * sidx + 3] : dref.kf1;
    const int kb0 = dref.kb0, kb1 = dref.kb1;
    const SubDesc s = a.subs[dref.sub];
    const int rhs0 = blockIdx.y * R;
    const int nr = CS == CS_UNIT ? a.ugroups[4 * sidx + 1] : min(R, a.nrhs - rhs0);
    __shared__ int su_k[R], su_c[R];   // CS_UNIT: the unit point of each right-hand side
    if (CS == CS_UNIT && threadIdx.x < R) {
        su_k[threadIdx.x] = threadIdx.x < nr ? a.descs[ufirst + threadIdx.x].unit_k : -1;
        su_c[threadIdx.x] = threadIdx.x < nr ? a.descs[ufirst + threadIdx.x].unit_c : -1;
    }
    const int W = s.W, H = s.H, m = s.mid, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int NB = (W + 15) / 16;   // row blocks of 16, at most 4 QM (wave w owns w, w + 4, ...)
    // rows past W stay zero; one padding entry per row, so that the row owners (thread x updates
    // sV[x][.]) hit different LDS banks
    __shared__ cx<T> sV[kMaxWindow][R + 1];
    __shared__ c128 a2h[kMaxWindow + 1];
    const c128* tab = a.geo.tab;
    const double ih2 = 1.0 / (a.geo.h * a.geo.h);
    for (int k = tid; k <= H; k += NT) a2h[k] = tab[s.ty + H + k];
    for (int e = tid; e < kMaxWindow * R; e += NT) sV[e / R][e % R] = cx<T>{T(0), T(0)};
    const bool mine = tid < W;
    const c128 ia_c = tab[s.tx + (mine ? tid : 0)];
    const cx<T>* Gs = reinterpret_cast<const cx<T>*>(a.G) + s.g_off;
    const size_t N = (size_t)a.geo.Nx * a.geo.Ny;
    auto zero = []() { return cx<T>{T(0), T(0)}; };
    auto cy = [&](int l) { return cvt<T>(-ih2 * (a2h[l + 1] * ia_c)); };
    const bool in_cols = mine && tid >= s.c0 && tid < s.c1;
    // g_k at my column for right-hand side r (zero outside the ranges that carry it)
    auto rhs_at = [&](int r, int k) -> cx<T> {
        if (!mine || r >= nr || k < kf0 || k > kf1) return zero();
        const int rhs = rhs0 + r;
        if constexpr (CS == CS_UNIT) return (k == su_k[r] && tid == su_c[r]) ? cx<T>{T(1), T(0)} : zero();
        if constexpr (CS == CS_FINAL) return cvt<T>(a.fw[(size_t)rhs * a.fw_stride + s.fw_off + (size_t)k * W + tid]);
        if (!(in_cols && k >= s.r0 && k < s.r1)) return zero();
        return cvt<T>(a.r[(size_t)rhs * N + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0 + tid]);
    };
    auto slab = [&](int r) {
        const size_t j = CS == CS_UNIT ? (size_t)sidx * R + r : (size_t)(rhs0 + r) * nsol + sidx;
        return reinterpret_cast<cx<T>*>(a.Y) + j * a.Y_stride;
    };
    // rhs_at for the right-hand sides r0 .. r0 + 7 of an owner lane, with every load unconditional
    // (an entry outside the ranges reads a valid one of right-hand side rhs0 and is scaled by 0), so
    // that the eight are in flight together; guarded loads compile to one wait each
    auto rhs_at8 = [&](int r0, int k, cx<T>* g) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int r = r0 + u;
            if constexpr (CS == CS_UNIT) {
                g[u] = rhs_at(r, k);
            } else {
                bool ok = r < nr && k >= kf0 && k <= kf1;
                if constexpr (CS == CS_STAGE1) ok = ok && in_cols && k >= s.r0 && k < s.r1;
                const size_t rhs = (size_t)rhs0 + (r < nr ? r : 0);
                const c128 v = CS == CS_FINAL ? a.fw[rhs * a.fw_stride + s.fw_off + (size_t)k * W + tid]
                                              : a.r[rhs * N + (size_t)(s.wy0 + k) * a.geo.Nx + s.wx0 + tid];
                const double f = ok ? 1.0 : 0.0;
                g[u] = cvt<T>(c128{v.re * f, v.im * f});
            }
        }
    };

    acc_t accr[QM][RB], acci[QM][RB];
    // acc = G_k V over this wave's row blocks
    auto product = [&](int k) {
#pragma unroll
        for (int q = 0; q < QM; ++q)
#pragma unroll
            for (int bj = 0; bj < RB; ++bj) {
                accr[q][bj] = acc_t{T(0), T(0), T(0), T(0)};
                acci[q][bj] = acc_t{T(0), T(0), T(0), T(0)};
            }
        const cx<T>* Gk = Gs + (size_t)k * W * W;
        // 32 columns of G_k per round (24 in complex128): the loads of all U k-steps are issued
        // before their products, so a block step waits for memory once per round instead of once
        // per 4 columns; the columns of V come from LDS at the product.  Both keep a wave within
        // 256 registers, so two waves share a SIMD
        constexpr int U = sizeof(T) == 8 ? 6 : 8;
        for (int c0 = 0; c0 < W; c0 += 4 * U) {
            cx<T> g[U][QM];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = c0 + 4 * u + lk;
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    const int row = 16 * (wv + 4 * q) + li;
                    g[u][q] = (c < W && row < W) ? Gk[(size_t)c * W + row] : zero();
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool live = c0 + 4 * u < W;   // the same for the whole wave
                if (!live) break;
                const int c = c0 + 4 * u + lk;
                cx<T> vb[RB];
#pragma unroll
                for (int bj = 0; bj < RB; ++bj) vb[bj] = sV[c < W ? c : kMaxWindow - 1][16 * bj + li];
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    if (wv + 4 * q >= NB) break;
#pragma unroll
                    for (int bj = 0; bj < RB; ++bj) {
                        // rows c >= W of V are zero, so padded columns add nothing
                        const T gr = g[u][q].re, gi = g[u][q].im, vr = vb[bj].re, vi = vb[bj].im;
                        accr[q][bj] = M::mac(gr, vr, accr[q][bj]);
                        accr[q][bj] = M::mac(-gi, vi, accr[q][bj]);
                        acci[q][bj] = M::mac(gr, vi, acci[q][bj]);
                        acci[q][bj] = M::mac(gi, vr, acci[q][bj]);
                    }
                }
            }
        }
    };
    // the product's entries (row x, right-hand side r) into sV and slab[r][off + x]; with `minus`, the
    // result is y_k - product (y_k from slab[r][k W + x] when has_y)
    auto store = [&](size_t off, bool minus, int k, bool has_y) {
        // with `minus`, the y entries first, all loads unconditional (an entry outside reads a valid one
        // and is scaled by 0) so that they are in flight together
        cx<T> yv[QM][RB][4];
        if (minus) {
#pragma unroll
            for (int q = 0; q < QM; ++q)
#pragma unroll
                for (int bj = 0; bj < RB; ++bj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int x = 16 * (wv + 4 * q) + M::row(lk, v), r = 16 * bj + li;
                        const bool ok = has_y && r < nr && x < W && wv + 4 * q < NB;
                        const cx<T> t = slab(r < nr ? r : 0)[(size_t)k * W + (x < W ? x : 0)];
                        const T f = ok ? T(1) : T(0);
                        yv[q][bj][v] = cx<T>{t.re * f, t.im * f};
                    }
        }
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            if (wv + 4 * q >= NB) break;
#pragma unroll
            for (int bj = 0; bj < RB; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int x = 16 * (wv + 4 * q) + M::row(lk, v), r = 16 * bj + li;
                    if (x >= W) continue;
                    cx<T> val = cx<T>{accr[q][bj][v], acci[q][bj][v]};
                    if (minus) val = yv[q][bj][v] - val;
                    sV[x][r] = val;
                    if (r < nr) slab(r)[off + x] = val;
                }
        }
    };
    __syncthreads();

    if constexpr (PH == 0) {
        // ---- forward elimination of this half towards the middle row
        const int kstart = h == 0 ? kf0 : kf1;
        const int dir = h == 0 ? 1 : -1;
        const int n = h == 0 ? m - kf0 : kf1 - m;
        for (int i = 0; i < n; ++i) {
            const int k = kstart + dir * i;
            if (mine) {
                const cx<T> c = cy(h == 0 ? k - 1 : k);
                for (int r0 = 0; r0 < R; r0 += 8) {
                    cx<T> g8[8];
                    rhs_at8(r0, k, g8);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        cx<T> g = g8[u];
                        if (i > 0) g = g - c * sV[tid][r0 + u];
                        sV[tid][r0 + u] = g;
                    }
                }
            }
            __syncthreads();
            product(k);
            __syncthreads();
            store((size_t)k * W, false, k, false);
            __syncthreads();
        }
        return;
    }

    // ---- phase 1: middle row, then back substitution of this half away from it
    if (mine) {
#pragma unroll 4
        for (int r = 0; r < R; ++r) {
            cx<T> g = rhs_at(r, m);
            if (r < nr) {
                if (m >= 1 && kf0 <= m - 1) g = g - cy(m - 1) * slab(r)[(size_t)(m - 1) * W + tid];
                if (m + 1 <= H - 1 && kf1 >= m + 1) g = g - cy(m) * slab(r)[(size_t)(m + 1) * W + tid];
            }
            sV[tid][r] = g;
        }
    }
    __syncthreads();
    product(m);
    __syncthreads();
    store((size_t)H * W + (size_t)m * W, false, m, false);
    __syncthreads();
    {
        const int kstart = h == 0 ? m - 1 : m + 1;
        const int dir = h == 0 ? -1 : 1;
        const int n = h == 0 ? m - kb0 : kb1 - m;
        for (int i = 0; i < n; ++i) {
            const int k = kstart + dir * i;
            if (mine) {
                const cx<T> c = cy(h == 0 ? k : k - 1);
#pragma unroll 4
                for (int r = 0; r < R; ++r) sV[tid][r] = c * sV[tid][r];
            }
            __syncthreads();
            product(k);
            __syncthreads();
            store((size_t)H * W + (size_t)k * W, true, k, h == 0 ? k >= kf0 : k <= kf1);
            __syncthreads();
        }
    }

    // ---- outputs of the block rows this half owns
    const int olo = h == 0 ? kb0 : max(kb0, m + 1);
    const int ohi = h == 0 ? min(kb1, m) : kb1;
    auto own = [&](int k) { return k >= olo && k <= ohi; };
    for (int r = 0; r < nr; ++r) {
        const int rhs = rhs0 + r;
        const cx<T>* X = slab(r) + (size_t)H * W;
        if constexpr (CS == CS_UNIT) {
            // Q column: the solution at the trace-line slots (B, T lines of W, then L, R lines of H)
            cx<T>* col = reinterpret_cast<cx<T>*>(a.Q) + a.descs[ufirst + r].q_col;
            const int L8 = 4 * W + 4 * H;
            for (int sl = tid; sl < L8; sl += NT) {
                int k, c, side;
                if (sl < 4 * W) {
                    const int line = sl / W;
                    c = sl - line * W;
                    side = line < 2 ? SIDE_B : SIDE_T;
                    k = line == 0 ? s.r0 - 1 : line == 1 ? s.r0 : line == 2 ? s.r1 - 1 : s.r1;
                } else {
                    const int q = sl - 4 * W, line = q / H;
                    k = q - line * H;
                    side = line < 2 ? SIDE_L : SIDE_R;
                    c = line == 0 ? s.c0 - 1 : line == 1 ? s.c0 : line == 2 ? s.c1 - 1 : s.c1;
                }
                if (((s.sides >> side) & 1) && own(k)) col[sl] = X[(size_t)k * W + c];
            }
        } else if constexpr (CS == CS_FINAL) {
            const int r0 = max(s.r0, olo), r1 = min(s.r1, ohi + 1);
            const int nc = s.c1 - s.c0, n = max(0, r1 - r0) * nc;
            c128* z = a.z + (size_t)rhs * N + (size_t)(s.wy0 + r0) * a.geo.Nx + s.wx0 + s.c0;
            for (int idx = tid; idx < n; idx += NT) {
                const int rr0 = idx / nc, cc = idx - rr0 * nc;
                z[(size_t)rr0 * a.geo.Nx + cc] = cvt<double>(X[(size_t)(r0 + rr0) * W + s.c0 + cc]);
            }
        } else {
            cx<T>* tr = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs * a.trace_stride;
            for (int o = 0; o < dref.nout; ++o) {
                const int side = dref.out_side[o];
                cx<T>* out = tr + dref.out_off[o];
                const bool acc = dref.out_acc[o] != 0;
                if (side == SIDE_B || side == SIDE_T) {
                    const int l0 = (side == SIDE_B) ? s.r0 - 1 : s.r1 - 1;
                    for (int idx = tid; idx < 2 * W; idx += NT) {
                        const int line = idx / W, c = idx - line * W;
                        if (!own(l0 + line)) continue;
                        const cx<T> xv = X[(size_t)(l0 + line) * W + c];
                        out[idx] = acc ? out[idx] + xv : xv;
                    }
                } else {
                    const int l0 = (side == SIDE_L) ? s.c0 - 1 : s.c1 - 1;
                    for (int idx = tid; idx < 2 * H; idx += NT) {
                        const int line = idx / H, k = idx - line * H;
                        if (!own(k)) continue;
                        const cx<T> xv = X[(size_t)k * W + l0 + line];
                        out[idx] = acc ? out[idx] + xv : xv;
                    }
                }
            }
        }
    }
}

// The sweep levels for many right-hand sides on matrix cores: per work item (at most 64 output
// rows of one sweep solve) out[rows x R] = Q'[rows x nin] U[nin x R], U the incoming trace values
// of R = 16 RB right-hand sides, gathered into LDS in chunks of KC inputs (zero past nin and past
// the batch); wave w owns the 16-row block w.  Q' (column-pair layout of k_gemv) is read once per
// item for all R right-hand sides, where k_gemv reads it once per chunk of 4.  Complex products as
// four real ones; the outputs are written (or added, out_acc) as in k_gemv.
template <typename T, int RB>
__global__ __launch_bounds__(256) void k_gemv_mma(GemvArgs a) {
    constexpr int NT = 256, R = 16 * RB, KC = 64;
    // LDS row stride: the four 16-entry rows one MFMA step reads fall in different banks (float)
    constexpr int SR = (sizeof(T) == 4 && R == 32) ? 48 : R;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    __shared__ T sUr[KC][SR], sUi[KC][SR];
    const GemvItem& it = a.items[blockIdx.x];
    const int rhs0 = blockIdx.y * R, nr = min(R, a.nrhs - rhs0);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int nin = it.nin, ld = it.ld, nrow = it.nrow;
    const __amdgpu_buffer_rsrc_t qr =
        make_rsrc(reinterpret_cast<const cx<T>*>(a.Q) + it.qoff, (uint32_t)((size_t)it.qlen * sizeof(cx<T>)));
    const int row = 16 * wv + li;   // the A-operand row of this lane
    // Q'[row][k] sits at (k / 2) 2 ld + 2 row + k % 2; rows past the item read nothing
    auto qload = [&](int k) -> cx<T> {
        const uint32_t off = (row < nrow && k < nin)
                                 ? (uint32_t)(((size_t)(k >> 1) * 2 * ld + 2 * row + (k & 1)) * sizeof(cx<T>))
                                 : kOob;
        return bload<T>(qr, off);
    };
    acc_t accr[RB], acci[RB];
#pragma unroll
    for (int bj = 0; bj < RB; ++bj) {
        accr[bj] = acc_t{T(0), T(0), T(0), T(0)};
        acci[bj] = acc_t{T(0), T(0), T(0), T(0)};
    }
    // The gather of a chunk: lane l of wave w reads input e = l of the chunk for the right-hand sides
    // w, w + 4, ... of the group (consecutive lanes, consecutive inputs of one right-hand side).  Input
    // i lies in range rg when it is past the first rg ranges, at rng_off[rg] + i - (lengths of ranges
    // < rg) (unused ranges have length 0).  Every load is a buffer load over one right-hand side's trace
    // pool that reads zero past the inputs or the batch (kOob), so the GJ of a lane are in flight together.
    constexpr int GJ = KC * R / NT;
    static_assert(KC == 64 && NT == 256, "one input per lane, four right-hand sides per pass");
    const int c1 = it.rng_len[0], c2 = c1 + it.rng_len[1], c3 = c2 + it.rng_len[2];
    const long long d0 = it.rng_off[0], d1 = it.rng_off[1] - c1, d2 = it.rng_off[2] - c2, d3 = it.rng_off[3] - c3;
    const uint32_t tbytes = (uint32_t)(a.trace_stride * sizeof(cx<T>));
    for (int c0 = 0; c0 < nin; c0 += KC) {
        const int kc = min(KC, nin - c0);
        {
            const int e = lane, ie = c0 + e;
            const long long off = (ie < c1 ? d0 : ie < c2 ? d1 : ie < c3 ? d2 : d3) + ie;
            cx<T> g[GJ];
#pragma unroll
            for (int j = 0; j < GJ; ++j) {
                const int r = wv + 4 * j;   // the same for the whole wave
                const __amdgpu_buffer_rsrc_t tr = make_rsrc(
                    reinterpret_cast<const cx<T>*>(a.traces) + (size_t)(rhs0 + (r < nr ? r : 0)) * a.trace_stride, tbytes);
                g[j] = bload<T>(tr, (r < nr && e < kc) ? (uint32_t)(off * (long long)sizeof(cx<T>)) : kOob);
            }
#pragma unroll
            for (int j = 0; j < GJ; ++j) {
                sUr[e][wv + 4 * j] = g[j].re;
                sUi[e][wv + 4 * j] = g[j].im;
            }
        }
        __syncthreads();
        // 16 inputs per round: the four Q' loads are issued before their products
        for (int k16 = 0; k16 < kc; k16 += 16) {
            cx<T> qv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) qv[u] = qload(c0 + k16 + 4 * u + lk);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = k16 + 4 * u + lk;
                if (k16 + 4 * u >= kc) break;
#pragma unroll
                for (int bj = 0; bj < RB; ++bj) {
                    const T ur = sUr[e][16 * bj + li], ui = sUi[e][16 * bj + li];
                    accr[bj] = M::mac(qv[u].re, ur, accr[bj]);
                    accr[bj] = M::mac(-qv[u].im, ui, accr[bj]);
                    acci[bj] = M::mac(qv[u].re, ui, acci[bj]);
                    acci[bj] = M::mac(qv[u].im, ur, acci[bj]);
                }
            }
        }
        __syncthreads();
    }
    // accumulator entry v of lane l: row M::row(l / 16, v) of the wave's block, column l % 16
    cx<T>* trw = reinterpret_cast<cx<T>*>(a.traces) + (size_t)rhs0 * a.trace_stride;
#pragma unroll
    for (int bj = 0; bj < RB; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int orow = 16 * wv + M::row(lk, v), col = 16 * bj + li;
            if (orow < nrow && col < nr) {
                cx<T>* t = trw + (size_t)col * a.trace_stride + it.out_off + orow;
                const cx<T> val{accr[bj][v], acci[bj][v]};
                *t = it.out_acc ? *t + val : val;
            }
        }
}

hipError_t launch_gemv_mma(const GemvArgs& a, bool c64mode, hipStream_t st) {
    if (a.nitems <= 0) return hipSuccess;
    if (c64mode) {
        if (a.nrhs > 16) k_gemv_mma<float, 2><<<dim3(a.nitems, (a.nrhs + 31) / 32), 256, 0, st>>>(a);
        else k_gemv_mma<float, 1><<<dim3(a.nitems, 1), 256, 0, st>>>(a);
    } else {
        k_gemv_mma<double, 1><<<dim3(a.nitems, (a.nrhs + 15) / 16), 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

// QM: row blocks of 16 per wave, 3 for windows up to 192 points wide, 4 up to kMaxWindow (fewer
// accumulators leave room for two waves per SIMD)
template <typename T, int CS, int RB>
static void launch_chain_mma_c(const ChainArgs& a, dim3 grid, int wmax, hipStream_t st) {
    if (wmax <= 192) {
        k_chain_mma<T, CS, RB, 0, 3><<<grid, 256, 0, st>>>(a);
        k_chain_mma<T, CS, RB, 1, 3><<<grid, 256, 0, st>>>(a);
    } else {
        k_chain_mma<T, CS, RB, 0, 4><<<grid, 256, 0, st>>>(a);
        k_chain_mma<T, CS, RB, 1, 4><<<grid, 256, 0, st>>>(a);
    }
}

hipError_t launch_chain_mma_unit(const ChainArgs& a, int ngroups, int wmax, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    launch_chain_mma_c<double, CS_UNIT, 1>(a, dim3(2 * ngroups, 1), wmax, st);
    return hipGetLastError();
}

hipError_t launch_chain_mma(const ChainArgs& a0, int nsolves, int nrhs, bool c64mode, int cs, int R, int wmax,
                            hipStream_t st) {
    if ((cs != 0 && cs != 1) || (R != 16 && R != 32) || (!c64mode && R != 16)) return hipErrorInvalidValue;
    ChainArgs a = a0;
    a.nrhs = nrhs;
    const dim3 grid(2 * nsolves, (nrhs + R - 1) / R);
    if (c64mode) {
        if (cs == 0) R == 16 ? launch_chain_mma_c<float, CS_STAGE1, 1>(a, grid, wmax, st) : launch_chain_mma_c<float, CS_STAGE1, 2>(a, grid, wmax, st);
        else R == 16 ? launch_chain_mma_c<float, CS_FINAL, 1>(a, grid, wmax, st) : launch_chain_mma_c<float, CS_FINAL, 2>(a, grid, wmax, st);
    } else {
        if (cs == 0) launch_chain_mma_c<double, CS_STAGE1, 1>(a, grid, wmax, st);
        else launch_chain_mma_c<double, CS_FINAL, 1>(a, grid, wmax, st);
    }
    return hipGetLastError();
}

hipError_t launch_chain_mr(const ChainArgs& a, int nsolves, int nrhs, int ept, bool c64mode, int cs, int rgroup,
                           hipStream_t st) {
    if ((cs != 0 && cs != 1) || (rgroup != 2 && rgroup != 4)) return hipErrorInvalidValue;
    return c64mode ? launch_chain_mr_t<float>(a, nsolves, nrhs, ept, cs, rgroup, st)
                   : launch_chain_mr_t<double>(a, nsolves, nrhs, ept, cs, rgroup, st);
}

// k_chain_sym in the shape kSymCfgs[cfg] (a tile is 32 VGPRs in complex64 and 64 in complex128;
// with 512 lanes two waves share a SIMD, so a wave keeps at most 256 registers: the shapes listed
// are those that compile without spills)
template <int CS, int PH, typename F>
static void sym_dispatch(int cfg, F&& f) {
    switch (cfg) {
        case 0: f(k_chain_sym<float, 256, 1, 3, 4, CS, PH>); break;
        case 1: f(k_chain_sym<float, 256, 1, 3, 2, CS, PH>); break;
        case 2: f(k_chain_sym<float, 512, 1, 3, 4, CS, PH>); break;
        case 3: f(k_chain_sym<float, 512, 1, 2, 4, CS, PH>); break;
        case 4: f(k_chain_sym<float, 256, 2, 2, 2, CS, PH>); break;
        case 5: f(k_chain_sym<float, 256, 3, 1, 1, CS, PH>); break;
        case 6: f(k_chain_sym<float, 512, 2, 1, 2, CS, PH>); break;
        case 7: f(k_chain_sym<double, 256, 1, 2, 4, CS, PH>); break;
        case 8: f(k_chain_sym<double, 256, 1, 2, 2, CS, PH>); break;
        case 9: f(k_chain_sym<double, 512, 1, 1, 4, CS, PH>); break;
        default: break;
    }
}
static_assert(kSymCfgCount == 10, "sym_dispatch covers every shape of kSymCfgs");

hipError_t prepare_chain_sym(int cfg, size_t lds) {
    if (cfg < 0 || cfg >= kSymCfgCount) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    auto set = [&](auto kern) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
    sym_dispatch<CS_STAGE1, 0>(cfg, set); sym_dispatch<CS_STAGE1, 1>(cfg, set);
    sym_dispatch<CS_FINAL, 0>(cfg, set); sym_dispatch<CS_FINAL, 1>(cfg, set);
    return e;
}

hipError_t launch_chain_sym(const ChainArgs& a, int nsolves, int nrhs, int cfg, int cs, size_t lds, hipStream_t st) {
    if ((cs != CS_STAGE1 && cs != CS_FINAL) || cfg < 0 || cfg >= kSymCfgCount) return hipErrorInvalidValue;
    const dim3 grid(2 * nsolves, nrhs);
    const int nt = kSymCfgs[cfg].threads;
    auto go = [&](auto kern) { kern<<<grid, nt, lds, st>>>(a); };
    if (cs == CS_STAGE1) {
        sym_dispatch<CS_STAGE1, 0>(cfg, go);
        sym_dispatch<CS_STAGE1, 1>(cfg, go);
    } else {
        sym_dispatch<CS_FINAL, 0>(cfg, go);
        sym_dispatch<CS_FINAL, 1>(cfg, go);
    }
    return hipGetLastError();
}

hipError_t launch_pack_sym(const SubDesc* subs, int nsub, const c128* G, void* Gp, bool c64mode, hipStream_t st) {
    if (nsub <= 0) return hipSuccess;
    dim3 grid(256, nsub);
    if (c64mode) k_pack_sym<float><<<grid, 256, 0, st>>>(subs, G, reinterpret_cast<c64*>(Gp));
    else k_pack_sym<double><<<grid, 256, 0, st>>>(subs, G, reinterpret_cast<c128*>(Gp));
    return hipGetLastError();
}

hipError_t launch_gemv(const GemvArgs& a, bool c64mode, hipStream_t st) {
    if (a.nitems <= 0) return hipSuccess;
    // measured on lens2d: the complex64 single-rhs variant is fastest with RC = 1; the
    // complex128 kernel is faster with RC = 4 even for one rhs (0.20 vs 0.26 ms per apply)
    if (c64mode) {
        if (a.nrhs == 1) k_gemv<float, 1><<<a.nitems, 512, 0, st>>>(a);
        else k_gemv<float, 4><<<a.nitems, 512, 0, st>>>(a);
    } else {
        k_gemv<double, 4><<<a.nitems, 512, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_final_rhs(const ChainArgs& a, int nsub, int nrhs, bool c64mode, hipStream_t st) {
    dim3 grid(nsub, nrhs, 32);   // about one window point per lane at W = H = 88
    if (c64mode) k_final_rhs<float><<<grid, 256, 0, st>>>(a);
    else k_final_rhs<double><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_qprime(const GemvSolve* gs, int ngs, int max_nin, const SubDesc* subs, const Geometry& geo,
                         const c128* Q, c128* Qp, hipStream_t st) {
    if (ngs == 0 || max_nin == 0) return hipSuccess;
    k_qprime<<<dim3(ngs, max_nin), 256, 0, st>>>(gs, subs, geo, Q, Qp);
    return hipGetLastError();
}

hipError_t launch_pmap(const GemvSolve* gs, int ngs, int max_nin, const SubDesc* subs, const Geometry& geo,
                       PEntry* out, hipStream_t st) {
    if (ngs == 0 || max_nin == 0) return hipSuccess;
    k_pmap<<<dim3(ngs, (max_nin + 255) / 256), 256, 0, st>>>(gs, max_nin, subs, geo, out);
    return hipGetLastError();
}

hipError_t launch_cast(const c128* src, c64* dst, size_t n, hipStream_t st) {
    k_cast<<<2048, 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_window(const c128* r, c128* out, const double* wx, const double* wy, int kx, int ky, int Nx,
                         int Ny, size_t N, int nrhs, hipStream_t st) {
    const size_t total = N * (size_t)nrhs;
    k_window<<<(unsigned)std::min<size_t>(4096, blocks_for(total, 256)), 256, 0, st>>>(r, out, wx, wy, kx, ky, Nx,
                                                                                      Ny, N, total);
    return hipGetLastError();
}

hipError_t launch_accumulate(c128* z, const c128* a, const c128* b, const c128* c, size_t n, hipStream_t st) {
    k_accumulate<<<(unsigned)std::min<size_t>(4096, blocks_for(n, 256)), 256, 0, st>>>(z, a, b, c, n);
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

hipError_t launch_dots(const DotsArgs& a, int nrhs, hipStream_t st) {
    k_dots_partial<<<dim3(a.nblk, a.nv, nrhs), 256, 0, st>>>(a);
    k_dots_finish<<<dim3(a.nv, nrhs), 64, 0, st>>>(a.partial, a.nblk, a.nv, a.out, a.ostride, a.accumulate);
    return hipGetLastError();
}

hipError_t launch_dots_partial(const DotsArgs& a, int nrhs, hipStream_t st) {
    k_dots_partial<<<dim3(a.nblk, a.nv, nrhs), 256, 0, st>>>(a);
    return hipGetLastError();
}

template <typename F>
static bool with_lc(int nv, F f) {
    if (nv <= 4) f(std::integral_constant<int, 4>{});
    else if (nv <= 8) f(std::integral_constant<int, 8>{});
    else if (nv <= 16) f(std::integral_constant<int, 16>{});
    else if (nv <= kFusedGsMax) f(std::integral_constant<int, kFusedGsMax>{});
    else return false;
    return true;
}

hipError_t launch_dots_w(const DotsArgs& a, int nrhs, hipStream_t st) {
    if (!with_lc(a.nv, [&](auto lc) { k_dots_w<decltype(lc)::value><<<dim3(a.nblk, nrhs), 256, 0, st>>>(a); }))
        return hipErrorInvalidValue;
    k_dots_finish<<<dim3(a.nv, nrhs), 64, 0, st>>>(a.partial, a.nblk, a.nv, a.out, a.ostride, a.accumulate);
    return hipGetLastError();
}

hipError_t launch_gs_dots(const GsArgs& g, const DotsArgs& d, int nrhs, hipStream_t st) {
    if (g.nv != d.nv) return hipErrorInvalidValue;
    if (!with_lc(d.nv, [&](auto lc) { k_gs_dots<decltype(lc)::value><<<dim3(d.nblk, nrhs), 256, 0, st>>>(g, d); }))
        return hipErrorInvalidValue;
    k_dots_finish<<<dim3(d.nv, nrhs), 64, 0, st>>>(d.partial, d.nblk, d.nv, d.out, d.ostride, d.accumulate);
    return hipGetLastError();
}

hipError_t launch_gs_update(const GsArgs& a, int nrhs, hipStream_t st) {
    if (a.partial && !a.norm_out && a.nblk > kScaleFinishMax) return hipErrorInvalidValue;
    if (a.cpart) {
        // the norm's partials must not share memory with the coefficients' partials read by the launch
        if (a.nv > kGsFinishMax || a.partial == a.cpart) return hipErrorInvalidValue;
        k_gs_update<true><<<dim3(a.nblk, nrhs), 256, 0, st>>>(a);
    } else {
        k_gs_update<false><<<dim3(a.nblk, nrhs), 256, 0, st>>>(a);
    }
    if (a.partial && a.norm_out)
        k_dots_finish<<<dim3(1, nrhs), 64, 0, st>>>(a.partial, a.nblk, 1, a.norm_out, a.nstride, 0);
    return hipGetLastError();
}

hipError_t launch_scale(const c128* src, c128* dst, const c128* nrm2, int nstride, const int* active, size_t N,
                        size_t sstride, size_t dstride, int nrhs, hipStream_t st) {
    dim3 grid(blocks_for(N, 256), nrhs);
    k_scale<false><<<grid, 256, 0, st>>>(src, dst, const_cast<c128*>(nrm2), nstride, active, N, sstride, dstride,
                                         nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_scale_partials(const c128* src, c128* dst, const c128* npart, int nnblk, c128* nrm2, int nstride,
                                 const int* active, size_t N, size_t sstride, size_t dstride, int nrhs,
                                 hipStream_t st) {
    if (nnblk < 1 || nnblk > kScaleFinishMax) return hipErrorInvalidValue;
    // at most 1024 workgroups per right-hand side, each summing the partials once
    dim3 grid((unsigned)std::min<size_t>(blocks_for(N, 256), 1024), nrhs);
    k_scale<true><<<grid, 256, 0, st>>>(src, dst, nrm2, nstride, active, N, sstride, dstride, npart, nnblk);
    return hipGetLastError();
}

hipError_t launch_zero16(void* p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    k_zero16<<<(unsigned)std::min<size_t>(2048, blocks_for(n, 256)), 256, 0, st>>>(reinterpret_cast<uint4*>(p), n);
    return hipGetLastError();
}

hipError_t launch_conj(const c128* src, c128* dst, size_t n, hipStream_t st) {
    k_conj<<<blocks_for(n, 256), 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_mass_gradient(const c128* lam, const c128* u, int nrhs, const Geometry& g, double* grad,
                                hipStream_t st) {
    const size_t N = (size_t)g.Nx * g.Ny * g.Nz;
    k_mass_gradient<<<blocks_for(N, 256), 256, 0, st>>>(lam, u, nrhs, g, grad);
    return hipGetLastError();
}

}  // namespace lsw
