// Host runtime and C ABI of the L-sweeps library.
//
//  - CDD partition and local windows (Sec. 2.1-2.2): bulk points split as evenly as
//    possible, edge groups owning the global PML, windows grown by 2 overlap lines and
//    n_pml_local PML lines on every interior side.
//  - PML tables (App. A): 1/alpha at integer points and alpha at half points, global
//    and per window (global sigma plus the local cubic layers).
//  - Front schedule of Alg. Scenario3 (App. C): stage 1; the four cardinal sweeps run
//    together (each reads only stage-1 traces and writes its own arrays); the four
//    diagonal sweeps run together (each reads only cardinal outputs), one anti-diagonal
//    per front.  Every front is one launch of the batched local-solve kernel.
//  - Flexible GMRES (Sec. 3, Phase 3), right preconditioned, CGS2 on the device in FP64,
//    Givens least squares on the host, true-residual stop test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>


#include "launch.h"
#include "launch3d.h"
#include "lsw.h"

using namespace lsw;
using cd = std::complex<double>;

namespace {

enum HArr { H_B_RUN = 0, H_T_RUN, H_B_LF, H_T_LF, H_B_RT, H_T_RT, H_COUNT };
enum VArr { V_L_RUN = 0, V_R_RUN, V_R_UP, V_L_UP, V_R_DN, V_L_DN, V_COUNT };

// One dependent step of an application: a batch of block substitutions (descs[offset..])
// or a trace-compressed batch (gsolves/gitems).
struct Front {
    int gemv;
    int offset, count;           // solves
    int ioffset, icount;         // GEMV work items
};

}  // namespace

struct lsw_plan {
    // problem
    int nx = 0, ny = 0, px = 0, py = 0, q = 0, r = 0, pl = 0, e = 0;
    int Nx = 0, Ny = 0;
    size_t N = 0;
    double h = 0, omega = 0, C = 0;
    int precision = LSW_FP64, restart = 50, maxit = 500, nrhs_max = 1, sweep_mode = LSW_SWEEP_COMPRESSED;
    // 3D (beam CDD): nz bulk / pz PML points along z, Nz extended; planes of up to Smax points
    int dim = 2, nz = 1, pz = 0, Nz = 1, Smax = 0;
    void* d_rhs3 = nullptr;     // [nrhs][front slot][Nz][Smax] right-hand sides of a front
    void* d_Y3 = nullptr;       // same layout: y then x
    double tol = 1e-6;
    hipStream_t stream = nullptr;
    // geometry
    std::vector<int> xlo, xhi, ylo, yhi, xw0, xw1, yw0, yw1;
    std::vector<SubDesc> subs;
    std::vector<SolveDesc> descs;
    std::vector<Front> fronts;
    std::vector<GemvSolve> gsolves;
    std::vector<GemvItem> gitems;
    int Wmax = 0, Hmax = 0, max_front = 0, ept = 1;
    size_t ylds = 0, ylds128 = 0;   // LDS bytes for y/x in the block substitutions (0: global scratch)
    size_t HT = 0, VT = 0;
    std::vector<size_t> hbase, vbase;
    // device
    double* d_m = nullptr;
    c128* d_tab = nullptr;
    SubDesc* d_subs = nullptr;
    SolveDesc* d_descs = nullptr;
    GemvSolve* d_gsolves = nullptr;
    GemvItem* d_gitems = nullptr;
    void* d_Q = nullptr;
    size_t Q_elems = 0;
    size_t QP_elems = 0;          // Q' pool (what the sweeps read)
    int max_nin = 0;
    int sweep_depth = 0;            // dependency levels of the sweep work items (one launch each)
    int rgroup = 1;                 // right-hand sides per workgroup of the stage-1 / final substitutions
    double rgroup_ms[5] = {0, 0, 0, 0, 0};   // timings of R = 1, 2, 4, 16, 32 when tuned
    bool gemv_mma = false;                    // sweep levels of several right-hand sides on matrix cores
    int gs_fused = -1;                        // Gram-Schmidt in three sweeps over V: 1, four: 0, by size: -1
    int gs_finish_max = kGsFinishMax;         // four sweeps: the update sums its coefficients up to this many
    double gemv_ms[2] = {0, 0};               // setup timings of the sweep levels: k_gemv, k_gemv_mma
    int* d_frp = nullptr;           // final right-hand side: polarization terms per window point
    long long* d_fpool = nullptr;
    c128* d_fcoef = nullptr;
    c128* d_fw = nullptr;
    size_t FWT = 0;
    void* d_G = nullptr;
    size_t G_elems = 0;
    // packed symmetric factors (2D): the stage-1 and final substitutions of one right-hand side
    // per workgroup read these; d_G (full blocks) stays only where something else needs it
    bool gsym = false;
    int sym_cfg = -1;               // shape of the packed substitutions (kSymCfgs index)
    double sym_tune_best_ms = 0, sym_tune_worst_ms = 0;
    int sym_timed = 0;              // shapes timed at setup
    size_t sym_lds = 0;             // dynamic LDS of the packed substitutions: the widest window's column sums
    void* d_Gs = nullptr;
    size_t GS_elems = 0;
    int ptiles3 = 0;                // 3D packed: tiles per plane of the largest block
    size_t pack3_max = 0;           // 3D packed: largest packed pool of one beam (entries)
    void* d_P3 = nullptr;           // 3D packed: partial products of a step
    void* d_traces = nullptr;
    size_t trace_stride = 0;
    void* d_zpart = nullptr;
    size_t zpart_stride = 0;
    void* d_Y = nullptr;
    size_t Y_stride = 0;
    int* d_xgroup = nullptr;
    int* d_ygroup = nullptr;
    int* d_status = nullptr;
    Geometry geo{};
    // Krylov workspace
    c128* d_V = nullptr;
    c128* d_Z = nullptr;
    c128* d_w = nullptr;
    c128* d_partial = nullptr;
    c128* d_npart = nullptr;        // [nrhs][gsblk] norm partials while d_partial holds dot-product partials
    c128* d_hbuf = nullptr;
    c128* d_coef = nullptr;
    c128* d_tmp1 = nullptr;
    c128* d_tmp2 = nullptr;
    int* d_active = nullptr;
    std::vector<int> dev_active;    // what d_active holds
    c128* h_hbuf = nullptr;   // pinned
    int* h_active = nullptr;
    c128* h_coef = nullptr;
    int nblk = 256;                 // workgroups per (column, rhs) of the Krylov dot products
    int gsblk = 256;                // workgroups per rhs of the Gram-Schmidt updates (grid-stride)
    // bookkeeping
    std::vector<void*> allocs;
    std::string err;
    double t_setup_ms = 0, t_factor_ms = 0, t_q_ms = 0, last_apply_ms = 0, last_chain_ms = 0, last_gemv_ms = 0;
    double apply_chain_bytes = 0, apply_gemv_bytes = 0, factor_flops = 0;
    int chain_launches = 0, gemv_launches = 0;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double last_stage1_ms = 0, last_final_ms = 0, last_final_rhs_ms = 0;
    // the dominant kernel of a timed application (2D: the final substitutions; 3D: the plane
    // steps' k_tile3 / k_step3 launches, bracketed one by one by the event pairs kev[2i], kev[2i+1])
    std::vector<hipEvent_t> kev;
    size_t kev_used = 0;
    double last_dom_ms = 0, dom_bytes = 0;
    int dom_launches = 0;
    // lsw_apply_noalloc: this GPU's scratch array and the bytes of each per-application buffer
    // (sized for nrhs_max, as the handle's own buffers)
    void* d_scratch = nullptr;
    size_t sz_traces = 0, sz_Y = 0, sz_fw = 0, sz_zpart = 0, sz_rhs3 = 0, sz_Y3 = 0, sz_P3 = 0;
    double apply_stage1_bytes = 0, apply_final_bytes = 0;
    double apply_stage1_full_bytes = 0, apply_final_full_bytes = 0;   // the same on the full blocks
    // scenario 4 (Sec. 2.1): this plan is the unshifted CDD; shifted[] holds the CDDs shifted along
    // x, y and both, each a complete plan without a Krylov basis (member = true)
    int windows = 0, shift_x = 0, shift_y = 0;
    bool member = false;
    lsw_plan* shifted[3] = {nullptr, nullptr, nullptr};
    double* d_wx = nullptr;         // a(x) on the Nx extended points
    double* d_wy = nullptr;         // b(y) on the Ny extended points
    c128* d_wr[4] = {nullptr, nullptr, nullptr, nullptr};   // windowed right-hand sides of each CDD [nrhs][N]
    c128* d_wz[3] = {nullptr, nullptr, nullptr};            // the shifted CDDs' sweep results [nrhs][N]
    hipEvent_t evw[2] = {nullptr, nullptr};   // start and end of a windowed application
    // the shifted CDDs run on streams of their own (default priority), forked from and joined to
    // the caller's stream by events, so that their latency-bound launches overlap
    hipStream_t own_stream = nullptr;         // a member's stream (created by the windowed plan)
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_spin = nullptr;   // polled by the Krylov loop's waits
    hipEvent_t ev_step[2] = {nullptr, nullptr};   // end of the column copy of Arnoldi step k (slot k % 2)
    int* h_act_stage = nullptr;     // pinned [2][nrhs_max] staging of the mask copies
    int act_slot = 0;
    void* (*ualloc)(size_t, void*) = nullptr;   // the caller's device allocator (optional)
    void (*ufree)(void*, void*) = nullptr;
    void* uctx = nullptr;
};

namespace {

std::string g_setup_error;

#define HIPCK(plan, expr)                                                        \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            (plan)->err = std::string(#expr) + ": " + hipGetErrorString(e_);     \
            return LSW_EHIP;                                                     \
        }                                                                        \
    } while (0)

// device workspace: the caller's allocator when given, else hipMalloc
template <typename T>
int dalloc(lsw_plan* p, T** out, size_t count) {
    void* ptr = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    if (p->ualloc) {
        ptr = p->ualloc(bytes, p->uctx);
        if (!ptr) {
            p->err = "the caller's allocator returned no memory for " + std::to_string(bytes) + " bytes";
            return LSW_ENOMEM;
        }
    } else {
        hipError_t e = hipMalloc(&ptr, bytes);
        if (e != hipSuccess) {
            p->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
            return LSW_ENOMEM;
        }
    }
    p->allocs.push_back(ptr);
    *out = static_cast<T*>(ptr);
    return LSW_OK;
}

void release_mem(lsw_plan* p, void* ptr) {
    if (p->ufree) p->ufree(ptr, p->uctx);
    else (void)hipFree(ptr);
}

// frees one buffer once the plan's stream has finished with it (hipFree waits by itself; a
// caller's allocator may hand the memory out again at once)
void dfree(lsw_plan* p, void* ptr) {
    if (!ptr) return;
    auto it = std::find(p->allocs.begin(), p->allocs.end(), ptr);
    if (it != p->allocs.end()) p->allocs.erase(it);
    if (p->ufree) (void)hipStreamSynchronize(p->stream);
    release_mem(p, ptr);
}

void free_plan(lsw_plan* p) {
    if (!p) return;
    for (lsw_plan*& c : p->shifted) {
        free_plan(c);
        c = nullptr;
    }
    if (p->ufree) (void)hipStreamSynchronize(p->stream);   // own_stream for a member
    for (void* a : p->allocs) release_mem(p, a);
    if (p->h_hbuf) (void)hipHostFree(p->h_hbuf);
    if (p->h_active) (void)hipHostFree(p->h_active);
    if (p->h_coef) (void)hipHostFree(p->h_coef);
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->evw)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
    if (p->ev_spin) (void)hipEventDestroy(p->ev_spin);
    for (hipEvent_t e : p->ev_step)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->kev)
        if (e) (void)hipEventDestroy(e);
    if (p->h_act_stage) (void)hipHostFree(p->h_act_stage);
    delete p;
}

// ---------------------------------------------------------------- geometry
// groups of one axis.  shift > 0 gives a shifted CDD of scenario 4: every group start of the even
// split, the first bulk point included, moves by shift points towards larger indices, so the axis
// has one more group (the first holds the PML and shift bulk points)
void split(int n_bulk, int n_pml, int groups, std::vector<int>& lo, std::vector<int>& hi, int shift = 0) {
    std::vector<int> bounds;
    int start = n_pml;
    for (int g = 0; g < groups; ++g) {
        if (g > 0 || shift > 0) bounds.push_back(start + shift);
        start += n_bulk / groups + (g < n_bulk % groups ? 1 : 0);
    }
    lo.assign(1, 0);
    lo.insert(lo.end(), bounds.begin(), bounds.end());
    hi = bounds;
    hi.push_back(n_bulk + 2 * n_pml);
}

// the window a of one axis (scenario 4): 0 on the trace lines of the interfaces at lo[g] - 1/2
// (g >= 1), 1 on those of the shifted interfaces at los[g] - 1/2, a linear ramp w(d) / (w(d) + w(d'))
// with w(t) = max(0, t - 1) between them; beyond the first and the last interface it takes the
// value of the nearest one's kind
std::vector<double> axis_window(int N, const std::vector<int>& lo, const std::vector<int>& los) {
    std::vector<double> a(N);
    double first = 1e300, last = -1e300;
    for (size_t g = 1; g < lo.size(); ++g) first = std::min(first, lo[g] - 0.5), last = std::max(last, lo[g] - 0.5);
    for (size_t g = 1; g < los.size(); ++g) first = std::min(first, los[g] - 0.5), last = std::max(last, los[g] - 0.5);
    for (int x = 0; x < N; ++x) {
        double d = 1e300, ds = 1e300;
        for (size_t g = 1; g < lo.size(); ++g) d = std::min(d, std::fabs(x - (lo[g] - 0.5)));
        for (size_t g = 1; g < los.size(); ++g) ds = std::min(ds, std::fabs(x - (los[g] - 0.5)));
        if (x < first || x > last) {
            a[x] = ds < d ? 1.0 : 0.0;
        } else {
            const double w = std::max(0.0, d - 1.0), ws = std::max(0.0, ds - 1.0);
            a[x] = w / (w + ws);
        }
    }
    return a;
}

double sigma_cubic(double dist, double delta, double C) {
    if (delta <= 0.0 || dist <= 0.0) return 0.0;
    const double t = dist / delta;
    return (C / delta) * t * t * t;
}

// coordinate of integer point a (2a even) or half point a - 1/2 (pass 2a - 1) on an axis
double coord2(int twice_a, int n_pml, double h) { return (0.5 * twice_a - n_pml + 1) * h; }

// 1/alpha and alpha for sigma at coordinate x on axis (n, p), plus optional local layers
struct AxisLayers {
    double L, delta;          // bulk [0, L], global layer width
    bool left, right;         // local layers present
    double xs_left, xs_right; // layer starts (sigma = 0 there)
    double delta_loc;
};

double sigma_at(const AxisLayers& a, double x, double C) {
    double s = 0.0;
    if (a.delta > 0) s += sigma_cubic(std::max(0.0, std::max(-x, x - a.L)), a.delta, C);
    if (a.left) s += sigma_cubic(a.xs_left - x, a.delta_loc, C);
    if (a.right) s += sigma_cubic(x - a.xs_right, a.delta_loc, C);
    return s;
}

// append the table of points [w0, w1) of an axis to the pool; returns its offset
int append_table(std::vector<c128>& pool, int w0, int w1, int n_pml, double h, double omega, double C,
                 const AxisLayers& lay) {
    const int off = (int)pool.size();
    for (int a = w0; a < w1; ++a) {
        const double s = sigma_at(lay, coord2(2 * a, n_pml, h), C);
        pool.push_back(c128{1.0, s / omega});                     // 1/alpha = 1 + i sigma/omega
    }
    for (int a = w0; a <= w1; ++a) {
        const double s = sigma_at(lay, coord2(2 * a - 1, n_pml, h), C);
        const cd alpha = 1.0 / cd(1.0, s / omega);
        pool.push_back(c128{alpha.real(), alpha.imag()});
    }
    return off;
}

void add_out(SolveDesc& d, long long off, int side, int acc) {
    d.out_off[d.nout] = off;
    d.out_side[d.nout] = side;
    d.out_acc[d.nout] = acc;
    d.nout++;
}

// Block rows where the right-hand side of a local solve can be nonzero ([kf0, kf1]) and
// where its solution is read ([kb0, kb1]): stage 1 has data on Omega only, a sweep solve on
// its incoming trace lines (the full height for a vertical interface, the receiving
// quadrant for an L-shaped one), and the final solve is read on Omega only.
SolveDesc blank(const SubDesc& s, int sub, int kind, int zpart) {
    SolveDesc d;
    std::memset(&d, 0, sizeof(d));
    d.sub = sub;
    d.kind = kind;
    d.zpart = zpart;
    d.in_h = -1;
    d.in_v = -1;
    const int H = s.H;
    int kf0 = 0, kf1 = H - 1, kb0 = 0, kb1 = H - 1;
    switch (kind) {
        case KIND_STAGE1: kf0 = s.r0; kf1 = s.r1 - 1; break;
        case KIND_FINAL: kb0 = s.r0; kb1 = s.r1 - 1; break;
        case KIND_B: kf0 = s.r0 - 1; kf1 = s.r0; kb0 = s.r0; break;
        case KIND_T: kf0 = s.r1 - 1; kf1 = s.r1; break;
        case KIND_BL: case KIND_BR: kf0 = s.r0 - 1; kb0 = s.r0; break;
        case KIND_TR: case KIND_TL: kf1 = s.r1; break;
        default: break;
    }
    d.kf0 = kf0;
    d.kf1 = kf1;
    d.kb0 = kb0;
    d.kb1 = kb1;
    return d;
}

void build_schedule(lsw_plan* p) {
    const int q = p->q, r = p->r;
    auto sid = [&](int i, int j) { return i * r + j; };
    auto offH = [&](int a, int i, int j) { return (long long)(a * p->HT + p->hbase[sid(i, j)]); };
    auto offV = [&](int b, int i, int j) {
        return (long long)(H_COUNT * p->HT + b * p->VT + p->vbase[sid(i, j)]);
    };
    p->descs.clear();
    p->fronts.clear();
    auto push_front = [&](std::vector<SolveDesc>& f) {
        if (f.empty()) return;
        p->fronts.push_back(Front{0, (int)p->descs.size(), (int)f.size(), 0, 0});
        p->descs.insert(p->descs.end(), f.begin(), f.end());
        p->max_front = std::max(p->max_front, (int)f.size());
    };
    std::vector<SolveDesc> f;
    // stage 1 (addLocSols): all subdomains
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < r; ++j) {
            const SubDesc& s = p->subs[sid(i, j)];
            SolveDesc d = blank(s, sid(i, j), KIND_STAGE1, 0);
            if (i > 0) add_out(d, offH(H_B_RUN, i, j), SIDE_B, 0);
            if (i < q - 1) add_out(d, offH(H_T_RUN, i, j), SIDE_T, 0);
            if (j > 0) add_out(d, offV(V_L_RUN, i, j), SIDE_L, 0);
            if (j < r - 1) add_out(d, offV(V_R_RUN, i, j), SIDE_R, 0);
            f.push_back(d);
        }
    push_front(f);
    // cardinal sweeps, one row / column step per front
    const int nc = std::max(q, r) - 1;
    for (int t = 0; t < nc; ++t) {
        f.clear();
        if (t + 1 <= q - 1) {  // up: row i = t+1, incoming bottom trace T_run(i-1, j)
            const int i = t + 1;
            for (int j = 0; j < r; ++j) {
                const SubDesc& s = p->subs[sid(i, j)];
                SolveDesc d = blank(s, sid(i, j), KIND_B, 1);
                d.in_h = offH(H_T_RUN, i - 1, j);
                if (i < q - 1) add_out(d, offH(H_T_RUN, i, j), SIDE_T, 1);
                if (j < r - 1) add_out(d, offV(V_R_UP, i, j), SIDE_R, 0);
                if (j > 0) add_out(d, offV(V_L_UP, i, j), SIDE_L, 0);
                f.push_back(d);
            }
        }
        if (q - 2 - t >= 0) {  // down: row i = q-2-t, incoming top trace B_run(i+1, j)
            const int i = q - 2 - t;
            for (int j = 0; j < r; ++j) {
                const SubDesc& s = p->subs[sid(i, j)];
                SolveDesc d = blank(s, sid(i, j), KIND_T, 2);
                d.in_h = offH(H_B_RUN, i + 1, j);
                if (i > 0) add_out(d, offH(H_B_RUN, i, j), SIDE_B, 1);
                if (j < r - 1) add_out(d, offV(V_R_DN, i, j), SIDE_R, 0);
                if (j > 0) add_out(d, offV(V_L_DN, i, j), SIDE_L, 0);
                f.push_back(d);
            }
        }
        if (t + 1 <= r - 1) {  // right: column j = t+1, incoming left trace R_run(i, j-1)
            const int j = t + 1;
            for (int i = 0; i < q; ++i) {
                SolveDesc d = blank(p->subs[sid(i, j)], sid(i, j), KIND_L, 3);
                d.in_v = offV(V_R_RUN, i, j - 1);
                if (j < r - 1) add_out(d, offV(V_R_RUN, i, j), SIDE_R, 1);
                if (i > 0) add_out(d, offH(H_B_RT, i, j), SIDE_B, 0);
                if (i < q - 1) add_out(d, offH(H_T_RT, i, j), SIDE_T, 0);
                f.push_back(d);
            }
        }
        if (r - 2 - t >= 0) {  // left: column j = r-2-t, incoming right trace L_run(i, j+1)
            const int j = r - 2 - t;
            for (int i = 0; i < q; ++i) {
                SolveDesc d = blank(p->subs[sid(i, j)], sid(i, j), KIND_R, 4);
                d.in_v = offV(V_L_RUN, i, j + 1);
                if (j > 0) add_out(d, offV(V_L_RUN, i, j), SIDE_L, 1);
                if (i > 0) add_out(d, offH(H_B_LF, i, j), SIDE_B, 0);
                if (i < q - 1) add_out(d, offH(H_T_LF, i, j), SIDE_T, 0);
                f.push_back(d);
            }
        }
        push_front(f);
    }
    // diagonal sweeps, one anti-diagonal per front, inputs bound as in Alg. Scenario3
    const int nd = (q - 1) + (r - 1) - 1;
    for (int dd = 0; dd < nd; ++dd) {
        f.clear();
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < r; ++j) {
                const SubDesc& s = p->subs[sid(i, j)];
                if (i >= 1 && j >= 1 && (i - 1) + (j - 1) == dd) {  // BL->TR (R^up, T^right)
                    SolveDesc d = blank(s, sid(i, j), KIND_BL, 5);
                    d.in_h = offH(H_T_RT, i - 1, j);
                    d.in_v = offV(V_R_UP, i, j - 1);
                    if (j < r - 1) add_out(d, offV(V_R_UP, i, j), SIDE_R, 1);
                    if (i < q - 1) add_out(d, offH(H_T_RT, i, j), SIDE_T, 1);
                    f.push_back(d);
                }
                if (i <= q - 2 && j <= r - 2 && (q - 2 - i) + (r - 2 - j) == dd) {  // TR->BL (L^down, B^left)
                    SolveDesc d = blank(s, sid(i, j), KIND_TR, 6);
                    d.in_h = offH(H_B_LF, i + 1, j);
                    d.in_v = offV(V_L_DN, i, j + 1);
                    if (j > 0) add_out(d, offV(V_L_DN, i, j), SIDE_L, 1);
                    if (i > 0) add_out(d, offH(H_B_LF, i, j), SIDE_B, 1);
                    f.push_back(d);
                }
                if (i >= 1 && j <= r - 2 && (i - 1) + (r - 2 - j) == dd) {  // BR->TL (L^up, T^left)
                    SolveDesc d = blank(s, sid(i, j), KIND_BR, 7);
                    d.in_h = offH(H_T_LF, i - 1, j);
                    d.in_v = offV(V_L_UP, i, j + 1);
                    if (j > 0) add_out(d, offV(V_L_UP, i, j), SIDE_L, 1);
                    if (i < q - 1) add_out(d, offH(H_T_LF, i, j), SIDE_T, 1);
                    f.push_back(d);
                }
                if (i <= q - 2 && j >= 1 && (q - 2 - i) + (j - 1) == dd) {  // TL->BR (R^down, B^right)
                    SolveDesc d = blank(s, sid(i, j), KIND_TL, 8);
                    d.in_h = offH(H_B_RT, i + 1, j);
                    d.in_v = offV(V_R_DN, i, j - 1);
                    if (j < r - 1) add_out(d, offV(V_R_DN, i, j), SIDE_R, 1);
                    if (i > 0) add_out(d, offH(H_B_RT, i, j), SIDE_B, 1);
                    f.push_back(d);
                }
            }
        push_front(f);
    }
}

// slot ranges that carry the polarized right-hand side of each kind (the sets Gamma_1 and
// Gamma_2 of eq. DiscPol2, each point once; the corner point of an L-shaped interface is
// taken on its horizontal leg)
void in_ranges(const SubDesc& s, int kind, GemvSolve& g) {
    const int W = s.W, H = s.H, r0 = s.r0, r1 = s.r1, c0 = s.c0, c1 = s.c1;
    const int B0 = 0, B1 = W, T0 = 2 * W, T1 = 3 * W, L0 = 4 * W, L1 = 4 * W + H, R0 = 4 * W + 2 * H,
              R1 = 4 * W + 3 * H;
    g.nin = 0;
    auto add = [&](int start, int len) {
        if (len <= 0) return;
        g.in_start[g.nin] = start;
        g.in_len[g.nin] = len;
        g.nin++;
    };
    switch (kind) {
        case KIND_B: add(B0, 2 * W); break;
        case KIND_T: add(T0, 2 * W); break;
        case KIND_L: add(L0, 2 * H); break;
        case KIND_R: add(R0, 2 * H); break;
        case KIND_BL: add(B0 + c0, W - c0); add(B1 + c0, W - c0); add(L0 + r0, H - r0); add(L1 + r0 + 1, H - r0 - 1); break;
        case KIND_BR: add(B0, c1); add(B1, c1); add(R0 + r0 + 1, H - r0 - 1); add(R1 + r0, H - r0); break;
        case KIND_TR: add(T0, c1); add(T1, c1); add(R0, r1 - 1); add(R1, r1); break;
        case KIND_TL: add(T0 + c0, W - c0); add(T1 + c0, W - c0); add(L0, r1); add(L1, r1 - 1); break;
        default: break;
    }
}

int fail(lsw_plan* p, int code, const std::string& msg) {
    p->err = msg;
    return code;
}

// Chained sweep mode (3D, and 2D with sweep_mode = chain): the sweep solves of the fronts above
// regrouped by data flow, as compress_schedule groups the compressed sweeps.  A solve waits for the
// last writer of every trace it reads or updates (stage 1 writes first), so independent sweeps of
// Alg. Scenario3 share a front: the first diagonal fronts run beside the last cardinal ones (7 fronts
// instead of 9 at q = r = 4).  Solves of one level touch disjoint traces, z parts and slots.  If a
// trace were written after a solve read it, the front order is kept.
void dataflow_fronts(lsw_plan* p) {
    if (p->fronts.size() <= 2) return;
    const Front f0 = p->fronts[0];
    std::vector<SolveDesc> sweeps;   // in the front order
    for (size_t fi = 1; fi < p->fronts.size(); ++fi)
        for (int n = 0; n < p->fronts[fi].count; ++n) sweeps.push_back(p->descs[p->fronts[fi].offset + n]);
    std::map<long long, int> last_writer;   // trace offset -> level of its last writer (stage 1: level 0)
    std::set<long long> read;
    for (int n = 0; n < f0.count; ++n) {
        const SolveDesc& d = p->descs[f0.offset + n];
        for (int o = 0; o < d.nout; ++o) last_writer[d.out_off[o]] = 0;
    }
    std::vector<int> level(sweeps.size(), 1);
    for (size_t k = 0; k < sweeps.size(); ++k) {
        const SolveDesc& d = sweeps[k];
        int lv = 1;
        auto dep = [&](long long off) {
            const auto w = last_writer.find(off);
            if (w != last_writer.end()) lv = std::max(lv, w->second + 1);
        };
        for (long long off : {d.in_h, d.in_v})
            if (off >= 0) {
                dep(off);
                read.insert(off);
            }
        for (int o = 0; o < d.nout; ++o) {
            if (read.count(d.out_off[o])) return;
            dep(d.out_off[o]);
        }
        for (int o = 0; o < d.nout; ++o) last_writer[d.out_off[o]] = lv;
        level[k] = lv;
    }
    const int depth = *std::max_element(level.begin(), level.end());
    std::vector<SolveDesc> descs(p->descs.begin() + f0.offset, p->descs.begin() + f0.offset + f0.count);
    std::vector<Front> fronts{Front{0, 0, f0.count, 0, 0}};
    p->max_front = f0.count;
    for (int lv = 1; lv <= depth; ++lv) {
        const int start = (int)descs.size();
        for (size_t k = 0; k < sweeps.size(); ++k)
            if (level[k] == lv) descs.push_back(sweeps[k]);
        const int count = (int)descs.size() - start;
        if (count == 0) continue;
        fronts.push_back(Front{0, start, count, 0, 0});
        p->max_front = std::max(p->max_front, count);
    }
    p->descs = descs;
    p->fronts = fronts;
}

// Trace-compressed schedule: stage 1 as block substitutions (traces only), all sweep fronts as
// one dataflow launch of GEMV work items with Q', and a final block substitution per window.
int compress_schedule(lsw_plan* p) {
    std::vector<SolveDesc> descs;
    std::vector<Front> fronts;
    const Front f0 = p->fronts[0];
    for (int n = 0; n < f0.count; ++n) {
        SolveDesc d = p->descs[f0.offset + n];
        d.zpart = -1;
        descs.push_back(d);
    }
    fronts.push_back(Front{0, 0, f0.count, 0, 0});
    p->gsolves.clear();
    p->gitems.clear();
    p->QP_elems = 0;
    p->max_nin = 0;
    for (size_t fi = 1; fi < p->fronts.size(); ++fi) {
        const Front& f = p->fronts[fi];
        for (int n = 0; n < f.count; ++n) {
            const SolveDesc& d = p->descs[f.offset + n];
            const SubDesc& s = p->subs[d.sub];
            GemvSolve gs;
            std::memset(&gs, 0, sizeof(gs));
            gs.sub = d.sub;
            gs.kind = d.kind;
            gs.sweep = d.zpart;
            gs.in_h = d.in_h;
            gs.in_v = d.in_v;
            in_ranges(s, d.kind, gs);
            gs.nout = d.nout;
            for (int o = 0; o < d.nout; ++o) {
                gs.out_off[o] = d.out_off[o];
                gs.out_side[o] = d.out_side[o];
                gs.out_acc[o] = d.out_acc[o];
            }
            // Q'_s block: rows = the slots of every output side, columns = the in entries
            int nin = 0;
            for (int r2 = 0; r2 < gs.nin; ++r2) nin += gs.in_len[r2];
            int ld = 0;
            for (int o = 0; o < d.nout; ++o) {
                gs.row_base[o] = ld;
                ld += (d.out_side[o] == SIDE_B || d.out_side[o] == SIDE_T) ? 2 * s.W : 2 * s.H;
            }
            gs.rows = ld;
            ld = (ld + 15) & ~15;
            gs.ld = ld;
            gs.qp_off = (long long)p->QP_elems;
            const int ninp = nin + (nin & 1);   // column pairs (k_qprime / k_gemv layout)
            p->QP_elems += (size_t)ld * ninp;
            p->max_nin = std::max(p->max_nin, nin);
            p->gsolves.push_back(gs);
            // trace-pool ranges of u~, in the order of the in-slot ranges
            GemvItem base;
            std::memset(&base, 0, sizeof(base));
            base.nin = nin;
            base.ld = ld;
            base.nrng = gs.nin;
            for (int r2 = 0; r2 < gs.nin; ++r2) {
                const int st = gs.in_start[r2];
                long long off;
                if (st < 4 * s.W) off = gs.in_h + (st < 2 * s.W ? st : st - 2 * s.W);
                else off = gs.in_v + (st < 4 * s.W + 2 * s.H ? st - 4 * s.W : st - 4 * s.W - 2 * s.H);
                base.rng_off[r2] = off;
                base.rng_len[r2] = gs.in_len[r2];
            }
            for (int o = 0; o < d.nout; ++o) {
                const int len = (d.out_side[o] == SIDE_B || d.out_side[o] == SIDE_T) ? 2 * s.W : 2 * s.H;
                for (int c = 0; c * 64 < len; ++c) {
                    GemvItem it = base;
                    const long long row = gs.row_base[o] + 64LL * c;
                    it.qoff = gs.qp_off + 2 * row;
                    it.qlen = (long long)ninp * ld - 2 * row;
                    it.nrow = std::min(64, len - 64 * c);
                    it.out_off = d.out_off[o] + 64LL * c;
                    it.out_acc = d.out_acc[o];
                    it.solve = (int)p->gsolves.size() - 1;
                    p->gitems.push_back(it);
                }
            }
        }
    }
    // Dependencies between sweep solves through the trace pool, in the front order of
    // Alg. Scenario3: a solve waits for the last writer of every trace it reads or updates
    // (and of every trace it overwrites).  The final right-hand side re-reads every incoming
    // trace after the sweeps, which is exact only if no trace is written after a solve read it.
    const int ngs = (int)p->gsolves.size();
    std::map<long long, int> last_writer;
    std::set<long long> read_once;
    std::vector<std::vector<int>> deps(ngs);
    std::vector<int> level(ngs, 0);
    for (int g2 = 0; g2 < ngs; ++g2) {
        const GemvSolve& gs = p->gsolves[g2];
        std::vector<int> dl;
        auto dep_on = [&](long long off) {
            auto w = last_writer.find(off);
            if (w != last_writer.end() && std::find(dl.begin(), dl.end(), w->second) == dl.end()) dl.push_back(w->second);
        };
        for (long long off : {gs.in_h, gs.in_v})
            if (off >= 0) {
                dep_on(off);
                read_once.insert(off);
            }
        for (int o = 0; o < gs.nout; ++o) {
            if (read_once.count(gs.out_off[o]))
                return fail(p, LSW_EINVAL, "internal: a sweep trace is written after it was read");
            dep_on(gs.out_off[o]);
        }
        for (int o = 0; o < gs.nout; ++o) last_writer[gs.out_off[o]] = g2;
        for (int d2 : dl) level[g2] = std::max(level[g2], level[d2] + 1);
        deps[g2] = dl;
    }
    // items grouped by dependency level: one launch per level, so independent sweeps overlap
    // (depth about 2q instead of the 3q-3 fronts of the front order)
    std::vector<int> order(ngs);
    for (int g2 = 0; g2 < ngs; ++g2) order[g2] = g2;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return level[x] < level[y]; });
    std::vector<std::vector<GemvItem>> by_solve(ngs);
    for (const GemvItem& it : p->gitems) by_solve[it.solve].push_back(it);
    p->gitems.clear();
    p->sweep_depth = ngs ? *std::max_element(level.begin(), level.end()) + 1 : 0;
    size_t at = 0;
    for (int lv = 0; lv < p->sweep_depth; ++lv) {
        const int start = (int)p->gitems.size();
        int nsol = 0;
        for (; at < order.size() && level[order[at]] == lv; ++at, ++nsol)
            for (const GemvItem& it : by_solve[order[at]]) p->gitems.push_back(it);
        fronts.push_back(Front{1, 0, nsol, start, (int)p->gitems.size() - start});
    }
    Front fin{0, (int)descs.size(), (int)p->subs.size(), 0, 0};
    for (size_t n = 0; n < p->subs.size(); ++n) descs.push_back(blank(p->subs[n], (int)n, KIND_FINAL, -1));
    fronts.push_back(fin);
    p->descs = descs;
    p->fronts = fronts;
    p->max_front = std::max(p->max_front, (int)p->subs.size());
    return LSW_OK;
}


// ---------------------------------------------------------------- the preconditioner
ChainArgs chain_args(lsw_plan* p, const c128* d_r, c128* d_z) {
    ChainArgs a{};
    a.subs = p->d_subs;
    a.geo = p->geo;
    a.G = p->d_G;
    a.traces = p->d_traces;
    a.trace_stride = p->trace_stride;
    a.Y = p->d_Y;
    a.Y_stride = p->Y_stride;
    a.zpart = p->d_zpart;
    a.zpart_stride = p->zpart_stride;
    a.z = d_z;
    a.r = d_r;
    a.frp = p->d_frp;
    a.fpool = p->d_fpool;
    a.fcoef = p->d_fcoef;
    a.Q = p->d_Q;
    a.fw = p->d_fw;
    a.fw_stride = p->FWT;
    return a;
}

int apply3d_impl(lsw_plan* p, const c128* d_r, c128* d_z, int nrhs, bool timed);
int setup_impl(lsw_plan* p, const double* d_m, double omega, double h, const lsw_grid_t* grid,
               const lsw_cdd_t* cdd, const lsw_pml_t* pml, const lsw_opts_t* opts);
int setup_windows(lsw_plan* p, const double* d_m, double omega, double h, const lsw_grid_t* grid,
                  const lsw_cdd_t* cdd, const lsw_pml_t* pml, const lsw_opts_t* opts);

// the stage-1 (cs 0) or final (cs 1) block substitutions of a 2D front: R right-hand sides per
// workgroup on the full blocks, or one per workgroup on the packed symmetric blocks when present
hipError_t launch_block_front(lsw_plan* p, ChainArgs a, const Front& f, int nrhs, int cs, int R) {
    const bool c64 = p->precision == LSW_MIXED;
    if (R >= 16 && nrhs > 1) return launch_chain_mma(a, f.count, nrhs, c64, cs, R, p->Wmax, p->stream);
    if (R > 1 && nrhs > 1) return launch_chain_mr(a, f.count, nrhs, p->ept, c64, cs, R, p->stream);
    if (p->gsym) {
        a.G = p->d_Gs;
        return launch_chain_sym(a, f.count, nrhs, p->sym_cfg, cs, p->sym_lds, p->stream);
    }
    return launch_chain(a, f.count, nrhs, p->ept, c64, cs, p->ylds, p->stream);
}

// z = M^-1 r on this plan's own CDD (Alg. Scenario3)
int apply_cdd(lsw_plan* p, const c128* d_r, c128* d_z, int nrhs, bool timed) {
    if (p->dim == 3) return apply3d_impl(p, d_r, d_z, nrhs, timed);
    const bool c64 = p->precision == LSW_MIXED;
    ChainArgs a = chain_args(p, d_r, d_z);
    GemvArgs ga{};
    ga.nrhs = nrhs;
    ga.Q = p->d_Q;
    ga.traces = p->d_traces;
    ga.trace_stride = p->trace_stride;
    const bool chain_mode = p->sweep_mode == LSW_SWEEP_CHAIN;
    // events: [0] start, [1] end of the leading block substitutions, [2] end of the
    // trace-compressed fronts (chained mode: end of all sweeps), [3] start of the final
    // block substitutions (chained mode: end of z assembly), [4] end
    if (timed) HIPCK(p, hipEventRecord(p->ev[0], p->stream));
    if (chain_mode) {
        for (const Front& f : p->fronts) {
            a.descs = p->d_descs + f.offset;
            HIPCK(p, launch_chain(a, f.count, nrhs, p->ept, c64, 3, p->ylds, p->stream));
        }
        if (timed) HIPCK(p, hipEventRecord(p->ev[1], p->stream));
        ZsumArgs zs{p->d_zpart, p->zpart_stride, d_z, p->d_xgroup, p->d_ygroup, p->Nx, p->Ny, p->q, p->r};
        HIPCK(p, launch_zsum(zs, nrhs, c64, p->stream));
        if (timed) HIPCK(p, hipEventRecord(p->ev[2], p->stream));
        if (timed) HIPCK(p, hipEventRecord(p->ev[3], p->stream));
    } else {
        // fronts are [stage 1 (block substitution)] [sweeps (GEMV)]... [final z (block substitution)]
        const size_t nf = p->fronts.size();
        for (size_t fi = 0; fi < nf; ++fi) {
            const Front& f = p->fronts[fi];
            if (fi == nf - 1) {
                if (timed) HIPCK(p, hipEventRecord(p->ev[2], p->stream));
                HIPCK(p, launch_final_rhs(a, (int)p->subs.size(), nrhs, c64, p->stream));
            }
            if (f.gemv) {
                ga.items = p->d_gitems + f.ioffset;
                ga.nitems = f.icount;
                HIPCK(p, p->gemv_mma && nrhs > 1 ? launch_gemv_mma(ga, c64, p->stream) : launch_gemv(ga, c64, p->stream));
            } else {
                if (fi == nf - 1 && timed) HIPCK(p, hipEventRecord(p->ev[3], p->stream));
                a.descs = p->d_descs + f.offset;
                HIPCK(p, launch_block_front(p, a, f, nrhs, fi == 0 ? 0 : 1, p->rgroup));
            }
            if (fi == 0 && timed) HIPCK(p, hipEventRecord(p->ev[1], p->stream));
        }
    }
    if (timed) HIPCK(p, hipEventRecord(p->ev[4], p->stream));
    return LSW_OK;
}

// z = M^-1 r: one CDD, or with windows the sum over the four CDDs of their sweeps of phi_k r
// (scenario 4, Sec. 2.1); with windows every CDD times its own kernel families and evw brackets
// the whole application
int apply_impl(lsw_plan* p, const c128* d_r, c128* d_z, int nrhs, bool timed) {
    if (!p->windows) return apply_cdd(p, d_r, d_z, nrhs, timed);
    for (const lsw_plan* c : p->shifted)
        if (!c) return fail(p, LSW_EINVAL, "windowed plan without its shifted CDDs");
    if (timed) HIPCK(p, hipEventRecord(p->evw[0], p->stream));
    HIPCK(p, hipEventRecord(p->ev_fork, p->stream));
    for (int k = 1; k < 4; ++k) {   // the shifted CDDs, each on its own stream
        lsw_plan* c = p->shifted[k - 1];
        HIPCK(p, hipStreamWaitEvent(c->stream, p->ev_fork, 0));
        HIPCK(p, launch_window(d_r, p->d_wr[k], p->d_wx, p->d_wy, k & 1, k >> 1, p->Nx, p->Ny, p->N, nrhs,
                               c->stream));
        const int rc = apply_cdd(c, p->d_wr[k], p->d_wz[k - 1], nrhs, timed);
        if (rc != LSW_OK) return fail(p, rc, c->err);
        HIPCK(p, hipEventRecord(p->ev_join[k - 1], c->stream));
    }
    HIPCK(p, launch_window(d_r, p->d_wr[0], p->d_wx, p->d_wy, 0, 0, p->Nx, p->Ny, p->N, nrhs, p->stream));
    const int rc = apply_cdd(p, p->d_wr[0], d_z, nrhs, timed);
    if (rc != LSW_OK) return rc;
    for (hipEvent_t e : p->ev_join) HIPCK(p, hipStreamWaitEvent(p->stream, e, 0));
    HIPCK(p, launch_accumulate(d_z, p->d_wz[0], p->d_wz[1], p->d_wz[2], p->N * (size_t)nrhs, p->stream));
    if (timed) HIPCK(p, hipEventRecord(p->evw[1], p->stream));
    return LSW_OK;
}

int matvec_impl(lsw_plan* p, const c128* x, c128* y, const c128* b, int nrhs) {
    if (p->dim == 3) {
        HIPCK(p, launch_matvec3(p->geo, x, y, b, nrhs, p->stream));
        return LSW_OK;
    }
    MatvecArgs a{p->geo, x, y, b};
    HIPCK(p, launch_matvec(a, nrhs, p->stream));
    return LSW_OK;
}

// out[rhs*ostride + l] = <V_l, w>  for l < nv
int dots_impl(lsw_plan* p, const c128* V, size_t vl, size_t vr, const c128* w, size_t ws, int nv, int nrhs,
              c128* out, int ostride) {
    DotsArgs a{V, vl, vr, w, ws, p->N, nv, p->nblk, p->d_partial, out, ostride, 0};
    HIPCK(p, launch_dots(a, nrhs, p->stream));
    return LSW_OK;
}

// w -= V c (sign -1) or += (sign +1) for nv columns
int gs_impl(lsw_plan* p, const c128* V, size_t vl, const c128* coef, int cstride, c128* w, int nv, int sign,
            int nrhs) {
    GsArgs a{V, vl, p->N, coef, cstride, w, p->N, p->N, nv, sign, p->d_active, p->gsblk, nullptr, 0, nullptr};
    HIPCK(p, launch_gs_update(a, nrhs, p->stream));
    return LSW_OK;
}

// the per-rhs mask on the device follows h_active (copied only when it changed)
// (the copy reads one of two pinned staging slots: a copy queued behind a step that was queued
// ahead may run after the host has moved on, so its source must not change before the next wait)
int sync_active(lsw_plan* p, int nrhs) {
    if (std::equal(p->h_active, p->h_active + nrhs, p->dev_active.begin())) return LSW_OK;
    std::copy(p->h_active, p->h_active + nrhs, p->dev_active.begin());
    p->act_slot ^= 1;
    int* stage = p->h_act_stage + (size_t)p->act_slot * p->nrhs_max;
    std::copy(p->h_active, p->h_active + nrhs, stage);
    HIPCK(p, hipMemcpyAsync(p->d_active, stage, sizeof(int) * nrhs, hipMemcpyHostToDevice, p->stream));
    return LSW_OK;
}

// waits for the stream by polling an event: the Krylov loop waits once per iteration, and a
// blocking wait adds its wake-up latency to every iteration
int spin_wait(lsw_plan* p) {
    HIPCK(p, hipEventRecord(p->ev_spin, p->stream));
    hipError_t e;
    while ((e = hipEventQuery(p->ev_spin)) == hipErrorNotReady) {
    }
    HIPCK(p, e);
    return LSW_OK;
}

int wait_event(lsw_plan* p, hipEvent_t e) {
    hipError_t r;
    while ((r = hipEventQuery(e)) == hipErrorNotReady) {
    }
    HIPCK(p, r);
    return LSW_OK;
}

// ---------------------------------------------------------------- FGMRES
int solve_impl(lsw_plan* p, const c128* d_b, c128* d_x, int nrhs, lsw_info_t* info) {
    const auto t0 = std::chrono::steady_clock::now();
    const int m = p->restart;
    const size_t N = p->N;
    const int HS = 2 * (m + 1) + 1;           // host buffer stride per rhs: h1 | h2 | norm
    const size_t vl = (size_t)nrhs * N;       // basis stride between Krylov vectors
    int rc;
    // ||b||^2 into entry 1 of every column; the host reads it with the first residual norm
    if ((rc = dots_impl(p, d_b, 0, N, d_b, N, 1, nrhs, p->d_hbuf + 1, HS)) != LSW_OK) return rc;
    bool first_cycle = true;
    std::vector<double> bnorm(nrhs), relres(nrhs, 1.0);
    std::vector<int> its(nrhs, 0), conv(nrhs, 0);
    std::vector<std::vector<double>> hist(nrhs);
    std::vector<cd> H((size_t)nrhs * (m + 1) * m), cs((size_t)nrhs * m), sn((size_t)nrhs * m),
        g((size_t)nrhs * (m + 1));
    std::vector<int> kend(nrhs), live(nrhs);
    int applies = 0;
    c128* V = p->d_V;
    c128* Z = p->d_Z;
    // The one-pass Gram-Schmidt kernels give every right-hand side d.nblk workgroups (the point
    // order of the dot products), against nblk per column and up to 1024 for the updates in the
    // four-sweep form: they pay once the batch holds a few million points (measured: 32 x 2077^2
    // gains 7% of the solve, one 531^2 vector loses 2.5%).
    const bool gs3 = p->gs_fused > 0 || (p->gs_fused < 0 && (double)N * nrhs >= 4.0e6);
    // below that size the Krylov kernels are launch-bound, and their consumers finish the reductions
    // themselves (every consumer workgroup re-reads the partials; above it a finishing launch is cheaper)
    const bool fin_inline = (double)N * nrhs < 4.0e6;
    while (true) {
        // r = b - A x into V_0, beta = ||r||
        if ((rc = matvec_impl(p, d_x, V, d_b, nrhs)) != LSW_OK) return rc;
        if ((rc = dots_impl(p, V, 0, N, V, N, 1, nrhs, p->d_hbuf, HS)) != LSW_OK) return rc;
        HIPCK(p, hipMemcpyAsync(p->h_hbuf, p->d_hbuf, sizeof(c128) * HS * nrhs, hipMemcpyDeviceToHost, p->stream));
        if ((rc = spin_wait(p)) != LSW_OK) return rc;
        if (first_cycle) {
            for (int s = 0; s < nrhs; ++s) bnorm[s] = std::sqrt(std::max(0.0, p->h_hbuf[(size_t)s * HS + 1].re));
            first_cycle = false;
        }
        int nlive = 0;
        for (int s = 0; s < nrhs; ++s) {
            const double beta = std::sqrt(std::max(0.0, p->h_hbuf[(size_t)s * HS].re));
            relres[s] = bnorm[s] > 0 ? beta / bnorm[s] : 0.0;
            conv[s] = relres[s] <= p->tol;
            live[s] = !conv[s] && its[s] < p->maxit;
            kend[s] = 0;
            p->h_active[s] = live[s];
            std::fill(g.begin() + (size_t)s * (m + 1), g.begin() + (size_t)(s + 1) * (m + 1), cd(0));
            g[(size_t)s * (m + 1)] = beta;
            nlive += live[s];
        }
        if (nlive == 0) break;
        if ((rc = sync_active(p, nrhs)) != LSW_OK) return rc;
        HIPCK(p, launch_scale(V, V, p->d_hbuf, HS, p->d_active, N, N, N, nrhs, p->stream));
        // One Arnoldi step on the device: z_k = M^-1 v_k, w = A z_k, two Gram-Schmidt passes (the second
        // also forms ||w||^2), v_{k+1} = w / ||w||, and the column copied to host slot k % 2.  Nothing in
        // it waits for the host, so step k+1 may be queued before the host has read column k.
        auto enqueue_step = [&](int k) -> int {
            c128* Vk = V + (size_t)k * vl;
            c128* Zk = Z + (size_t)k * vl;
            int rc2;
            if ((rc2 = apply_impl(p, Vk, Zk, nrhs, false)) != LSW_OK) return rc2;
            applies++;
            if ((rc2 = matvec_impl(p, Zk, p->d_w, nullptr, nrhs)) != LSW_OK) return rc2;
            const bool fused = gs3 && k + 1 <= kFusedGsMax;
            // Every form leaves the workgroup partials of ||w||^2 (after the second pass) in d_npart. With
            // fin_inline the scaling of v_{k+1} sums them itself and stores the norm into the column;
            // otherwise the update finishes the norm with a launch of its own.
            c128* nrm = p->d_hbuf + 2 * (m + 1);
            c128* nrm_gs = fin_inline ? nullptr : nrm;
            if (fused) {
                // the same two passes in three sweeps over V: the dots of pass 1 reading w once, the
                // update of pass 1 fused with the dots of pass 2, the update of pass 2 with ||w||^2
                c128* h1 = p->d_hbuf;
                c128* h2 = p->d_hbuf + (m + 1);
                DotsArgs d1{V, vl, N, p->d_w, N, p->N, k + 1, p->nblk, p->d_partial, h1, HS, 0};
                HIPCK(p, launch_dots_w(d1, nrhs, p->stream));
                GsArgs g1{V, vl, p->N, h1, HS, p->d_w, p->N, p->N, k + 1, -1, p->d_active, p->gsblk, nullptr, HS,
                          nullptr};
                DotsArgs d2{V, vl, N, p->d_w, N, p->N, k + 1, p->nblk, p->d_partial, h2, HS, 0};
                HIPCK(p, launch_gs_dots(g1, d2, nrhs, p->stream));
                GsArgs g2{V, vl, p->N, h2, HS, p->d_w, p->N, p->N, k + 1, -1, p->d_active, p->gsblk, nrm_gs, HS,
                          p->d_npart};
                HIPCK(p, launch_gs_update(g2, nrhs, p->stream));
            }
            for (int pass = 0; pass < 2 && !fused; ++pass) {
                c128* hcoef = p->d_hbuf + pass * (m + 1);
                c128* npart = pass == 1 ? p->d_npart : nullptr;
                c128* nout = pass == 1 ? nrm_gs : nullptr;
                if (fin_inline && k + 1 <= p->gs_finish_max) {
                    // the update sums the coefficients from the dot products' partials itself (and stores
                    // them in the column): no finishing launch between the two
                    DotsArgs d{V, vl, N, p->d_w, N, p->N, k + 1, p->nblk, p->d_partial, hcoef, HS, 0};
                    HIPCK(p, launch_dots_partial(d, nrhs, p->stream));
                    GsArgs g{V, vl, p->N, nullptr, HS, p->d_w, p->N, p->N, k + 1, -1, p->d_active, p->gsblk,
                             nout, HS, npart, p->d_partial, p->nblk, hcoef, HS, 0};
                    HIPCK(p, launch_gs_update(g, nrhs, p->stream));
                    continue;
                }
                if ((rc2 = dots_impl(p, V, vl, N, p->d_w, N, k + 1, nrhs, hcoef, HS)) != LSW_OK) return rc2;
                GsArgs g{V, vl, p->N, hcoef, HS, p->d_w, p->N, p->N, k + 1, -1, p->d_active, p->gsblk, nout, HS,
                         npart};
                HIPCK(p, launch_gs_update(g, nrhs, p->stream));
            }
            // (v_{k+1} is unused if every right-hand side stops here; V has room for m + 1 vectors)
            if (fin_inline)
                HIPCK(p, launch_scale_partials(p->d_w, V + (size_t)(k + 1) * vl, p->d_npart, p->gsblk, nrm, HS,
                                               p->d_active, N, N, N, nrhs, p->stream));
            else
                HIPCK(p, launch_scale(p->d_w, V + (size_t)(k + 1) * vl, nrm, HS, p->d_active, N, N, N, nrhs,
                                      p->stream));
            HIPCK(p, hipMemcpyAsync(p->h_hbuf + (size_t)(k & 1) * nrhs * HS, p->d_hbuf, sizeof(c128) * HS * nrhs,
                                    hipMemcpyDeviceToHost, p->stream));
            HIPCK(p, hipEventRecord(p->ev_step[k & 1], p->stream));
            return LSW_OK;
        };
        bool queued = false;   // step k was queued ahead, while the host read column k - 1
        for (int k = 0; k < m; ++k) {
            if (!queued && (rc = enqueue_step(k)) != LSW_OK) return rc;
            // queue step k + 1 now unless every live right-hand side is expected to stop at step k
            // (geometric extrapolation of its residual estimates); a step queued in vain costs one
            // application, a step queued late the host's round trip
            bool ahead = false;
            if (k + 1 < m) {
                for (int s = 0; s < nrhs && !ahead; ++s) {
                    if (!live[s] || its[s] + 1 >= p->maxit) continue;
                    const std::vector<double>& hs = hist[s];
                    const size_t nh = hs.size();
                    const double pred = nh == 0 ? 1.0 : nh == 1 ? 0.5 * hs[0] : hs[nh - 1] * (hs[nh - 1] / hs[nh - 2]);
                    ahead = pred > p->tol;
                }
                if (ahead && (rc = enqueue_step(k + 1)) != LSW_OK) return rc;
            }
            if ((rc = wait_event(p, p->ev_step[k & 1])) != LSW_OK) return rc;
            queued = ahead;
            const c128* hslot = p->h_hbuf + (size_t)(k & 1) * nrhs * HS;
            int still = 0;
            for (int s = 0; s < nrhs; ++s) {
                if (!live[s]) continue;
                const c128* hb = hslot + (size_t)s * HS;
                std::vector<cd> h(k + 2);
                for (int l = 0; l <= k; ++l) h[l] = cd(hb[l].re + hb[m + 1 + l].re, hb[l].im + hb[m + 1 + l].im);
                const double nrm = std::sqrt(std::max(0.0, hb[2 * (m + 1)].re));
                h[k + 1] = nrm;
                cd* CS = cs.data() + (size_t)s * m;
                cd* SN = sn.data() + (size_t)s * m;
                cd* gg = g.data() + (size_t)s * (m + 1);
                for (int l = 0; l < k; ++l) {   // previous rotations [[conj c, conj s], [-s, c]]
                    const cd a0 = h[l], b0 = h[l + 1];
                    h[l] = std::conj(CS[l]) * a0 + std::conj(SN[l]) * b0;
                    h[l + 1] = -SN[l] * a0 + CS[l] * b0;
                }
                const double rho = std::sqrt(std::norm(h[k]) + std::norm(h[k + 1]));
                if (rho == 0.0) {
                    CS[k] = 1.0;
                    SN[k] = 0.0;
                } else {
                    CS[k] = h[k] / rho;
                    SN[k] = h[k + 1] / rho;
                }
                h[k] = rho;
                h[k + 1] = 0.0;
                gg[k + 1] = -SN[k] * gg[k];
                gg[k] = std::conj(CS[k]) * gg[k];
                for (int l = 0; l <= k; ++l) H[((size_t)s * (m + 1) + l) * m + k] = h[l];
                its[s]++;
                kend[s] = k + 1;
                const double est = bnorm[s] > 0 ? std::abs(gg[k + 1]) / bnorm[s] : 0.0;
                hist[s].push_back(est);
                if (est <= p->tol || its[s] >= p->maxit || nrm == 0.0) live[s] = 0;
                p->h_active[s] = live[s];
                still += live[s];
            }
            if (still == 0 || k == m - 1) break;   // a step queued ahead only wrote unused slots
            if ((rc = sync_active(p, nrhs)) != LSW_OK) return rc;
        }
        // x += Z y with y = H^-1 g (upper triangular back substitution on the host)
        int kmax = 0;
        for (int s = 0; s < nrhs; ++s) {
            const int kk = kend[s];
            kmax = std::max(kmax, kk);
            std::vector<cd> y(m, cd(0));
            for (int l = kk - 1; l >= 0; --l) {
                cd acc = g[(size_t)s * (m + 1) + l];
                for (int c = l + 1; c < kk; ++c) acc -= H[((size_t)s * (m + 1) + l) * m + c] * y[c];
                y[l] = acc / H[((size_t)s * (m + 1) + l) * m + l];
            }
            for (int l = 0; l < m; ++l) p->h_coef[(size_t)s * m + l] = c128{y[l].real(), y[l].imag()};
            p->h_active[s] = kk > 0;
        }
        if (kmax > 0) {
            HIPCK(p, hipMemcpyAsync(p->d_coef, p->h_coef, sizeof(c128) * m * nrhs, hipMemcpyHostToDevice, p->stream));
            if ((rc = sync_active(p, nrhs)) != LSW_OK) return rc;
            if ((rc = gs_impl(p, Z, vl, p->d_coef, m, d_x, kmax, +1, nrhs)) != LSW_OK) return rc;
        }
        bool any_left = false;
        for (int s = 0; s < nrhs; ++s) any_left |= (!conv[s] && its[s] < p->maxit);
        if (!any_left) {
            // final true residual for the report
            if ((rc = matvec_impl(p, d_x, V, d_b, nrhs)) != LSW_OK) return rc;
            if ((rc = dots_impl(p, V, 0, N, V, N, 1, nrhs, p->d_hbuf, HS)) != LSW_OK) return rc;
            HIPCK(p, hipMemcpyAsync(p->h_hbuf, p->d_hbuf, sizeof(c128) * HS * nrhs, hipMemcpyDeviceToHost,
                                    p->stream));
            if ((rc = spin_wait(p)) != LSW_OK) return rc;
            for (int s = 0; s < nrhs; ++s) {
                const double beta = std::sqrt(std::max(0.0, p->h_hbuf[(size_t)s * HS].re));
                relres[s] = bnorm[s] > 0 ? beta / bnorm[s] : 0.0;
                conv[s] = relres[s] <= p->tol;
            }
            break;
        }
    }
    if ((rc = spin_wait(p)) != LSW_OK) return rc;
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int s = 0; s < nrhs; ++s) all &= conv[s] != 0;
    if (info) {
        info->t_solve_ms = ms;
        info->applies = applies;
        for (int s = 0; s < nrhs; ++s) {
            if (info->h_rhs) info->h_rhs[s] = lsw_rhs_info_t{its[s], conv[s], relres[s]};
            if (info->h_history && info->history_len > 0)
                for (int t = 0; t < info->history_len; ++t)
                    info->h_history[(size_t)s * info->history_len + t] = t < (int)hist[s].size() ? hist[s][t] : 0.0;
        }
    }
    if (!all) return fail(p, LSW_ENOCONV, "GMRES did not reach tol within maxit");
    return LSW_OK;
}

int check_nrhs(lsw_plan* p, int nrhs) {
    if (nrhs < 1 || nrhs > p->nrhs_max)
        return fail(p, LSW_EINVAL, "nrhs must be in [1, nrhs_max=" + std::to_string(p->nrhs_max) + "]");
    return LSW_OK;
}

// ---------------------------------------------------------------- 3D (beam CDD)
// Twisted block factorisation along z of every beam: plane blocks S_k (s = W*H unknowns,
// the xy plane of the window) are inverted in batches, one batch per elimination step of
// both halves of every subdomain, by blocked Gauss-Jordan: a panel kernel eliminates b
// columns with row pivoting and the accumulated transformation reaches the other columns as
// one rank-b update, a batched complex FP64 GEMM on matrix cores (k_f3_update).
// Twisted block factorisation of every local problem by batched blocked Gauss-Jordan (Phase 2 of
// Sec. 3): block k is grid line k of a 2D window (s = W, line = true) or xy plane k of a 3D beam
// (s = W H).  Each elimination step of both halves of every subdomain is one batch of dense
// blocks S_k = D_k - C G C (padded to the largest s with identity), inverted by blocked
// Gauss-Jordan: a panel kernel eliminates b columns with row pivoting and the accumulated
// transformation reaches the other columns as one rank-b update, a batched complex FP64 GEMM on
// matrix cores (k_f3_update); the middle blocks of all subdomains form the last batch.
// G_k = S_k^-1 lands column-major in G128 (FP64).
int batched_gj(lsw_plan* p, c128* G128, bool line) {
    int rc;
    const int nsub = (int)p->subs.size();
    const int n = line ? p->Wmax : p->Smax, b = std::min(32, n);
    auto blocks = [&](const SubDesc& s) { return line ? s.H : p->Nz; };
    int T = 0;
    for (const SubDesc& s : p->subs) T = std::max(T, std::max(s.mid, blocks(s) - 1 - s.mid));
    // batches: step t of half 0 (block t, from below) and half 1 (block H-1-t, from above), then the middles
    std::vector<std::vector<Fact3Item>> batches;
    for (int t = 0; t < T; ++t) {
        std::vector<Fact3Item> bt;
        for (int sidx = 0; sidx < nsub; ++sidx) {
            const int H = blocks(p->subs[sidx]), m = p->subs[sidx].mid;
            if (t < m) bt.push_back(Fact3Item{sidx, t, t > 0 ? t - 1 : -1, -1});
            if (t < H - 1 - m) bt.push_back(Fact3Item{sidx, H - 1 - t, -1, t > 0 ? H - t : -1});
        }
        if (!bt.empty()) batches.push_back(bt);
    }
    {
        std::vector<Fact3Item> bt;
        for (int sidx = 0; sidx < nsub; ++sidx) {
            const int H = blocks(p->subs[sidx]), m = p->subs[sidx].mid;
            bt.push_back(Fact3Item{sidx, m, m >= 1 ? m - 1 : -1, m + 1 <= H - 1 ? m + 1 : -1});
        }
        batches.push_back(bt);
    }
    std::vector<Fact3Item> all;
    std::vector<size_t> boff;
    size_t maxb = 0;
    for (auto& bt : batches) {
        boff.push_back(all.size());
        all.insert(all.end(), bt.begin(), bt.end());
        maxb = std::max(maxb, bt.size());
    }
    Fact3Item* d_items = nullptr;
    c128 *ws = nullptr, *Pbar = nullptr, *Tb = nullptr;
    int *perm = nullptr, *src = nullptr;
    if ((rc = dalloc(p, &d_items, all.size())) != LSW_OK) return rc;
    if ((rc = dalloc(p, &src, maxb * (size_t)n)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &ws, maxb * n * (size_t)n)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &Pbar, maxb * n * (size_t)b)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &Tb, maxb * n * (size_t)b)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &perm, maxb * (size_t)n)) != LSW_OK) return rc;
    HIPCK(p, hipMemcpy(d_items, all.data(), sizeof(Fact3Item) * all.size(), hipMemcpyHostToDevice));
    Fact3Args fa{};
    fa.subs = p->d_subs;
    fa.geo = p->geo;
    fa.ws = ws;
    fa.n = n;
    fa.G = G128;
    fa.perm = perm;
    fa.status = p->d_status;
    fa.line = line ? 1 : 0;
    HIPCK(p, hipStreamSynchronize(p->stream));
    const auto tf = std::chrono::steady_clock::now();
    for (size_t bi = 0; bi < batches.size(); ++bi) {
        const int nb = (int)batches[bi].size();
        fa.items = d_items + boff[bi];
        HIPCK(p, line ? launch_fact2_build(fa, nb, p->stream) : launch_fact3_build(fa, nb, p->stream));
        for (int p0 = 0; p0 < n; p0 += b) {
            const int bb = std::min(b, n - p0);
            HIPCK(p, launch_fact3_panel(fa, nb, p0, bb, p->stream));
            HIPCK(p, launch_fact3_prep(fa, nb, p0, bb, Pbar, Tb, p->stream));
            // the other columns, [0, p0) and [p0 + bb, n), take the panel's transformation
            const int parts[2][2] = {{0, p0}, {p0 + bb, n - p0 - bb}};
            for (const auto& pt : parts)
                HIPCK(p, launch_fact3_update(Pbar, Tb, ws, n, bb, p0, pt[0], pt[1], nb, p->stream));
        }
        HIPCK(p, launch_fact3_finish(fa, nb, src, p->stream));
    }
    HIPCK(p, hipStreamSynchronize(p->stream));
    p->t_factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();
    dfree(p, ws);
    dfree(p, Pbar);
    dfree(p, Tb);
    dfree(p, perm);
    dfree(p, src);
    dfree(p, d_items);
    std::vector<int> status(nsub);
    HIPCK(p, hipMemcpy(status.data(), p->d_status, sizeof(int) * nsub, hipMemcpyDeviceToHost));
    for (int sidx = 0; sidx < nsub; ++sidx)
        if (status[sidx])
            return fail(p, LSW_ESINGULAR, std::string("zero pivot in the block factorisation of ") +
                                              (line ? "subdomain (" : "beam (") + std::to_string(p->subs[sidx].i) +
                                              "," + std::to_string(p->subs[sidx].j) + ")");
    return LSW_OK;
}

int setup3d_factor(lsw_plan* p) {
    int rc;
    const int nsub = (int)p->subs.size(), Nz = p->Nz;
    c128* G128 = nullptr;
    if ((rc = dalloc(p, &G128, p->G_elems)) != LSW_OK) return rc;
    if ((rc = batched_gj(p, G128, false)) != LSW_OK) return rc;
    const size_t eb = p->precision == LSW_MIXED ? sizeof(c64) : sizeof(c128);
    if (p->gsym) {   // the steps read only the packed blocks
        HIPCK(p, hipMemcpy(p->d_subs, p->subs.data(), sizeof(SubDesc) * p->subs.size(), hipMemcpyHostToDevice));
        char* GS = nullptr;
        if ((rc = dalloc(p, &GS, p->GS_elems * eb)) != LSW_OK) return rc;
        HIPCK(p, launch_pack3(p->d_subs, nsub, Nz, G128, GS, p->pack3_max, p->precision == LSW_MIXED, p->stream));
        HIPCK(p, hipStreamSynchronize(p->stream));
        dfree(p, G128);
        p->d_Gs = GS;
        p->d_G = nullptr;
        char* P3 = nullptr;
        if ((rc = dalloc(p, &P3, (size_t)p->nrhs_max * p->max_front * 2 * p->ptiles3 * 128 * eb)) != LSW_OK) return rc;
        p->d_P3 = P3;
        p->sz_P3 = (size_t)p->nrhs_max * p->max_front * 2 * p->ptiles3 * 128 * eb;
    } else if (p->precision == LSW_MIXED) {
        c64* G64 = nullptr;
        if ((rc = dalloc(p, &G64, p->G_elems)) != LSW_OK) return rc;
        HIPCK(p, launch_cast(G128, G64, p->G_elems, p->stream));
        HIPCK(p, hipStreamSynchronize(p->stream));
        dfree(p, G128);
        p->d_G = G64;
    } else {
        p->d_G = G128;
    }
    const size_t slots = (size_t)p->nrhs_max * p->max_front * Nz * p->Smax;
    char *r3 = nullptr, *y3 = nullptr;
    if ((rc = dalloc(p, &r3, slots * eb)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &y3, slots * eb)) != LSW_OK) return rc;
    p->d_rhs3 = r3;
    p->d_Y3 = y3;
    p->sz_rhs3 = p->sz_Y3 = slots * eb;
    return LSW_OK;
}

// One application over a beam CDD: every front (Alg. Scenario3, concurrent sweeps) is a
// twisted block substitution along z of all its solves, one launch per plane step.
int apply3d_impl(lsw_plan* p, const c128* d_r, c128* d_z, int nrhs, bool timed) {
    const bool c64 = p->precision == LSW_MIXED;
    const int Nz = p->Nz, m = Nz / 2, mh = std::max(m, Nz - 1 - m);
    Chain3Args a{};
    a.subs = p->d_subs;
    a.geo = p->geo;
    a.G = p->d_G;
    a.traces = p->d_traces;
    a.trace_stride = p->trace_stride;
    a.rhs = p->d_rhs3;
    a.Y = p->d_Y3;
    a.slot_stride = (size_t)Nz * p->Smax;
    a.zpart = p->d_zpart;
    a.zpart_stride = p->zpart_stride;
    a.r = d_r;
    a.P3 = p->d_P3;
    a.ptiles = p->ptiles3;
    if (p->gsym) a.G = p->d_Gs;
    p->kev_used = 0;
    auto step = [&](int phase, int t) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed && p->kev_used + 2 <= p->kev.size()) {
            e0 = p->kev[p->kev_used++];
            e1 = p->kev[p->kev_used++];
        }
        return p->gsym ? launch_step3_packed(a, p->Smax, nrhs, phase, t, c64, p->stream, e0, e1)
                       : launch_step3(a, p->Smax, nrhs, phase, t, c64, p->stream, e0, e1);
    };
    if (timed) HIPCK(p, hipEventRecord(p->ev[0], p->stream));
    for (size_t fi = 0; fi < p->fronts.size(); ++fi) {
        const Front& f = p->fronts[fi];
        a.descs = p->d_descs + f.offset;
        a.nslots = f.count;
        HIPCK(p, launch_rhs3(a, p->Smax, nrhs, c64, p->stream));
        for (int t = 0; t < mh; ++t) HIPCK(p, step(0, t));
        HIPCK(p, step(1, 0));
        for (int t = 0; t < mh; ++t) HIPCK(p, step(2, t));
        HIPCK(p, launch_epi3(a, p->Smax, nrhs, c64, p->stream));
        if (fi == 0 && timed) HIPCK(p, hipEventRecord(p->ev[1], p->stream));
    }
    if (timed) {
        HIPCK(p, hipEventRecord(p->ev[2], p->stream));
        HIPCK(p, hipEventRecord(p->ev[3], p->stream));
    }
    HIPCK(p, launch_zsum3(p->d_zpart, p->zpart_stride, d_z, (size_t)nrhs * p->N, c64, p->stream));
    if (timed) HIPCK(p, hipEventRecord(p->ev[4], p->stream));
    return LSW_OK;
}

// Autotuning of the batched substitutions: with several right-hand sides, the stage-1 and
// final fronts can carry R = 1, 2 or 4 of them per workgroup (every factor block read once per
// group), or R = 16 or 32 (complex64 only) on matrix cores (k_chain_mma).  Larger R reads less
// but holds more registers and LDS per step; each candidate is timed on the real factors (zero
// inputs, the stage-1 and final fronts, nrhs_max right-hand sides) and the fastest is kept.
// The shape of the packed one-right-hand-side substitutions (lanes, tiles per lane, ring depth,
// lanes per row of the reduction): every shape the widest window fits is timed on the real
// blocks (zero right-hand side, the first stage-1 and the last final front) and the fastest kept.
// LSW_SYM_CONFIG = i fixes kSymCfgs[i] if the windows fit it.
int tune_sym(lsw_plan* p) {
    p->sym_timed = 0;
    p->sym_tune_best_ms = p->sym_tune_worst_ms = 0;
    if (!p->gsym) return LSW_OK;
    const bool c64 = p->precision == LSW_MIXED;
    if (const char* env = std::getenv("LSW_SYM_CONFIG")) {
        const int c = std::atoi(env);
        if (c >= 0 && c < kSymCfgCount && sym_cfg_fits(c, c64, p->Wmax)) {
            p->sym_cfg = c;
            return LSW_OK;
        }
    }
    int ncand = 0;
    for (int c = 0; c < kSymCfgCount; ++c) ncand += sym_cfg_fits(c, c64, p->Wmax) ? 1 : 0;
    if (ncand < 2) return LSW_OK;
    HIPCK(p, hipMemsetAsync(p->d_tmp1, 0, sizeof(c128) * p->N, p->stream));
    HIPCK(p, hipMemsetAsync(p->d_fw, 0, sizeof(c128) * p->FWT, p->stream));
    ChainArgs a = chain_args(p, p->d_tmp1, p->d_tmp2);
    a.G = p->d_Gs;
    const Front& f0 = p->fronts.front();
    const Front& f1 = p->fronts.back();
    double best = 1e30, worst = 0;
    int pick = p->sym_cfg;
    for (int c = 0; c < kSymCfgCount; ++c) {
        if (!sym_cfg_fits(c, c64, p->Wmax)) continue;
        double tmin = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCK(p, hipEventRecord(p->ev[0], p->stream));
            for (const Front* f : {&f0, &f1}) {
                a.descs = p->d_descs + f->offset;
                HIPCK(p, launch_chain_sym(a, f->count, 1, c, f == &f0 ? 0 : 1, p->sym_lds, p->stream));
            }
            HIPCK(p, hipEventRecord(p->ev[1], p->stream));
            HIPCK(p, hipEventSynchronize(p->ev[1]));
            float ms = 0;
            HIPCK(p, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
            if (rep > 0) tmin = std::min(tmin, (double)ms);   // the first run warms up
        }
        ++p->sym_timed;
        worst = std::max(worst, tmin);
        if (tmin < best) {
            best = tmin;
            pick = c;
        }
    }
    p->sym_cfg = pick;
    p->sym_tune_best_ms = best;
    p->sym_tune_worst_ms = worst;
    return LSW_OK;
}

// Whether the sweep levels of several right-hand sides run on matrix cores (k_gemv_mma, Q' read
// once per item for 16 or 32 right-hand sides) or as batched GEMVs (k_gemv, 4 per pass over Q'):
// every level is timed both ways at nrhs_max on the real Q' and the faster kept.  LSW_GEMV_MMA = 0
// or 1 fixes the choice.
int tune_gemv(lsw_plan* p) {
    p->gemv_mma = false;
    p->gemv_ms[0] = p->gemv_ms[1] = 0;
    if (p->dim != 2 || p->sweep_mode != LSW_SWEEP_COMPRESSED || p->nrhs_max < 2) return LSW_OK;
    if (const char* env = std::getenv("LSW_GEMV_MMA")) {
        p->gemv_mma = std::atoi(env) != 0;
        return LSW_OK;
    }
    const bool c64 = p->precision == LSW_MIXED;
    GemvArgs ga{};
    ga.nrhs = p->nrhs_max;
    ga.Q = p->d_Q;
    ga.traces = p->d_traces;
    ga.trace_stride = p->trace_stride;
    for (int mode = 0; mode < 2; ++mode) {
        double tmin = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCK(p, hipEventRecord(p->ev[0], p->stream));
            for (const Front& f : p->fronts) {
                if (!f.gemv) continue;
                ga.items = p->d_gitems + f.ioffset;
                ga.nitems = f.icount;
                HIPCK(p, mode ? launch_gemv_mma(ga, c64, p->stream) : launch_gemv(ga, c64, p->stream));
            }
            HIPCK(p, hipEventRecord(p->ev[1], p->stream));
            HIPCK(p, hipEventSynchronize(p->ev[1]));
            float ms = 0;
            HIPCK(p, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
            if (rep > 0) tmin = std::min(tmin, (double)ms);   // the first run warms up
        }
        p->gemv_ms[mode] = tmin;
    }
    p->gemv_mma = p->gemv_ms[1] < p->gemv_ms[0];
    return LSW_OK;
}

int tune_rgroup(lsw_plan* p) {
    p->rgroup = 1;
    if (p->dim != 2 || p->sweep_mode != LSW_SWEEP_COMPRESSED || p->nrhs_max < 2) return LSW_OK;
    const bool c64 = p->precision == LSW_MIXED;
    // LSW_RHS_PER_WORKGROUP = 1, 2, 4, 16 or 32 (complex64) fixes the choice (no timing)
    if (const char* env = std::getenv("LSW_RHS_PER_WORKGROUP")) {
        const int R = std::atoi(env);
        if (R == 1 || R == 2 || R == 4 || R == 16 || (R == 32 && c64)) {
            p->rgroup = R;
            return LSW_OK;
        }
    }
    const int nrhs = p->nrhs_max;
    HIPCK(p, hipMemsetAsync(p->d_tmp1, 0, sizeof(c128) * (size_t)nrhs * p->N, p->stream));
    HIPCK(p, hipMemsetAsync(p->d_fw, 0, sizeof(c128) * (size_t)nrhs * p->FWT, p->stream));
    ChainArgs a = chain_args(p, p->d_tmp1, p->d_tmp2);
    const Front& f0 = p->fronts.front();
    const Front& f1 = p->fronts.back();
    double best = 1e30;
    const int cands[5] = {1, 2, 4, 16, 32};
    for (int ci = 0; ci < 5; ++ci) {
        const int R = cands[ci];
        // the matrix-core groups pay off once a 16-wide block is at least a quarter full
        if (R <= 4 ? R > nrhs : (R == 16 ? nrhs < 4 : (!c64 || nrhs <= 16))) continue;
        double tmin = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCK(p, hipEventRecord(p->ev[0], p->stream));
            for (const Front* f : {&f0, &f1}) {
                a.descs = p->d_descs + f->offset;
                const int cs = f == &f0 ? 0 : 1;
                HIPCK(p, launch_block_front(p, a, *f, nrhs, cs, R));
            }
            HIPCK(p, hipEventRecord(p->ev[1], p->stream));
            HIPCK(p, hipEventSynchronize(p->ev[1]));
            float ms = 0;
            HIPCK(p, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
            if (rep > 0) tmin = std::min(tmin, (double)ms);   // the first run warms up
        }
        p->rgroup_ms[ci] = tmin;
        if (tmin < best) {
            best = tmin;
            p->rgroup = R;
        }
    }
    return LSW_OK;
}

int setup_impl(lsw_plan* p, const double* d_m, double omega, double h, const lsw_grid_t* grid,
               const lsw_cdd_t* cdd, const lsw_pml_t* pml, const lsw_opts_t* opts) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!grid || !cdd || !d_m) return fail(p, LSW_EINVAL, "grid, cdd and m are required");
    if (grid->dim != 2 && grid->dim != 3) return fail(p, LSW_EINVAL, "dim must be 2 or 3");
    p->dim = grid->dim;
    if (!(omega > 0) || !(h > 0) || !std::isfinite(omega) || !std::isfinite(h))
        return fail(p, LSW_EINVAL, "omega and h must be positive and finite");
    p->nx = grid->n[0];
    p->ny = grid->n[1];
    p->px = grid->n_pml[0];
    p->py = grid->n_pml[1];
    if (p->nx < 1 || p->ny < 1 || p->px < 0 || p->py < 0) return fail(p, LSW_EINVAL, "bad grid sizes");
    if (p->dim == 3) {
        p->nz = grid->n[2];
        p->pz = grid->n_pml[2];
        if (p->nz < 1 || p->pz < 0) return fail(p, LSW_EINVAL, "bad grid sizes");
    }
    p->q = cdd->q;
    p->r = cdd->r;
    if (p->q < 1 || p->r < 1) return fail(p, LSW_EINVAL, "q and r must be >= 1");
    if (cdd->windows != 0 && cdd->windows != 1) return fail(p, LSW_EINVAL, "cdd.windows must be 0 or 1");
    int own_sx = 0, own_sy = 0;   // shift of this plan's own CDD
    if (cdd->windows) {
        if (p->q < 2 || p->r < 2) return fail(p, LSW_EINVAL, "windows need q >= 2 and r >= 2");
        const int gx = p->nx / p->r, gy = p->ny / p->q;   // smallest bulk group of each axis
        p->shift_x = cdd->shift[0] > 0 ? cdd->shift[0] : gx / 2;
        p->shift_y = cdd->shift[1] > 0 ? cdd->shift[1] : gy / 2;
        if (p->shift_x < 3 || p->shift_x > gx - 3 || p->shift_y < 3 || p->shift_y > gy - 3)
            return fail(p, LSW_EINVAL, "the window shift must lie in [3, smallest group - 3] along each axis");
        p->windows = 1;
    } else {
        own_sx = cdd->shift[0];
        own_sy = cdd->shift[1];
        if (own_sx < 0 || own_sy < 0) return fail(p, LSW_EINVAL, "cdd.shift must be >= 0");
    }
    if (const char* env = std::getenv("LSW_FUSED_GS")) p->gs_fused = std::atoi(env) != 0 ? 1 : 0;
    if (const char* env = std::getenv("LSW_GS_FINISH_MAX"))
        p->gs_finish_max = std::clamp(std::atoi(env), 0, kGsFinishMax);
    p->omega = omega;
    p->h = h;
    p->C = (pml && pml->C > 0) ? pml->C : 16.0 * std::log(omega);
    p->pl = (pml && pml->n_pml_local >= 0) ? pml->n_pml_local : p->px;
    p->e = 2 + p->pl;
    if (opts) {
        if ((opts->alloc == nullptr) != (opts->release == nullptr))
            return fail(p, LSW_EINVAL, "opts.alloc and opts.release must be given together");
        p->ualloc = opts->alloc;
        p->ufree = opts->release;
        p->uctx = opts->alloc_ctx;
        p->precision = opts->precision == LSW_MIXED ? LSW_MIXED : LSW_FP64;
        if (opts->restart > 0) p->restart = opts->restart;
        if (opts->maxit > 0) p->maxit = opts->maxit;
        if (opts->tol > 0) p->tol = opts->tol;
        if (opts->nrhs_max > 0) p->nrhs_max = opts->nrhs_max;
        p->stream = static_cast<hipStream_t>(opts->stream);
        p->sweep_mode = opts->sweep_mode == LSW_SWEEP_CHAIN ? LSW_SWEEP_CHAIN : LSW_SWEEP_COMPRESSED;
    }
    if (p->dim == 3) p->sweep_mode = LSW_SWEEP_CHAIN;   // trace planes are too large to compress
    p->Nx = p->nx + 2 * p->px;
    p->Ny = p->ny + 2 * p->py;
    p->Nz = p->dim == 3 ? p->nz + 2 * p->pz : 1;
    p->N = (size_t)p->Nx * p->Ny * p->Nz;
    split(p->nx, p->px, p->r, p->xlo, p->xhi, own_sx);
    split(p->ny, p->py, p->q, p->ylo, p->yhi, own_sy);
    p->r = (int)p->xlo.size();   // a shifted axis has one more group
    p->q = (int)p->ylo.size();
    auto windows = [&](const std::vector<int>& lo, const std::vector<int>& hi, int Nax, std::vector<int>& w0,
                       std::vector<int>& w1) -> bool {
        const int G = (int)lo.size();
        w0.resize(G);
        w1.resize(G);
        for (int g = 0; g < G; ++g) {
            if (hi[g] - lo[g] < 2) return false;
            w0[g] = lo[g] - (g > 0 ? p->e : 0);
            w1[g] = hi[g] + (g < G - 1 ? p->e : 0);
            if (w0[g] < 0 || w1[g] > Nax) return false;
        }
        return true;
    };
    if (!windows(p->xlo, p->xhi, p->Nx, p->xw0, p->xw1) || !windows(p->ylo, p->yhi, p->Ny, p->yw0, p->yw1))
        return fail(p, LSW_EINVAL, "every CDD group needs >= 2 points and its window (2 + n_pml_local extra "
                                   "lines per interior side) must fit in the extended grid");
    // tables
    std::vector<c128> pool;
    AxisLayers gx{(p->nx + 1) * h, p->px * h, false, false, 0, 0, 0};
    AxisLayers gy{(p->ny + 1) * h, p->py * h, false, false, 0, 0, 0};
    p->geo.gtx = append_table(pool, 0, p->Nx, p->px, h, omega, p->C, gx);
    p->geo.gty = append_table(pool, 0, p->Ny, p->py, h, omega, p->C, gy);
    p->geo.Nz = p->Nz;
    if (p->dim == 3) {
        AxisLayers gz{(p->nz + 1) * h, p->pz * h, false, false, 0, 0, 0};
        p->geo.gtz = append_table(pool, 0, p->Nz, p->pz, h, omega, p->C, gz);
    }
    std::vector<int> txj(p->r), tyi(p->q);
    for (int j = 0; j < p->r; ++j) {
        AxisLayers a = gx;
        a.delta_loc = p->pl * h;
        a.left = p->pl > 0 && j > 0;
        a.right = p->pl > 0 && j < p->r - 1;
        if (a.left) a.xs_left = coord2(2 * (p->xlo[j] - 3), p->px, h);
        if (a.right) a.xs_right = coord2(2 * (p->xhi[j] + 2), p->px, h);
        txj[j] = append_table(pool, p->xw0[j], p->xw1[j], p->px, h, omega, p->C, a);
    }
    for (int i = 0; i < p->q; ++i) {
        AxisLayers a = gy;
        a.delta_loc = p->pl * h;
        a.left = p->pl > 0 && i > 0;
        a.right = p->pl > 0 && i < p->q - 1;
        if (a.left) a.xs_left = coord2(2 * (p->ylo[i] - 3), p->py, h);
        if (a.right) a.xs_right = coord2(2 * (p->yhi[i] + 2), p->py, h);
        tyi[i] = append_table(pool, p->yw0[i], p->yw1[i], p->py, h, omega, p->C, a);
    }
    // subdomains
    p->subs.clear();
    p->G_elems = 0;
    p->GS_elems = 0;
    p->sym_cfg = -1;
    p->sym_lds = 0;
    p->hbase.clear();
    p->vbase.clear();
    p->HT = p->VT = 0;
    p->factor_flops = 0;
    for (int i = 0; i < p->q; ++i)
        for (int j = 0; j < p->r; ++j) {
            SubDesc s{};
            s.W = p->xw1[j] - p->xw0[j];
            s.H = p->yw1[i] - p->yw0[i];
            s.mid = p->dim == 3 ? p->Nz / 2 : s.H / 2;   // the twisted factorisation meets at this block
            s.wx0 = p->xw0[j];
            s.wy0 = p->yw0[i];
            s.r0 = p->ylo[i] - p->yw0[i];
            s.r1 = p->yhi[i] - p->yw0[i];
            s.c0 = p->xlo[j] - p->xw0[j];
            s.c1 = p->xhi[j] - p->xw0[j];
            s.i = i;
            s.j = j;
            s.tx = txj[j];
            s.ty = tyi[i];
            s.sides = (i > 0 ? 1 << SIDE_B : 0) | (i < p->q - 1 ? 1 << SIDE_T : 0) |
                      (j > 0 ? 1 << SIDE_L : 0) | (j < p->r - 1 ? 1 << SIDE_R : 0);
            s.L = slot_count(s.W, s.H);
            s.g_off = (long long)p->G_elems;
            s.gs_off = (long long)p->GS_elems;
            p->GS_elems += (size_t)s.H * sym_block(s.W);
            // column sums c, and one zero row that the reduction reads past the last one
            p->sym_lds = std::max(p->sym_lds, (size_t)(tile_nt(s.W) + 1) * sym_cstride(s.W));
            const size_t S3 = (size_t)s.W * s.H;
            p->G_elems += p->dim == 3 ? (size_t)p->Nz * S3 * S3 : (size_t)s.H * s.W * s.W;
            p->Smax = std::max(p->Smax, (int)S3);
            s.q_off = (long long)p->Q_elems;
            p->Q_elems += (size_t)s.L * s.L;
            s.fw_off = (long long)p->FWT;
            p->FWT += (size_t)s.H * s.W;
            p->ept = std::max(p->ept, (s.W + (1024 / s.W) - 1) / (1024 / s.W));
            p->hbase.push_back(p->HT);
            p->vbase.push_back(p->VT);
            p->HT += 2 * (size_t)s.W * p->Nz;   // trace arrays: [line][z][along the side]
            p->VT += 2 * (size_t)s.H * p->Nz;
            p->Wmax = std::max(p->Wmax, s.W);
            p->Hmax = std::max(p->Hmax, s.H);
            p->factor_flops += p->dim == 3 ? 8.0 * p->Nz * (double)S3 * S3 * S3 : 8.0 * s.H * (double)s.W * s.W * s.W;
            p->subs.push_back(s);
        }
    if (p->Wmax > kMaxWindow)
        return fail(p, LSW_EINVAL, "local window wider than " + std::to_string(kMaxWindow) + " points");
    if (p->dim == 3 && p->Smax > 4096)
        return fail(p, LSW_EINVAL, "3D local windows are limited to 4096 points per xy plane");
    build_schedule(p);
    if (p->sweep_mode == LSW_SWEEP_COMPRESSED) {
        const int rc0 = compress_schedule(p);
        if (rc0 != LSW_OK) return rc0;
    }
    else {
        p->Q_elems = 0;
        dataflow_fronts(p);
    }
    // packed symmetric factors where the substitution kernel's registers allow (LSW_SYMMETRIC_FACTORS=0
    // keeps the full blocks)
    {
        const char* env = std::getenv("LSW_SYMMETRIC_FACTORS");
        const bool off = env && std::atoi(env) == 0;
        const bool mixed = p->precision == LSW_MIXED;
        const size_t eb = mixed ? sizeof(c64) : sizeof(c128);
        p->sym_lds *= eb;
        // static LDS of the kernel: v and the y and x coefficient tables
        const size_t stat = eb * (kMaxWindow + 4) + sizeof(c128) * (2 * kMaxWindow + 1) + 256;
        int dev = 0, max_lds = 0;
        HIPCK(p, hipGetDevice(&dev));
        HIPCK(p, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        // the first shape every window fits is the default; the rest are timed once the blocks exist
        p->sym_cfg = -1;
        for (int c = 0; c < kSymCfgCount && p->sym_cfg < 0; ++c)
            if (sym_cfg_fits(c, mixed, p->Wmax)) p->sym_cfg = c;
        p->gsym = !off && p->dim == 2 && p->sweep_mode == LSW_SWEEP_COMPRESSED && p->sym_cfg >= 0 &&
                  p->sym_lds + stat <= (size_t)max_lds;
        if (p->gsym)
            for (int c = 0; c < kSymCfgCount; ++c)
                if (sym_cfg_fits(c, mixed, p->Wmax)) HIPCK(p, prepare_chain_sym(c, p->sym_lds));
        if (p->dim == 3) {   // packed 64 x 64 tiles of every plane block (k_tile3 / k_red3)
            p->gsym = !off;
            p->GS_elems = 0;
            p->ptiles3 = 0;
            for (SubDesc& s : p->subs) {
                const int S3 = s.W * s.H;
                s.gs_off = (long long)p->GS_elems;
                p->GS_elems += (size_t)p->Nz * plane3_tiles(S3) * 4096;
                p->ptiles3 = std::max(p->ptiles3, plane3_tiles(S3));
                p->pack3_max = std::max(p->pack3_max, (size_t)p->Nz * plane3_tiles(S3) * 4096);
            }
        }
    }
    const size_t eb = p->precision == LSW_MIXED ? sizeof(c64) : sizeof(c128);
    p->apply_chain_bytes = p->apply_gemv_bytes = p->apply_stage1_bytes = p->apply_final_bytes = 0;
    p->apply_stage1_full_bytes = p->apply_final_full_bytes = 0;
    p->chain_launches = p->gemv_launches = 0;
    for (const Front& f : p->fronts) {
        if (f.gemv) {
            p->gemv_launches++;
            for (int n = 0; n < f.icount; ++n) {
                const GemvItem& it = p->gitems[f.ioffset + n];
                p->apply_gemv_bytes += (double)it.nin * it.nrow * eb;
            }
        } else if (p->dim == 3) {
            // forward planes of both halves, the middle plane, backward planes: 2 Nz - 1 blocks
            const int mh = std::max(p->Nz / 2, p->Nz - 1 - p->Nz / 2);
            p->chain_launches += 2 * mh + 1;
            for (int n = 0; n < f.count; ++n) {
                const SubDesc& s = p->subs[p->descs[f.offset + n].sub];
                const double S3 = (double)s.W * s.H;
                const double block = p->gsym ? 4096.0 * plane3_tiles(s.W * s.H) : S3 * S3;
                const double bytes = (2.0 * p->Nz - 1.0) * block * eb;
                p->apply_chain_bytes += bytes;
                if (&f == &p->fronts.front()) p->apply_stage1_bytes += bytes;
            }
        } else {
            p->chain_launches += 2;   // forward halves, then middle row and backward halves
            for (int n = 0; n < f.count; ++n) {
                const SolveDesc& d = p->descs[f.offset + n];
                const SubDesc& s = p->subs[d.sub];
                // forward halves, the middle row, backward halves (each G_k read once per pass)
                const int m = s.mid;
                const double blocks = std::max(0, m - d.kf0) + std::max(0, d.kf1 - m) + 1 +
                                      std::max(0, m - d.kb0) + std::max(0, d.kb1 - m);
                // full blocks W^2 entries; packed blocks 16 per 4x4 tile of the upper triangle
                const double per = p->gsym ? (double)sym_block(s.W) : s.W * (double)s.W;
                const double bytes = blocks * per * eb;
                const double full = blocks * s.W * (double)s.W * eb;
                p->apply_chain_bytes += bytes;
                if (&f == &p->fronts.front()) {
                    p->apply_stage1_bytes += bytes;
                    p->apply_stage1_full_bytes += full;
                } else if (&f == &p->fronts.back()) {
                    p->apply_final_bytes += bytes;
                    p->apply_final_full_bytes += full;
                }
            }
        }
    }
    // m: copy, validate
    std::vector<double> hm(p->N);
    int rc;
    if ((rc = dalloc(p, &p->d_m, p->N)) != LSW_OK) return rc;
    HIPCK(p, hipMemcpy(hm.data(), d_m, sizeof(double) * p->N, hipMemcpyDeviceToHost));
    for (double v : hm)
        if (!std::isfinite(v)) return fail(p, LSW_ENAN, "non-finite value in m");
    HIPCK(p, hipMemcpy(p->d_m, hm.data(), sizeof(double) * p->N, hipMemcpyHostToDevice));
    // device buffers
    if ((rc = dalloc(p, &p->d_tab, pool.size())) != LSW_OK) return rc;
    HIPCK(p, hipMemcpy(p->d_tab, pool.data(), sizeof(c128) * pool.size(), hipMemcpyHostToDevice));
    if ((rc = dalloc(p, &p->d_subs, p->subs.size())) != LSW_OK) return rc;
    HIPCK(p, hipMemcpy(p->d_subs, p->subs.data(), sizeof(SubDesc) * p->subs.size(), hipMemcpyHostToDevice));
    if ((rc = dalloc(p, &p->d_descs, p->descs.size())) != LSW_OK) return rc;
    HIPCK(p, hipMemcpy(p->d_descs, p->descs.data(), sizeof(SolveDesc) * p->descs.size(), hipMemcpyHostToDevice));
    if (!p->gsolves.empty()) {
        if ((rc = dalloc(p, &p->d_gsolves, p->gsolves.size())) != LSW_OK) return rc;
        HIPCK(p, hipMemcpy(p->d_gsolves, p->gsolves.data(), sizeof(GemvSolve) * p->gsolves.size(),
                           hipMemcpyHostToDevice));
        if ((rc = dalloc(p, &p->d_gitems, std::max<size_t>(1, p->gitems.size()))) != LSW_OK) return rc;
        HIPCK(p, hipMemcpy(p->d_gitems, p->gitems.data(), sizeof(GemvItem) * p->gitems.size(),
                           hipMemcpyHostToDevice));
    }
    std::vector<int> xg(p->Nx), yg(p->Ny);
    for (int j = 0; j < p->r; ++j)
        for (int x = p->xlo[j]; x < p->xhi[j]; ++x) xg[x] = j;
    for (int i = 0; i < p->q; ++i)
        for (int y = p->ylo[i]; y < p->yhi[i]; ++y) yg[y] = i;
    if ((rc = dalloc(p, &p->d_xgroup, p->Nx)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_ygroup, p->Ny)) != LSW_OK) return rc;
    HIPCK(p, hipMemcpy(p->d_xgroup, xg.data(), sizeof(int) * p->Nx, hipMemcpyHostToDevice));
    HIPCK(p, hipMemcpy(p->d_ygroup, yg.data(), sizeof(int) * p->Ny, hipMemcpyHostToDevice));
    const int nsub = (int)p->subs.size();
    if ((rc = dalloc(p, &p->d_status, nsub)) != LSW_OK) return rc;
    HIPCK(p, hipMemset(p->d_status, 0, sizeof(int) * nsub));
    p->trace_stride = H_COUNT * p->HT + V_COUNT * p->VT;
    char* tr = nullptr;
    if ((rc = dalloc(p, &tr, p->trace_stride * p->nrhs_max * eb)) != LSW_OK) return rc;
    p->d_traces = tr;
    p->sz_traces = p->trace_stride * p->nrhs_max * eb;
    HIPCK(p, hipMemset(tr, 0, p->trace_stride * p->nrhs_max * eb));
    if (p->sweep_mode == LSW_SWEEP_CHAIN) {
        p->zpart_stride = (size_t)p->nrhs_max * p->N;
        char* zp = nullptr;
        if ((rc = dalloc(p, &zp, 9 * p->zpart_stride * eb)) != LSW_OK) return rc;
        p->d_zpart = zp;
        p->sz_zpart = 9 * p->zpart_stride * eb;
        HIPCK(p, hipMemset(zp, 0, 9 * p->zpart_stride * eb));
    } else {
        if ((rc = dalloc(p, &p->d_fw, (size_t)p->nrhs_max * p->FWT)) != LSW_OK) return rc;
        p->sz_fw = (size_t)p->nrhs_max * p->FWT * sizeof(c128);
    }
    // y of both forward halves, then x when it does not stay in LDS
    p->Y_stride = 2 * (size_t)p->Wmax * p->Hmax;
    char* Y = nullptr;
    if ((rc = dalloc(p, &Y, p->Y_stride * p->max_front * p->nrhs_max * eb)) != LSW_OK) return rc;
    p->d_Y = Y;
    p->sz_Y = p->Y_stride * p->max_front * p->nrhs_max * eb;
    // Krylov
    const int m = p->restart, nr = p->nrhs_max;
    const int HS = 2 * (m + 1) + 1;
    if (!p->member) {   // the shifted CDDs of scenario 4 only apply their sweeps
        if ((rc = dalloc(p, &p->d_V, (size_t)(m + 1) * nr * p->N)) != LSW_OK) return rc;
        if ((rc = dalloc(p, &p->d_Z, (size_t)m * nr * p->N)) != LSW_OK) return rc;
    }
    if ((rc = dalloc(p, &p->d_w, (size_t)nr * p->N)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_tmp1, (size_t)nr * p->N)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_tmp2, (size_t)nr * p->N)) != LSW_OK) return rc;
    p->gsblk = (int)std::min<size_t>(1024, (p->N + 255) / 256);
    if ((rc = dalloc(p, &p->d_partial, (size_t)nr * std::max<size_t>((size_t)(m + 1) * p->nblk, p->gsblk))) != LSW_OK)
        return rc;
    if ((rc = dalloc(p, &p->d_npart, (size_t)nr * p->gsblk)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_hbuf, (size_t)nr * HS)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_coef, (size_t)nr * m)) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_active, (size_t)nr)) != LSW_OK) return rc;
    HIPCK(p, hipMemset(p->d_active, 0, sizeof(int) * (size_t)nr));
    p->dev_active.assign(nr, 0);
    HIPCK(p, hipHostMalloc((void**)&p->h_hbuf, sizeof(c128) * 2 * nr * HS, hipHostMallocDefault));   // 2 slots
    HIPCK(p, hipHostMalloc((void**)&p->h_active, sizeof(int) * nr, hipHostMallocDefault));
    HIPCK(p, hipHostMalloc((void**)&p->h_coef, sizeof(c128) * nr * m, hipHostMallocDefault));
    for (hipEvent_t& e : p->ev) HIPCK(p, hipEventCreate(&e));
    HIPCK(p, hipEventCreateWithFlags(&p->ev_spin, hipEventDisableTiming));
    for (hipEvent_t& e : p->ev_step) HIPCK(p, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCK(p, hipHostMalloc((void**)&p->h_act_stage, sizeof(int) * 2 * nr, hipHostMallocDefault));
    p->geo.tab = p->d_tab;
    p->geo.m = p->d_m;
    p->geo.Nx = p->Nx;
    p->geo.Ny = p->Ny;
    p->geo.h = h;
    p->geo.omega = omega;
    if (p->dim == 3) {
        // one event pair per plane step of a timed application (the dominant kernel's launches)
        const int mz = p->Nz / 2, mhz = std::max(mz, p->Nz - 1 - mz);
        p->kev.assign(2 * p->fronts.size() * (size_t)(2 * mhz + 1), nullptr);
        for (hipEvent_t& e : p->kev) HIPCK(p, hipEventCreate(&e));
        if ((rc = setup3d_factor(p)) != LSW_OK) return rc;
        if (p->windows && (rc = setup_windows(p, d_m, omega, h, grid, cdd, pml, opts)) != LSW_OK) return rc;
        p->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return LSW_OK;
    }
    // factorisation, always in FP64 (complex64 factors are rounded copies)
    c128* G128 = nullptr;
    if ((rc = dalloc(p, &G128, p->G_elems)) != LSW_OK) return rc;
    int dev = 0;
    HIPCK(p, hipGetDevice(&dev));
    int max_lds = 0;
    HIPCK(p, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    {
        // k_chain static LDS: v (kMaxWindow), part (1024) and the y table (kMaxWindow + 1)
        const size_t stat64 = sizeof(c64) * (kMaxWindow + 1024), stat128 = sizeof(c128) * (kMaxWindow + 1024);
        const size_t tabb = sizeof(c128) * (kMaxWindow + 1) + 256;
        const size_t ywin = (size_t)p->Wmax * p->Hmax;
        const size_t y64 = sizeof(c64) * ywin, y128 = sizeof(c128) * ywin;
        const size_t want = p->precision == LSW_MIXED ? y64 + stat64 : y128 + stat128;
        p->ylds = want + tabb <= (size_t)max_lds ? (p->precision == LSW_MIXED ? y64 : y128) : 0;
        p->ylds128 = y128 + stat128 + tabb <= (size_t)max_lds ? y128 : 0;
    }
    if ((rc = batched_gj(p, G128, true)) != LSW_OK) return rc;
    // Q = A_ij^-1 restricted to the trace lines: one unit solve per slot of an interior side
    if (p->sweep_mode == LSW_SWEEP_COMPRESSED) {
        // polarization terms of every sweep solve, grouped by window point for the final solve
        {
            const size_t nent = p->gsolves.size() * (size_t)p->max_nin * 4;
            PEntry* d_pe = nullptr;
            if ((rc = dalloc(p, &d_pe, std::max<size_t>(1, nent))) != LSW_OK) return rc;
            HIPCK(p, launch_pmap(p->d_gsolves, (int)p->gsolves.size(), p->max_nin, p->d_subs, p->geo, d_pe, p->stream));
            std::vector<PEntry> pe(nent);
            HIPCK(p, hipStreamSynchronize(p->stream));
            if (nent) HIPCK(p, hipMemcpy(pe.data(), d_pe, sizeof(PEntry) * nent, hipMemcpyDeviceToHost));
            dfree(p, d_pe);
            // row pointers over the points of every window: window n's H*W+1 entries start at fw_off + n
            std::vector<int> cnt(p->FWT + nsub, 0);
            for (const PEntry& t : pe)
                if (t.sub >= 0) cnt[p->subs[t.sub].fw_off + t.sub + t.point + 1]++;
            std::vector<int> rp(p->FWT + nsub, 0);
            for (int n = 0; n < nsub; ++n) {
                const size_t b = p->subs[n].fw_off + n, np = (size_t)p->subs[n].H * p->subs[n].W;
                rp[b] = 0;
                for (size_t i = 1; i <= np; ++i) rp[b + i] = rp[b + i - 1] + cnt[b + i];
            }
            // global term offsets: window n's terms follow those of windows < n
            std::vector<int> wbase(nsub + 1, 0);
            for (int n = 0; n < nsub; ++n)
                wbase[n + 1] = wbase[n] + rp[p->subs[n].fw_off + n + (size_t)p->subs[n].H * p->subs[n].W];
            for (int n = 0; n < nsub; ++n) {
                const size_t b = p->subs[n].fw_off + n, np = (size_t)p->subs[n].H * p->subs[n].W;
                for (size_t i = 0; i <= np; ++i) rp[b + i] += wbase[n];
            }
            const int nterm = wbase[nsub];
            std::vector<long long> fpool(std::max(1, nterm));
            std::vector<c128> fcoef(std::max(1, nterm));
            std::vector<int> fill(p->FWT + nsub, 0);
            for (const PEntry& t : pe) {
                if (t.sub < 0) continue;
                const size_t row = p->subs[t.sub].fw_off + t.sub + t.point;
                const int at = rp[row] + fill[row]++;
                fpool[at] = t.pool;
                fcoef[at] = t.coef;
            }
            if ((rc = dalloc(p, &p->d_frp, rp.size())) != LSW_OK) return rc;
            if ((rc = dalloc(p, &p->d_fpool, fpool.size())) != LSW_OK) return rc;
            if ((rc = dalloc(p, &p->d_fcoef, fcoef.size())) != LSW_OK) return rc;
            HIPCK(p, hipMemcpy(p->d_frp, rp.data(), sizeof(int) * rp.size(), hipMemcpyHostToDevice));
            HIPCK(p, hipMemcpy(p->d_fpool, fpool.data(), sizeof(long long) * fpool.size(), hipMemcpyHostToDevice));
            HIPCK(p, hipMemcpy(p->d_fcoef, fcoef.data(), sizeof(c128) * fcoef.size(), hipMemcpyHostToDevice));
        }
        const auto tq = std::chrono::steady_clock::now();
        c128* Q128 = nullptr;
        if ((rc = dalloc(p, &Q128, p->Q_elems)) != LSW_OK) return rc;
        HIPCK(p, hipMemsetAsync(Q128, 0, sizeof(c128) * p->Q_elems, p->stream));
        std::vector<SolveDesc> units;
        for (int n = 0; n < nsub; ++n) {
            const SubDesc& s = p->subs[n];
            const int W = s.W, H = s.H;
            const int base[4] = {0, 4 * W + 2 * H, 2 * W, 4 * W};   // indexed by Side: B, R, T, L
            const int len[4] = {2 * W, 2 * H, 2 * W, 2 * H};
            for (int side = 0; side < 4; ++side) {
                if (!((s.sides >> side) & 1)) continue;
                for (int u = 0; u < len[side]; ++u) {
                    const int sl = base[side] + u;
                    int k, c;
                    if (sl < 4 * W) {
                        const int line = sl / W;
                        c = sl - line * W;
                        k = line == 0 ? s.r0 - 1 : line == 1 ? s.r0 : line == 2 ? s.r1 - 1 : s.r1;
                    } else {
                        const int v = sl - 4 * W, line = v / H;
                        k = v - line * H;
                        c = line == 0 ? s.c0 - 1 : line == 1 ? s.c0 : line == 2 ? s.c1 - 1 : s.c1;
                    }
                    SolveDesc d = blank(s, n, KIND_UNIT, -1);
                    d.kf0 = d.kf1 = k;
                    d.unit_k = k;
                    d.unit_c = c;
                    d.q_col = s.q_off + (long long)sl * s.L;
                    units.push_back(d);
                }
            }
        }
        // the unit solves on matrix cores: groups of up to 16 consecutive units of one subdomain, each
        // group one workgroup pair carrying its 16 right-hand sides through every block (FP64)
        constexpr int kGroup = 16, kGroupsPerLaunch = 64;
        std::vector<int> groups;   // {first, count, kf0, kf1} per group
        for (size_t u = 0; u < units.size();) {
            size_t e = u + 1;
            while (e < units.size() && e - u < (size_t)kGroup && units[e].sub == units[u].sub) ++e;
            int k0 = units[u].unit_k, k1 = units[u].unit_k;
            for (size_t v = u; v < e; ++v) {
                k0 = std::min(k0, units[v].unit_k);
                k1 = std::max(k1, units[v].unit_k);
            }
            groups.insert(groups.end(), {(int)u, (int)(e - u), k0, k1});
            u = e;
        }
        const size_t ngroups = groups.size() / 4;
        SolveDesc* d_units = nullptr;
        int* d_groups = nullptr;
        c128* Yq = nullptr;
        if (!units.empty()) {
            if ((rc = dalloc(p, &d_units, units.size())) != LSW_OK) return rc;
            HIPCK(p, hipMemcpy(d_units, units.data(), sizeof(SolveDesc) * units.size(), hipMemcpyHostToDevice));
            if ((rc = dalloc(p, &d_groups, groups.size())) != LSW_OK) return rc;
            HIPCK(p, hipMemcpy(d_groups, groups.data(), sizeof(int) * groups.size(), hipMemcpyHostToDevice));
            if ((rc = dalloc(p, &Yq, p->Y_stride * (size_t)kGroup * std::min<size_t>(kGroupsPerLaunch, ngroups))) != LSW_OK)
                return rc;
        }
        ChainArgs ua = chain_args(p, nullptr, nullptr);
        ua.G = G128;
        ua.Q = Q128;
        ua.Y = Yq;
        ua.descs = d_units;
        for (size_t g0 = 0; g0 < ngroups; g0 += kGroupsPerLaunch) {
            ua.ugroups = d_groups + 4 * g0;
            HIPCK(p, launch_chain_mma_unit(ua, (int)std::min<size_t>(kGroupsPerLaunch, ngroups - g0), p->Wmax, p->stream));
        }
        HIPCK(p, hipStreamSynchronize(p->stream));
        dfree(p, d_units);
        dfree(p, d_groups);
        dfree(p, Yq);
        // fold the polarization map of every sweep solve into its trace-to-trace operator
        c128* QP128 = nullptr;
        if ((rc = dalloc(p, &QP128, std::max<size_t>(1, p->QP_elems))) != LSW_OK) return rc;
        HIPCK(p, hipMemsetAsync(QP128, 0, sizeof(c128) * std::max<size_t>(1, p->QP_elems), p->stream));   // odd-column pads
        HIPCK(p, launch_qprime(p->d_gsolves, (int)p->gsolves.size(), p->max_nin, p->d_subs, p->geo, Q128, QP128,
                               p->stream));
        HIPCK(p, hipStreamSynchronize(p->stream));
        dfree(p, Q128);
        if (p->precision == LSW_MIXED) {
            c64* Q64 = nullptr;
            if ((rc = dalloc(p, &Q64, std::max<size_t>(1, p->QP_elems))) != LSW_OK) return rc;
            HIPCK(p, launch_cast(QP128, Q64, p->QP_elems, p->stream));
            HIPCK(p, hipStreamSynchronize(p->stream));
            dfree(p, QP128);
            p->d_Q = Q64;
        } else {
            p->d_Q = QP128;
        }
        p->t_q_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tq).count();
    }
    if (p->gsym) {
        if (p->precision == LSW_MIXED) {
            c64* GS = nullptr;
            if ((rc = dalloc(p, &GS, p->GS_elems)) != LSW_OK) return rc;
            p->d_Gs = GS;
        } else {
            c128* GS = nullptr;
            if ((rc = dalloc(p, &GS, p->GS_elems)) != LSW_OK) return rc;
            p->d_Gs = GS;
        }
        HIPCK(p, launch_pack_sym(p->d_subs, (int)p->subs.size(), G128, p->d_Gs, p->precision == LSW_MIXED, p->stream));
        HIPCK(p, hipStreamSynchronize(p->stream));
    }
    // the full blocks stay for several right-hand sides per workgroup (and wherever no packed copy exists)
    const bool keep_full = !p->gsym || p->nrhs_max > 1;
    if (!keep_full) {
        dfree(p, G128);
        p->d_G = nullptr;
    } else if (p->precision == LSW_MIXED) {
        c64* G64 = nullptr;
        if ((rc = dalloc(p, &G64, p->G_elems)) != LSW_OK) return rc;
        HIPCK(p, launch_cast(G128, G64, p->G_elems, p->stream));
        HIPCK(p, hipStreamSynchronize(p->stream));
        dfree(p, G128);
        p->d_G = G64;
    } else {
        p->d_G = G128;
    }
    if ((rc = tune_sym(p)) != LSW_OK) return rc;
    if ((rc = tune_rgroup(p)) != LSW_OK) return rc;
    if ((rc = tune_gemv(p)) != LSW_OK) return rc;
    if (p->windows && (rc = setup_windows(p, d_m, omega, h, grid, cdd, pml, opts)) != LSW_OK) return rc;
    p->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return LSW_OK;
}

// scenario 4 (Sec. 2.1): the three shifted CDDs, each set up and factorised as a plan of its own,
// and the window tables of both axes
int setup_windows(lsw_plan* p, const double* d_m, double omega, double h, const lsw_grid_t* grid,
                  const lsw_cdd_t* cdd, const lsw_pml_t* pml, const lsw_opts_t* opts) {
    const int kx[3] = {1, 0, 1}, ky[3] = {0, 1, 1};
    for (int k = 0; k < 3; ++k) {
        lsw_plan* c = new (std::nothrow) lsw_plan();
        if (!c) return fail(p, LSW_ENOMEM, "host allocation failed");
        p->shifted[k] = c;
        c->member = true;
        lsw_cdd_t ck{cdd->q, cdd->r, 0, {kx[k] * p->shift_x, ky[k] * p->shift_y}};
        const int rc = setup_impl(c, d_m, omega, h, grid, &ck, pml, opts);
        if (rc != LSW_OK) return fail(p, rc, "shifted CDD " + std::to_string(k + 1) + ": " + c->err);
    }
    std::vector<int> lo, hi;
    split(p->nx, p->px, p->r, lo, hi, p->shift_x);
    const std::vector<double> ax = axis_window(p->Nx, p->xlo, lo);
    split(p->ny, p->py, p->q, lo, hi, p->shift_y);
    const std::vector<double> ay = axis_window(p->Ny, p->ylo, lo);
    int rc;
    if ((rc = dalloc(p, &p->d_wx, ax.size())) != LSW_OK) return rc;
    if ((rc = dalloc(p, &p->d_wy, ay.size())) != LSW_OK) return rc;
    for (c128*& b : p->d_wr)
        if ((rc = dalloc(p, &b, (size_t)p->nrhs_max * p->N)) != LSW_OK) return rc;
    for (c128*& b : p->d_wz)
        if ((rc = dalloc(p, &b, (size_t)p->nrhs_max * p->N)) != LSW_OK) return rc;
    HIPCK(p, hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    for (hipEvent_t& e : p->ev_join) HIPCK(p, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (lsw_plan* c : p->shifted) {   // set up on the caller's stream; applied on their own
        HIPCK(p, hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
        c->stream = c->own_stream;
    }
    HIPCK(p, hipMemcpy(p->d_wx, ax.data(), sizeof(double) * ax.size(), hipMemcpyHostToDevice));
    HIPCK(p, hipMemcpy(p->d_wy, ay.data(), sizeof(double) * ay.size(), hipMemcpyHostToDevice));
    for (hipEvent_t& e : p->evw) HIPCK(p, hipEventCreate(&e));
    return LSW_OK;
}

// the kernel-family times of the last timed application of one CDD (its events are complete)
// ---------------------------------------------------------------- no-allocation application
// lsw_apply_noalloc keeps its per-application scratch in this array: one copy per GPU, held until
// the process ends.  In host code the name is only a stand-in; the device address of the current
// GPU's copy comes from hipGetSymbolAddress (resolve_scratch) and only that address is used.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[LSW_NOALLOC_SCRATCH_BYTES];

namespace {

// the address of the current GPU's scratch array, looked up once per device with that device
// current (lsw_setup, on the device of the new handle)
int resolve_scratch(lsw_plan* p) {
    int dev = 0;
    HIPCK(p, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(p, LSW_EINVAL, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        HIPCK(p, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(p, LSW_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_addr[dev] = ptr;
    }
    p->d_scratch = g_scratch_addr[dev];
    return LSW_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// scratch bytes of one application at nrhs_max (every buffer 256-byte aligned); 0 with windows
size_t noalloc_bytes(const lsw_plan* p) {
    if (p->windows) return 0;
    size_t b = round256(p->sz_traces) + round256(p->sz_zpart) + round256(p->sz_fw);
    if (p->dim == 2) b += round256(p->sz_Y);
    else b += round256(p->sz_rhs3) + round256(p->sz_Y3) + round256(p->sz_P3);
    return b;
}

// the application of lsw_apply with the handle's per-application buffers replaced by carved
// pieces of the scratch array for the duration of the call (the handle is single-threaded by
// contract, so the swap is not observable); the trace pool, the z parts and the final right-hand
// side terms start at zero, as the handle's own buffers after setup
int apply_noalloc_impl(lsw_plan* p, const c128* d_r, c128* d_z, int nrhs) {
    if (p->windows) return fail(p, LSW_EINVAL, "lsw_apply_noalloc does not support windowed (scenario 4) handles");
    if (!p->d_scratch) return fail(p, LSW_EINVAL, "the scratch array of this device was not resolved at setup");
    const size_t need = noalloc_bytes(p);
    if (need > LSW_NOALLOC_SCRATCH_BYTES)
        return fail(p, LSW_EINVAL, "lsw_apply_noalloc needs " + std::to_string(need) + " bytes of scratch for this "
                                   "handle (nrhs_max " + std::to_string(p->nrhs_max) + "), more than the " +
                                   std::to_string((unsigned long long)LSW_NOALLOC_SCRATCH_BYTES) + " bytes it has");
    char* base = static_cast<char*>(p->d_scratch);
    size_t off = 0;
    auto carve = [&](size_t bytes) -> void* {
        if (bytes == 0) return nullptr;
        void* ptr = base + off;
        off += round256(bytes);
        return ptr;
    };
    void* saved[7] = {p->d_traces, p->d_zpart, p->d_fw, p->d_Y, p->d_rhs3, p->d_Y3, p->d_P3};
    void* traces = carve(p->sz_traces);
    void* zpart = carve(p->sz_zpart);
    void* fw = carve(p->sz_fw);
    void* Y = p->dim == 2 ? carve(p->sz_Y) : nullptr;
    void* rhs3 = p->dim == 3 ? carve(p->sz_rhs3) : nullptr;
    void* Y3 = p->dim == 3 ? carve(p->sz_Y3) : nullptr;
    void* P3 = p->dim == 3 ? carve(p->sz_P3) : nullptr;
    HIPCK(p, launch_zero16(base, round256(p->sz_traces) + round256(p->sz_zpart) + round256(p->sz_fw), p->stream));
    p->d_traces = traces;
    p->d_zpart = zpart;
    p->d_fw = static_cast<c128*>(fw);
    if (p->dim == 2) p->d_Y = Y;
    else {
        p->d_rhs3 = rhs3;
        p->d_Y3 = Y3;
        p->d_P3 = P3;
    }
    const int rc = apply_cdd(p, d_r, d_z, nrhs, false);
    p->d_traces = saved[0];
    p->d_zpart = saved[1];
    p->d_fw = static_cast<c128*>(saved[2]);
    p->d_Y = saved[3];
    p->d_rhs3 = saved[4];
    p->d_Y3 = saved[5];
    p->d_P3 = saved[6];
    return rc;
}

int read_apply_times(lsw_plan* p) {
    float t01 = 0, t12 = 0, t23 = 0, t34 = 0, t04 = 0;
    HIPCK(p, hipEventElapsedTime(&t01, p->ev[0], p->ev[1]));
    HIPCK(p, hipEventElapsedTime(&t12, p->ev[1], p->ev[2]));
    HIPCK(p, hipEventElapsedTime(&t23, p->ev[2], p->ev[3]));
    HIPCK(p, hipEventElapsedTime(&t34, p->ev[3], p->ev[4]));
    HIPCK(p, hipEventElapsedTime(&t04, p->ev[0], p->ev[4]));
    p->last_apply_ms = t04;
    if (p->dim == 3) {   // [0,1] stage-1 front, [1,2] the other fronts, [3,4] the sum of the sweep parts
        p->last_stage1_ms = t01;
        p->last_gemv_ms = t12;
        p->last_final_rhs_ms = 0;
        p->last_final_ms = t34;
        p->last_chain_ms = t01 + t12;
        double dom = 0;
        for (size_t i = 0; i + 1 < p->kev_used; i += 2) {
            float t = 0;
            HIPCK(p, hipEventElapsedTime(&t, p->kev[i], p->kev[i + 1]));
            dom += t;
        }
        p->last_dom_ms = dom;
        p->dom_launches = (int)(p->kev_used / 2);
        p->dom_bytes = p->apply_chain_bytes;
    } else if (p->sweep_mode == LSW_SWEEP_CHAIN) {
        p->last_chain_ms = t01;
        p->last_gemv_ms = 0;
        p->last_stage1_ms = p->last_final_ms = p->last_final_rhs_ms = 0;
    } else {
        p->last_stage1_ms = t01;
        p->last_gemv_ms = t12;
        p->last_final_rhs_ms = t23;
        p->last_final_ms = t34;
        p->last_chain_ms = t01 + t34;
        p->last_dom_ms = t34;     // the two launches of the final z substitutions
        p->dom_launches = 2;
        p->dom_bytes = p->apply_final_bytes;
    }
    return LSW_OK;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

int lsw_setup(lsw_handle_t* out, const double* d_m, double omega, double h, const lsw_grid_t* grid,
              const lsw_cdd_t* cdd, const lsw_pml_t* pml, const lsw_opts_t* opts) {
    if (!out) return LSW_EINVAL;
    *out = nullptr;
    lsw_plan* p = new (std::nothrow) lsw_plan();
    if (!p) return LSW_ENOMEM;
    int rc;
    try {
        rc = setup_impl(p, d_m, omega, h, grid, cdd, pml, opts);
        if (rc == LSW_OK) rc = resolve_scratch(p);   // on the device of the new handle
    } catch (const std::bad_alloc&) {
        p->err = "host allocation failed";
        rc = LSW_ENOMEM;
    } catch (...) {
        p->err = "unexpected host exception";
        rc = LSW_EINVAL;
    }
    if (rc != LSW_OK) {
        g_setup_error = p->err;
        free_plan(p);
        return rc;
    }
    *out = p;
    return LSW_OK;
}

int lsw_apply(lsw_handle_t p, const double* d_r, double* d_z, int nrhs) {
    if (!p || !d_r || !d_z) return LSW_EINVAL;
    int rc = check_nrhs(p, nrhs);
    if (rc != LSW_OK) return rc;
    rc = apply_impl(p, reinterpret_cast<const c128*>(d_r), reinterpret_cast<c128*>(d_z), nrhs, true);
    if (rc != LSW_OK) return rc;
    if (p->windows) {   // per-family times summed over the four CDDs, the total from the bracket
        HIPCK(p, hipEventSynchronize(p->evw[1]));
        if ((rc = read_apply_times(p)) != LSW_OK) return rc;
        double s1 = p->last_stage1_ms, gv = p->last_gemv_ms, fr = p->last_final_rhs_ms, fi = p->last_final_ms,
               ch = p->last_chain_ms, dm = p->last_dom_ms, db = p->dom_bytes;
        int dl = p->dom_launches;
        for (lsw_plan* c : p->shifted) {
            if ((rc = read_apply_times(c)) != LSW_OK) return fail(p, rc, c->err);
            s1 += c->last_stage1_ms;
            gv += c->last_gemv_ms;
            fr += c->last_final_rhs_ms;
            fi += c->last_final_ms;
            ch += c->last_chain_ms;
            dm += c->last_dom_ms;
            db += c->dom_bytes;
            dl += c->dom_launches;
        }
        float t = 0;
        HIPCK(p, hipEventElapsedTime(&t, p->evw[0], p->evw[1]));
        p->last_apply_ms = t;
        p->last_stage1_ms = s1;
        p->last_gemv_ms = gv;
        p->last_final_rhs_ms = fr;
        p->last_final_ms = fi;
        p->last_chain_ms = ch;
        p->last_dom_ms = dm;
        p->dom_bytes = db;
        p->dom_launches = dl;
        return LSW_OK;
    }
    HIPCK(p, hipEventSynchronize(p->ev[4]));
    return read_apply_times(p);
}

int lsw_apply_noalloc(lsw_handle_t p, const double* d_r, double* d_z, int nrhs) {
    if (!p || !d_r || !d_z) return LSW_EINVAL;
    const int rc = check_nrhs(p, nrhs);
    if (rc != LSW_OK) return rc;
    return apply_noalloc_impl(p, reinterpret_cast<const c128*>(d_r), reinterpret_cast<c128*>(d_z), nrhs);
}

int lsw_solve(lsw_handle_t p, const double* d_f, double* d_u, int nrhs, lsw_info_t* info) {
    if (!p || !d_f || !d_u) return LSW_EINVAL;
    int rc = check_nrhs(p, nrhs);
    if (rc != LSW_OK) return rc;
    try {
        return solve_impl(p, reinterpret_cast<const c128*>(d_f), reinterpret_cast<c128*>(d_u), nrhs, info);
    } catch (...) {
        p->err = "host exception in solve";
        return LSW_ENOMEM;
    }
}

int lsw_adjoint(lsw_handle_t p, const double* d_g, double* d_v, int nrhs, lsw_info_t* info) {
    if (!p || !d_g || !d_v) return LSW_EINVAL;
    int rc = check_nrhs(p, nrhs);
    if (rc != LSW_OK) return rc;
    const size_t n = (size_t)nrhs * p->N;
    c128* v = reinterpret_cast<c128*>(d_v);
    HIPCK(p, launch_conj(reinterpret_cast<const c128*>(d_g), p->d_tmp1, n, p->stream));
    HIPCK(p, launch_conj(v, p->d_tmp2, n, p->stream));
    try {
        rc = solve_impl(p, p->d_tmp1, p->d_tmp2, nrhs, info);
    } catch (...) {
        p->err = "host exception in adjoint";
        return LSW_ENOMEM;
    }
    HIPCK(p, launch_conj(p->d_tmp2, v, n, p->stream));
    HIPCK(p, hipStreamSynchronize(p->stream));
    return rc;
}

int lsw_matvec(lsw_handle_t p, const double* d_x, double* d_y, int nrhs) {
    if (!p || !d_x || !d_y || d_x == d_y) return LSW_EINVAL;
    int rc = check_nrhs(p, nrhs);
    if (rc != LSW_OK) return rc;
    rc = matvec_impl(p, reinterpret_cast<const c128*>(d_x), reinterpret_cast<c128*>(d_y), nullptr, nrhs);
    if (rc != LSW_OK) return rc;
    HIPCK(p, hipStreamSynchronize(p->stream));
    return LSW_OK;
}

int lsw_mass_gradient(lsw_handle_t p, const double* d_lam, const double* d_u, int nrhs, double* d_grad) {
    if (!p || !d_lam || !d_u || !d_grad || nrhs < 1) return LSW_EINVAL;
    HIPCK(p, launch_mass_gradient(reinterpret_cast<const c128*>(d_lam), reinterpret_cast<const c128*>(d_u), nrhs,
                                  p->geo, d_grad, p->stream));
    HIPCK(p, hipStreamSynchronize(p->stream));
    return LSW_OK;
}

int lsw_query(lsw_handle_t p, lsw_stats_t* st) {
    if (!p || !st) return LSW_EINVAL;
    std::memset(st, 0, sizeof(*st));
    st->q = p->q;
    st->r = p->r;
    st->n_subdomains = (int)p->subs.size();
    st->W_max = p->Wmax;
    st->H_max = p->Hmax;
    st->N = (long long)p->N;
    st->factor_elems = (long long)p->G_elems;
    st->factor_elem_bytes = p->precision == LSW_MIXED ? 8 : 16;
    st->solves_per_apply = (int)p->descs.size();
    st->fronts_per_apply = (int)p->fronts.size();
    st->apply_chain_bytes = p->apply_chain_bytes;
    st->apply_gemv_bytes = p->apply_gemv_bytes;
    st->chain_launches = p->chain_launches;
    st->gemv_launches = p->gemv_launches;
    st->q_elems = (long long)p->QP_elems;
    st->factor_flops = p->factor_flops;
    st->t_setup_ms = p->t_setup_ms;
    st->t_factor_ms = p->t_factor_ms;
    st->t_q_ms = p->t_q_ms;
    st->last_apply_ms = p->last_apply_ms;
    st->last_chain_ms = p->last_chain_ms;
    st->last_gemv_ms = p->last_gemv_ms;
    st->apply_stage1_bytes = p->apply_stage1_bytes;
    st->apply_final_bytes = p->apply_final_bytes;
    st->last_stage1_ms = p->last_stage1_ms;
    st->last_final_ms = p->last_final_ms;
    st->last_final_rhs_ms = p->last_final_rhs_ms;
    st->rhs_per_workgroup = p->rgroup;
    for (int i = 0; i < 5; ++i) st->tune_ms[i] = p->rgroup_ms[i];
    st->symmetric_factors = p->gsym ? 1 : 0;
    if (p->gsym && p->dim == 2 && p->sym_cfg >= 0) {
        const SymCfg& c = kSymCfgs[p->sym_cfg];
        st->sym_threads = c.threads;
        st->sym_tiles_per_lane = c.tiles_per_lane;
        st->sym_ring = c.ring;
        st->sym_lanes_per_row = c.lanes_per_row;
    }
    st->sym_shapes_timed = p->sym_timed;
    st->apply_stage1_full_bytes = p->apply_stage1_full_bytes;
    st->gemv_mma = p->gemv_mma ? 1 : 0;
    st->gemv_tune_ms[0] = p->gemv_ms[0];
    st->gemv_tune_ms[1] = p->gemv_ms[1];
    st->apply_final_full_bytes = p->apply_final_full_bytes;
    st->sym_tune_best_ms = p->sym_tune_best_ms;
    st->sym_tune_worst_ms = p->sym_tune_worst_ms;
    st->packed_factor_elems = p->gsym ? (long long)p->GS_elems : 0;
    st->gemv_items = (int)p->gitems.size();
    st->gemv_max_inputs = p->max_nin;
    st->cdd_count = p->windows ? 4 : 1;
    st->window_shift[0] = p->shift_x;
    st->window_shift[1] = p->shift_y;
    st->last_dom_ms = p->last_dom_ms;
    st->dom_launches = p->dom_launches;
    st->dom_bytes = p->dom_bytes;
    st->noalloc_bytes = (long long)noalloc_bytes(p);
    if (p->windows) {   // totals over the four CDDs (the setup time already covers all four)
        for (const lsw_plan* c : p->shifted) {
            if (!c) continue;
            st->n_subdomains += (int)c->subs.size();
            st->factor_elems += (long long)c->G_elems;
            st->solves_per_apply += (int)c->descs.size();
            st->fronts_per_apply += (int)c->fronts.size();
            st->apply_chain_bytes += c->apply_chain_bytes;
            st->apply_gemv_bytes += c->apply_gemv_bytes;
            st->chain_launches += c->chain_launches;
            st->gemv_launches += c->gemv_launches;
            st->q_elems += (long long)c->QP_elems;
            st->factor_flops += c->factor_flops;
            st->t_factor_ms += c->t_factor_ms;
            st->t_q_ms += c->t_q_ms;
            st->apply_stage1_bytes += c->apply_stage1_bytes;
            st->apply_final_bytes += c->apply_final_bytes;
            st->apply_stage1_full_bytes += c->apply_stage1_full_bytes;
            st->apply_final_full_bytes += c->apply_final_full_bytes;
            st->packed_factor_elems += c->gsym ? (long long)c->GS_elems : 0;
            st->gemv_items += (int)c->gitems.size();
            st->gemv_max_inputs = std::max(st->gemv_max_inputs, c->max_nin);
        }
    }
    return LSW_OK;
}

const char* lsw_last_error(lsw_handle_t p) { return p ? p->err.c_str() : g_setup_error.c_str(); }

int lsw_destroy(lsw_handle_t p) {
    if (!p) return LSW_OK;
    (void)hipStreamSynchronize(p->stream);
    free_plan(p);
    return LSW_OK;
}

}  // extern "C"
