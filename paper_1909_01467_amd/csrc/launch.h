// Argument blocks and launch wrappers of the device kernels (kernels.hip).
#pragma once

#include "common.h"

namespace lsw {

static constexpr int kMaxWindow = 256;   // largest local window edge the kernels accept

struct ChainArgs {
    const SolveDesc* descs;
    const SubDesc* subs;
    Geometry geo;
    const void* G;          // factor pool
    void* traces;           // trace pool of rhs 0
    size_t trace_stride;    // elements between right-hand sides
    void* Y;                // forward-substitution scratch, one slab per (solve, rhs)
    size_t Y_stride;
    void* zpart;            // [9][nrhs_max][N] per-sweep accumulators (chained sweep mode)
    size_t zpart_stride;    // nrhs_max * N
    c128* z;                // final output (KIND_FINAL)
    const c128* r;          // input [nrhs][N]
    const int* frp;         // final right-hand side: per window, row pointers over its H*W points (H*W+1)
    const long long* fpool; // ... trace-pool offsets of the polarization terms
    const c128* fcoef;      // ... and their coefficients
    void* Q;                // Q pool (KIND_UNIT writes columns)
    c128* fw;               // right-hand sides of the final z solves, window layout [nrhs][sum H*W]
    size_t fw_stride;       // sum over windows of H*W
    int nrhs;               // set by launch_chain_mr: right-hand sides of the launch
    const int* ugroups;     // launch_chain_mma_unit: per group of unit solves {first desc, count, kf0, kf1}
};

struct GemvArgs {
    const GemvItem* items;  // the work items of one dependency level
    int nitems;
    int nrhs;
    const void* Q;          // Q' pool
    void* traces;
    size_t trace_stride;
};

struct ZsumArgs {
    const void* zpart;
    size_t zpart_stride;
    c128* z;
    const int* xgroup;
    const int* ygroup;
    int Nx, Ny, q, r;
};

struct MatvecArgs {
    Geometry geo;
    const c128* x;
    c128* y;
    const c128* b;   // if non-null: y = b - A x
};

struct DotsArgs {
    const c128* V;
    size_t vstride_l, vstride_rhs;
    const c128* w;
    size_t wstride;
    size_t N;
    int nv;
    int nblk;          // workgroups per (l, rhs)
    c128* partial;     // [nrhs][nv][nblk]
    c128* out;         // out[rhs * ostride + l]
    int ostride;
    int accumulate;    // 1: out += sum
};

struct GsArgs {
    const c128* V;
    size_t vstride_l, vstride_rhs;
    const c128* coef;
    int cstride;
    c128* w;
    size_t wstride;
    size_t N;
    int nv;
    int sign;          // -1: w -= V c ; +1: w += V c
    const int* active; // optional per-rhs mask
    int nblk;          // workgroups per rhs (grid-stride over the points)
    c128* norm_out;    // with partial: ||w||^2 after the update into norm_out[rhs * nstride] (null: the
                       // partials are left for launch_scale_partials)
    int nstride;
    c128* partial;     // optional [nrhs][nblk] workgroup partials of the norm
    // optional: the coefficients as unfinished dot products, cpart[(rhs * nv + l) * cnblk + b] (the
    // partials of launch_dots_partial; coef unused), stored once finished to cout[rhs * costride + l]
    // (added to it when caccum); nv <= kGsFinishMax, and partial must be another buffer
    const c128* cpart;
    int cnblk;
    c128* cout;
    int costride;
    int caccum;
};
constexpr int kGsFinishMax = 64;

// ept = max over the launched windows of ceil(W / floor(1024 / W)) (elements per thread)
// Two launches (forward halves, then middle + backward halves) of 2 workgroups per solve.
// cs: 0 stage 1, 1 final z solves, 2 unit solves (Q), 3 any kind (chained sweep mode).
// ylds: bytes of LDS for y/x (H_max * W_max elements), or 0 to keep x in a.Y as well
// (then a.Y_stride must hold 2 * H_max * W_max elements).
hipError_t launch_chain(const ChainArgs& a, int nsolves, int nrhs, int ept, bool c64mode, int cs, size_t ylds,
                        hipStream_t st);
// one dependency level of the trace-compressed sweeps: one workgroup per work item
// stage 1 (cs 0) or final (cs 1) substitutions with rgroup (2 or 4) right-hand sides per
// workgroup; y and x in a.Y (Y_stride >= 2 H_max W_max)
hipError_t launch_chain_mr(const ChainArgs& a, int nsolves, int nrhs, int ept, bool c64mode, int cs, int rgroup,
                           hipStream_t st);
// Shapes of the packed substitution kernel k_chain_sym: lanes per workgroup, tiles per lane,
// blocks in flight in the register ring, lanes per row of the reduction, and the precision.  A
// window of width W fits a shape when its tiles fit the lanes (tile_count(W) <= threads x
// tiles_per_lane) and every row has its reduction lanes (lanes_per_row x W <= threads).
struct SymCfg {
    int threads, tiles_per_lane, ring, lanes_per_row;
    bool c64;
};
inline constexpr SymCfg kSymCfgs[] = {
    {256, 1, 3, 4, true},  {256, 1, 3, 2, true},  {512, 1, 3, 4, true}, {512, 1, 2, 4, true},
    {256, 2, 2, 2, true},  {256, 3, 1, 1, true},  {512, 2, 1, 2, true},
    {256, 1, 2, 4, false}, {256, 1, 2, 2, false}, {512, 1, 1, 4, false},
};
inline constexpr int kSymCfgCount = (int)(sizeof(kSymCfgs) / sizeof(kSymCfgs[0]));
inline bool sym_cfg_fits(int cfg, bool c64mode, int W) {
    const SymCfg& c = kSymCfgs[cfg];
    return c.c64 == c64mode && tile_count(W) <= c.threads * c.tiles_per_lane && c.lanes_per_row * W <= c.threads;
}
// stage 1 (cs 0) or final (cs 1) substitutions, one right-hand side per workgroup, on the packed
// symmetric factors (a.G = packed pool, SubDesc::gs_off) with shape kSymCfgs[cfg], which every
// window must fit; lds = dynamic LDS bytes, >= the column sums of the widest window,
// (tile_nt(W) + 1) sym_cstride(W) entries (set once per shape with prepare_chain_sym); y and x in a.Y
// (Y_stride >= 2 H_max W_max)
hipError_t prepare_chain_sym(int cfg, size_t lds);
// The stage-1 (cs 0) or final (cs 1) substitutions with R = 16 or 32 right-hand sides per workgroup
// on matrix cores (full blocks in a.G; R = 32 in complex64 only); two launches like launch_chain_mr;
// wmax = the widest window of the launch (sizes the per-wave accumulators).
hipError_t launch_chain_mma(const ChainArgs& a, int nsolves, int nrhs, bool c64mode, int cs, int R, int wmax,
                            hipStream_t st);
// One dependency level of the trace-compressed sweeps for many right-hand sides on matrix cores
// (k_gemv_mma: 16 or 32 right-hand sides per workgroup, Q' read once per item and group); the
// same outputs as launch_gemv.
hipError_t launch_gemv_mma(const GemvArgs& a, bool c64mode, hipStream_t st);
// The unit solves that build Q (complex128, full blocks in a.G): groups of up to 16 unit right-hand
// sides of one subdomain (a.descs = the unit descriptors, a.ugroups = ngroups groups), group g's
// right-hand side r using the y/x slab g * 16 + r of a.Y; each writes its column of a.Q.
hipError_t launch_chain_mma_unit(const ChainArgs& a, int ngroups, int wmax, hipStream_t st);
hipError_t launch_chain_sym(const ChainArgs& a, int nsolves, int nrhs, int cfg, int cs, size_t lds, hipStream_t st);
// packed symmetric copy (complex64 or complex128) of the FP64 factor pool
hipError_t launch_pack_sym(const SubDesc* subs, int nsub, const c128* G, void* Gp, bool c64mode, hipStream_t st);
hipError_t launch_gemv(const GemvArgs& a, bool c64mode, hipStream_t st);
hipError_t launch_final_rhs(const ChainArgs& a, int nsub, int nrhs, bool c64mode, hipStream_t st);
hipError_t launch_cast(const c128* src, c64* dst, size_t n, hipStream_t st);
hipError_t launch_window(const c128* r, c128* out, const double* wx, const double* wy, int kx, int ky, int Nx,
                         int Ny, size_t N, int nrhs, hipStream_t st);
// z = ((z + a) + b) + c over n entries (the sum of the four CDDs of scenario 4, in a fixed order)
hipError_t launch_accumulate(c128* z, const c128* a, const c128* b, const c128* c, size_t n, hipStream_t st);
// the polarization maps of all sweep solves as PEntry terms, 4 per (solve, entry) slot (sub = -1: none)
hipError_t launch_pmap(const GemvSolve* gs, int ngs, int max_nin, const SubDesc* subs, const Geometry& geo,
                       PEntry* out, hipStream_t st);
// Q'_s = Q_sub P_s for every sweep solve (complex128), P_s the polarization map from u~ to g
hipError_t launch_qprime(const GemvSolve* gs, int ngs, int max_nin, const SubDesc* subs, const Geometry& geo,
                         const c128* Q, c128* Qp, hipStream_t st);
hipError_t launch_zsum(const ZsumArgs& a, int nrhs, bool c64mode, hipStream_t st);
hipError_t launch_matvec(const MatvecArgs& a, int nrhs, hipStream_t st);
// out[rhs * ostride + l] (+)= <V_l, w> for l < nv (workgroup partials, then a fixed-order sum)
hipError_t launch_dots(const DotsArgs& a, int nrhs, hipStream_t st);
// only the workgroup partials of launch_dots (for launch_gs_update with GsArgs::cpart)
hipError_t launch_dots_partial(const DotsArgs& a, int nrhs, hipStream_t st);
// w -= V c (or +=), optionally followed by ||w||^2 (same point order as launch_dots); with
// GsArgs::cpart, c is first summed from the dot products' partials (bitwise what launch_dots gives)
hipError_t launch_gs_update(const GsArgs& a, int nrhs, hipStream_t st);
// the one-pass forms for nv <= kFusedGsMax columns (hipErrorInvalidValue above): launch_dots_w is
// launch_dots reading w once; launch_gs_dots is launch_gs_update without the norm followed by
// launch_dots of the updated w (d.w = g.w), reading V once; both give launch_dots' sums bitwise
constexpr int kFusedGsMax = 24;
hipError_t launch_dots_w(const DotsArgs& a, int nrhs, hipStream_t st);
hipError_t launch_gs_dots(const GsArgs& g, const DotsArgs& d, int nrhs, hipStream_t st);
// dst = src / ||.|| with the squared norm read from nrm2[rhs * nstride] on the device
hipError_t launch_scale(const c128* src, c128* dst, const c128* nrm2, int nstride, const int* active, size_t N,
                        size_t sstride, size_t dstride, int nrhs, hipStream_t st);
// the same with the squared norm summed from the nnblk <= kScaleFinishMax workgroup partials
// npart[rhs * nnblk + b] of launch_gs_update (GsArgs::partial set, norm_out null) and stored to
// nrm2[rhs * nstride]: bitwise what launch_gs_update's own norm gives, one launch fewer (every
// workgroup re-reads the partials, so it pays only where launches, not bytes, set the time)
constexpr int kScaleFinishMax = 1024;
hipError_t launch_scale_partials(const c128* src, c128* dst, const c128* npart, int nnblk, c128* nrm2, int nstride,
                                 const int* active, size_t N, size_t sstride, size_t dstride, int nrhs,
                                 hipStream_t st);
hipError_t launch_conj(const c128* src, c128* dst, size_t n, hipStream_t st);
// zeros bytes / 16 16-byte words at p (16-byte aligned)
hipError_t launch_zero16(void* p, size_t bytes, hipStream_t st);
hipError_t launch_mass_gradient(const c128* lam, const c128* u, int nrhs, const Geometry& g, double* grad,
                                hipStream_t st);

}  // namespace lsw
