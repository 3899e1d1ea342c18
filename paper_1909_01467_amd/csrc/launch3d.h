// Argument blocks and launch wrappers of the 3D (beam CDD) device kernels (kernels3d.hip).
//
// A 3D local problem is a beam: the window W x H of its CDD cell times all Nz extended z
// points.  Its unknowns are ordered plane by plane (z slowest, then y, then x), so the matrix
// is block tridiagonal along z with dense-inverse blocks of size s = W*H (one xy plane) and
// diagonal couplings between neighbouring planes.
#pragma once

#include "common.h"

namespace lsw {

// One matrix of a batched plane-block factorisation step.
struct Fact3Item {
    int sub;        // subdomain
    int k;          // plane being factorised
    int below;      // plane whose inverse enters the Schur complement from below (-1: none)
    int above;      // ... from above (-1: none)
};

struct Fact3Args {
    const Fact3Item* items;
    const SubDesc* subs;
    Geometry geo;
    c128* ws;           // [batch][n][n] column-major matrices being inverted (n = padded size)
    int n;              // padded matrix size (largest s)
    c128* G;            // factor pool (complex128, column-major s x s blocks)
    int* perm;          // [batch][n] pivot rows
    int* status;        // per subdomain: 1 if a zero pivot was met
    int line;           // 1: 2D line blocks (s = W, block k = grid line k of the window); 0: 3D planes (s = W H)
};

struct Chain3Args {
    const SolveDesc* descs;   // the solves of one front
    const SubDesc* subs;
    Geometry geo;
    const void* G;            // factor pool (complex64 or complex128)
    void* traces;
    size_t trace_stride;
    void* rhs;                // [nrhs][front slot][Nz][s_max] right-hand sides of the front's solves
    void* Y;                  // same layout: y, then x (in place)
    size_t slot_stride;       // Nz * s_max
    int nslots;               // solves in the front
    void* zpart;              // [9][nrhs][N] per-sweep parts of z
    size_t zpart_stride;      // nrhs * N
    const c128* r;            // input vectors [nrhs][N]
    void* P3;                 // packed steps: [nrhs][front slot][half][tile][2][64] partial products
    int ptiles;               // tiles per plane of the largest block (partial stride)
};

// S = D_k - C G_below C - C G_above C into ws (identity padding), for every item (3D plane blocks)
hipError_t launch_fact3_build(const Fact3Args& a, int nbatch, hipStream_t st);
// the same for the 2D line blocks (a.line = 1): D_k tridiagonal along x, C the diagonal y couplings
hipError_t launch_fact2_build(const Fact3Args& a, int nbatch, hipStream_t st);
// Gauss-Jordan on columns [p0, p0 + b) of every matrix (b <= 32, n <= 4096; row pivoting), then its
// row interchanges applied to all other columns
hipError_t launch_fact3_panel(const Fact3Args& a, int nbatch, int p0, int b, hipStream_t st);
// P = the panel's columns (its transformation, n x b), T = rows [p0, p0 + b) of all columns (b x n)
hipError_t launch_fact3_prep(const Fact3Args& a, int nbatch, int p0, int b, c128* Pbar, c128* T, hipStream_t st);
// W[:, c0 + c] += P T[:, c0 + c] for c in [0, m) outside the pivot rows [j0, j0 + b), which are
// overwritten by P T instead, for every matrix (P: [batch] n x b, T: [batch] b x n, W: [batch] n x n,
// all column-major complex128; b <= 32), on FP64 matrix cores
hipError_t launch_fact3_update(const c128* P, const c128* T, c128* W, int n, int b, int j0, int c0, int m,
                               int nbatch, hipStream_t st);
// undo the row interchanges as column interchanges, then copy the s x s inverse into the pool
// (src: [batch][n] ints of workspace for the composed column permutation)
hipError_t launch_fact3_finish(const Fact3Args& a, int nbatch, int* src, hipStream_t st);

// right-hand sides of a front's solves (stage 1: r on Omega; sweeps: polarized sources)
hipError_t launch_rhs3(const Chain3Args& a, int smax, int nrhs, bool f32, hipStream_t st);
// one step of the twisted block substitution of every solve of a front:
// phase 0 forward (step t of each half), 1 middle plane, 2 backward (step t of each half)
// (e0, e1: optional events recorded before and after the step's main kernel)
hipError_t launch_step3(const Chain3Args& a, int smax, int nrhs, int phase, int t, bool f32, hipStream_t st,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// the same step on the packed symmetric plane blocks (a.G = packed pool, SubDesc::gs_off): one
// workgroup per 64 x 64 tile forms tile v_J and tile^T v_I (a.P3), then one workgroup per 64-row
// block adds its row and column partials in a fixed order into y (phase 2: x = y - sum)
hipError_t launch_step3_packed(const Chain3Args& a, int smax, int nrhs, int phase, int t, bool f32, hipStream_t st,
                               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// packs the symmetrised mean (G + G^T)/2 of every plane block of the full FP64 pool into the
// tile layout of plane3_tiles (complex64 when f32); maxper = the largest Nz*plane3_tiles*4096
hipError_t launch_pack3(const SubDesc* subs, int nsub, int Nz, const c128* G, void* Gs, size_t maxper, bool f32,
                        hipStream_t st);
// solution on Omega into the sweep's part of z, outgoing traces into the trace pool
hipError_t launch_epi3(const Chain3Args& a, int smax, int nrhs, bool f32, hipStream_t st);
// z = sum of the 9 per-sweep parts (n = nrhs * N entries, parts `stride` apart)
hipError_t launch_zsum3(const void* zpart, size_t stride, c128* z, size_t n, bool f32, hipStream_t st);
// y = A x (or b - A x) with the 7-point operator
hipError_t launch_matvec3(const Geometry& g, const c128* x, c128* y, const c128* b, int nrhs, hipStream_t st);

}  // namespace lsw
