// Device data layouts and kernel launchers of the KFBI library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace kfbi {

// Per y-mode constants of the tridiagonal solve along x (Alg. 4).  For mode l
// the system is x[i-1] - beta x[i] + x[i+1] = e[i], beta = 2 + h^2 (kappa - lambda_l),
// lambda_l = -(4/h^2) sin^2(pi l / 2N); r is the root of r^2 - beta r + 1 = 0 in (0, 1).
struct ModeConst {
    double r;      // decay root
    double rinv;   // 1 / r
    double logr;   // log r
    double rC;     // r^C (C = N / 64, the chunk one lane owns)
    double smc;    // -r / (1 - r^(2N)): scale of the rank-one boundary fix
    double pad[3];
};

constexpr int kModeWaves = 8;      // wavefronts of a sparse-fast-solve workgroup (= node sub-tables)

// Everything a kernel needs to read one problem's plan on the device.
struct DevPlan {
    int n, N, M, Q, I;
    int log2N;
    int normal_jump;          // 0: the density is [v] ([d_n v] = 0); 1: it is [d_n v] ([v] = 0)
    double lo, h, inv_h2, h2, kappa;
    const PointGeom* q_geo;   // Q
    const int* q_axis;        // Q
    const PointGeom* z_geo;   // M
    const double* zx;         // M sample positions
    const double* zy;         // M
    const int* irr_i;         // I
    const int* irr_j;         // I
    const double* irr_s;      // I
    const int* arm_q;         // 4 I
    const double* arm_d;      // 4 I
    const int* col_ptr;       // N + 1 entries used (i = 0..N)
    const int* sub_off;       // kModeWaves + 1: rows [sub_off[w], sub_off[w+1]) of the interleaved
                              // table are sub-table w (multiples of kSlots)
    int sub_offv[kModeWaves + 1];   // the same offsets by value, so that a kernel given the plan by
                                    // value reads them with its arguments
    const int* split;         // 3 n_split: (place, first extra piece, extra pieces) of each column
                              // whose nodes are cut into several pieces (see il_ij)
    int n_split;
    const int* il_ij;         // T x 64, slot t*64 + L: node (i, j) of lane L of the sub-table owning row t, packed as
                              // (last-of-piece << 31) | (dest << 16) | j  (0: pad).  A column's nodes
                              // form one piece, or several when the column is long; dest of the
                              // first piece is xpos = i + (i - 1) / (N / 64), column i's place in
                              // the padded per-wavefront mode solution; dest of an extra piece is
                              // kExtraFlag | its index in the extra-sums buffer
    const int* il_pos;        // I: slot of irregular node r in the interleaved layout
    int T;                    // slots per lane, a multiple of kSlots
    const int4* cp_pack;      // M: (i0, j0, sxy, 0)
    const int* cp_i0;         // M
    const int* cp_j0;         // M
    const int* cp_sxy;        // M: bit 0 sx>0, bit 1 sy>0
    const double* cp_w;       // 6 M: weights of the six stencil values in the extracted quantity (v+, or
                              // d_n v+ for a plan that extracts the normal derivative)
    const unsigned char* cp_out;   // 6 M
    const unsigned char* inside;   // (n+1)^2
    const double* sinq;       // N/2 + 1: sin(pi k / N)
    const ModeConst* modes;   // N (index l = 1..N-1 used)
    const double* taps;       // 2 K + 3 spline filter taps
    int K;                    // must equal kSplineK
    // the irregular nodes in the order of their first crossing along Gamma, cut
    // into chunks of at most kCorrChunk nodes whose crossings' spline segments
    // span at most a window of kCorrWindow knots (with the filter's reach):
    // chunk c = (first, end, first window knot, window length) of that order.
    // Per node, at place c kCorrChunk + (its place in the order - first): its
    // arms (crossing index, -1 unused; the distance d), its side and its slot in
    // the sparse-sum layout; the places past a chunk's end are pads with no arms.
    const int4* cc_arm;       // n_cc kCorrChunk
    const double4* cc_d;      // n_cc kCorrChunk
    const double* cc_s;       // n_cc kCorrChunk
    const int* cc_pos;        // n_cc kCorrChunk
    const int4* cc_chunk;     // n_cc
    int n_cc;
};

constexpr int kSplineK = 30;
constexpr int kCorrChunk = 256;    // irregular nodes per correction chunk (one workgroup)
constexpr int kCorrWindow = 256;   // knots of a chunk's density window
constexpr int kSlots = 4;          // table rows loaded together by the sparse sine sums
constexpr int kMaxModesPerGroup = 8;
constexpr int kMaxExtra = 128;      // extra pieces of long columns (per mode, in LDS)
constexpr int kExtraFlag = 0x4000;  // dest field of an extra piece
constexpr int kMaxRestart = 64;
constexpr int kMaxSamples = 12288; // boundary samples per problem (the GMRES step keeps one M-vector in LDS)   // GMRES restart length cap (LDS-resident Hessenberg)

// Source of the interface jumps: either computed from densities on the
// spline (phi, fgam may be null) or given directly (jq / jz, 6 per point).
struct JumpSrc {
    const double* phi;
    const double* phi_s2;    // spline second derivatives of phi (required with phi)
    const double* fgam;
    const double* fgam_s2;   // spline second derivatives of fgam (required with fgam)
    const double* jq;
    const double* jz;
};

struct GmresState {
    int mode;        // 0: residual step pending, 1: Arnoldi, 2: done
    int j;           // Arnoldi column inside the cycle
    int it;          // K_D applications made by the Arnoldi process
    int first;       // 1 until r0 is known
    int converged;   // 1 converged, -1 iteration cap, -2 a NaN or Inf met (kGmNonfinite), 0 running
    int cycles;
    double r0;
    double relres;
    double tol;      // stop when the relative residual drops below tol (<= 0: never)
    int max_iter;    // cap on Arnoldi steps
    int kind;        // what the last commit left for the emit launch (GmKind in gmres.h)
    int jn;          // columns of the cycle just finished (kGmCycleEnd)
    int res_applies; // K applications made for residuals (cycle starts and the final check)
    double scale;    // 1/beta (new cycle) or 1/h_{j+1,j} (next vector)
    double reorth;   // second Gram-Schmidt pass when |z| < reorth |w| (0: never, 1: always)
    double* xout;    // where the emit launch of the finishing step copies the iterate (null: nowhere)
};

struct GmresBufs {
    double* V;       // (m+1) M
    double* H;       // (m+1) m, column j at H + j (m+1)
    double* cs;      // m
    double* sn;      // m
    double* g;       // m + 1
    double* ghat;    // M
    double* phi;     // M
    double* xcur;    // M: input of the next K_D apply
    double* s2cur;   // M: spline second derivatives of xcur
    double* w;       // M: output of the last K_D apply
    double* z;       // M: the vector being orthogonalised (or the residual)
    double* part;    // gm_part_size(m, gc, gc64): per-chunk partial dots and norms
    double* y;       // m + 1: solution of the cycle's triangular system
    GmresState* st;  // state machine; also holds tol and max_iter so launches are call independent
    GmresState* pub; // host-visible mirror of the state (pinned host memory; may be null)
    unsigned* cnt;   // chunks of the current update launch that have finished (0 between launches)
    int m;
    int gc;          // chunks of kGmChunk elements covering the M samples
    int gc64;        // chunks of 64 samples (the first Gram-Schmidt pass)
};

constexpr int kIterNonfinite = -2;

// State of a Richardson or BiCGSTAB run (krylov.hip), in device memory.
struct IterState {
    int it;          // Richardson: updates made; BiCGSTAB: iterations begun
    int done;        // 0 running, 1 converged, -1 iteration cap or breakdown, -2 (kIterNonfinite)
                     // a NaN or Inf met (launches skip while nonzero)
    int max_iter;
    int started;     // 1 once r0 is known
    int half;        // BiCGSTAB: 1 if it stopped half way through an iteration (one apply short)
    int pad;
    double tol, r0, relres;
    double rho, alpha, omega;
    double gamma;    // Richardson relaxation
};

// Vectors of a Richardson or BiCGSTAB run (M doubles each).  The apply reads q
// (BiCGSTAB) or x (Richardson) and writes w.
struct IterBufs {
    double *b, *x, *r, *rhat, *p, *v, *s, *q, *w, *s2;
    IterState* st;
    int M;
};

constexpr int kIterRich = 0, kIterBicgInit = 1, kIterBicgHalf = 2, kIterBicgFull = 3, kIterTrueRes = 4;

// One single-workgroup step of the iterations (krylov.hip): which = kIter*.
hipError_t launch_iter_step(int which, const IterBufs& B, hipStream_t s);

// launchers (return hipError_t of the launch)
hipError_t launch_correct(const DevPlan& p, JumpSrc js, double* corr, double* corr_il, double* dense,
                          const int* skip, hipStream_t s);
// R modes per workgroup (a power of two <= kMaxModesPerGroup whose LDS fits);
// ceil((N-1) / R) workgroups, each writing one row of M partial sums
hipError_t launch_modes(const DevPlan& p, const double* corr, double* partial, int R,
                        const int* skip, hipStream_t s);
hipError_t launch_spline(const DevPlan& p, const double* y, double* s2, const int* skip, hipStream_t s);
// with gm non-null (a GMRES step) the output goes to gm->w, the launch is skipped
// once GMRES is done, and it also makes the first Gram-Schmidt pass (gmres.h)
hipError_t launch_reduce_interp(const DevPlan& p, JumpSrc js, const double* partial, int G, double* out,
                                const int* skip, const GmresBufs* gm, hipStream_t s);
hipError_t launch_interp_grid(const DevPlan& p, JumpSrc js, const double* R, double* out, hipStream_t s);
hipError_t launch_fill_rhs(const DevPlan& p, const double* f, bool mask, double* R, hipStream_t s);
// column sine transforms (dst.hip): FP64, and FP32 arithmetic reading an FP64
// grid into FP32 storage or reading FP32 storage into an FP64 grid (written or
// accumulated)
// B: columns per workgroup (4, 8 or 16; 32 or 64 with FP64 pairs; see dst_tile_ok)
hipError_t launch_dst_cols(const DevPlan& p, const double* in, double* out, double alpha, bool acc, int B,
                           hipStream_t s);
hipError_t launch_dst_cols_f32(const DevPlan& p, const double* in, float* out, double alpha, int B, hipStream_t s);
hipError_t launch_dst_cols_f32_to64(const DevPlan& p, const float* in, double* out, double alpha, bool acc, int B,
                                    hipStream_t s);
// In-place FP64 transforms of `slices` N-row arrays (rows ld elements apart,
// ld columns, arrays `slice` elements apart): the column transforms of the
// planes of a 3D grid.  Skipped while *skip is nonzero (skip may be null).
hipError_t launch_dst_lines(int N, int log2N, const double* sinq, double* a, double alpha, int B, int ld, int slices,
                            size_t slice, const int* skip, hipStream_t s);
// LDS of a column-transform workgroup with B columns whose complex pairs take
// cpx_bytes each; whether B is a valid tile for N within lds_max.
size_t dst_lds_bytes(int N, int B, size_t cpx_bytes);
bool dst_tile_ok(int N, int B, size_t cpx_bytes, size_t lds_max);
// The default tile: the widest valid one that splits `lines` columns into at
// least min_groups workgroups, else the narrowest valid one (0 if none).
int dst_default_tile(int N, size_t cpx_bytes, size_t lds_max, long lines, int min_groups);
// tridiagonal solves along x of every sine mode (FP64 arithmetic; FP64 or FP32 storage)
hipError_t launch_rows_solve(const DevPlan& p, double* A, hipStream_t s);
hipError_t launch_rows_solve_f32(const DevPlan& p, float* A, hipStream_t s);
// R <- R - (L_h - kappa) V on the interior nodes (FP64): the refinement
// residual; with A non-null also A <- A + V (V a correction being applied)
hipError_t launch_residual(const DevPlan& p, const double* V, double* R, double* A, hipStream_t s);
hipError_t launch_grid_out(const DevPlan& p, const double* V, bool mask, double* u, hipStream_t s);
hipError_t launch_axpby(int n, double a, const double* x, double b, const double* y, double* z,
                        hipStream_t s);
// x[0..n) <- v (a kernel, so it may sit in a graph where a memset node may not)
hipError_t launch_fill(size_t n, double v, double* x, hipStream_t s);
// *flag = 1 if x[0..n) holds a NaN or Inf, else 0 (one workgroup; n up to a few 10^4)
hipError_t launch_nonfinite(int n, const double* x, int* flag, hipStream_t s);
// The start of a GMRES run (gm_begin in gmres.h), one launch: the state and
// the first K input (its spline second derivatives with taps; with p and
// corr_il also its corrections, in the sparse-sum layout).  rhs may be null
// (ghat already in place); phi_in may be null (a zero guess); xout (may be
// null) receives the iterate from the emit launch of the step that ends the run.
hipError_t launch_gmres_start(const DevPlan* p, const double* taps, int M, GmresBufs b, const double* rhs,
                              const double* phi_in, double tol, int max_iter, double reorth, double* xout,
                              double* corr_il, hipStream_t s);
// taps: the spline filter of the density (null: no spline, the surface problem)
hipError_t launch_gmres_step(const double* taps, int M, GmresBufs b, hipStream_t s);
// default of GmresState::reorth (see gmres.h)
constexpr double kGmReorthDefault = 1e-3;
// the same step with the next apply's corrections made in the emit launch
// (into corr_il, the sparse-sum layout)
hipError_t launch_gmres_step_corr(const DevPlan& p, GmresBufs b, double* corr_il, hipStream_t s);

size_t modes_lds_bytes(int N, int R);

}  // namespace kfbi
