// Internal structures shared by the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cstring>
#include <vector>

namespace fcsph {

constexpr int kMaxStages = 16;
constexpr int kSymR = 3;                 // largest tap offset per axis (|s_a| <= 3)
constexpr int kSymW = 2 * kSymR + 1;     // taps per axis in the dense weight cube
constexpr int kMaxLds = 160 * 1024;      // LDS per workgroup on gfx950
constexpr int kMaxThreads = 512;         // workgroup size bound of the line kernels

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T r, i;
};

// Odd prime radices from kStreamRadix up (PPE plans only) are streamed
// through LDS between the line and a second region of its buffer, by
// kStreamThreads waves per 64 butterflies (each thread holds a block of
// output pairs, never the R inputs).  Such a stage needs one wave per block;
// the waves loop over further chunks of 64 butterflies, so that it does not
// widen the line group (a wider group fits fewer lines per CU).
constexpr int kStreamRadix = 11;
constexpr int kStreamThreads = 3;
__host__ __device__ constexpr int stream_threads(int, int) { return kStreamThreads * 64; }

// Largest number of butterflies per thread and stage for radix R; a line
// group needs ceil(N / (R nb_max(R))) threads for a stage of radix R on N
// points.  The stage keeps nb_max(R) butterflies in registers across its
// barrier, so this bounds the kernels' register budget: with at most 8
// complex values per thread the operator kernels of the FP64 step stay near
// 128 VGPRs (3-4 waves per SIMD instead of 2).  The PPE kernels use the wide
// rule (up to 16 values per thread) for lines the narrow rule cannot fit in
// one 512-thread workgroup: transforms of length 2(n - 1) then fit up to a
// 8192-point Bluestein work length.
__host__ __device__ constexpr int nb_max(int R, bool wide = false) {
  return wide ? (R <= 2 ? 6 : R == 3 ? 4 : R == 4 ? 3 : R <= 8 ? 2 : 1) : (R <= 4 ? 2 : 1);
}

// LDS line buffers hold one padding slot after every 16 complex values, so
// that the strided accesses of the Stockham stages spread over the LDS banks,
// and consecutive lines start one bank group apart.
// pad_index / padded_len take the shift (0: no padding).
__host__ __device__ constexpr int pad_index(int p, int pad) { return pad ? p + (p >> pad) : p; }
__host__ __device__ constexpr int padded_len(int m, int pad) { return ((pad_index(m, pad) + 8) & ~7) + 1; }

// LDS line buffers hold one padding slot after every 2^kLdsPadShift elements
// (fewer bank conflicts on the strided butterfly reads).  The shift is a
// compile-time constant so that the index arithmetic folds; plans record it
// in LinePlan::pad for the host-side sizes.
constexpr int kLdsPadShift = 4;

template <typename T>
struct Line {
  cpx<T> *p;
  __device__ __forceinline__ cpx<T> &operator[](int i) const { return p[i + (i >> kLdsPadShift)]; }
};

// One batched 1D DFT of length n along a line, executed by a group of TL
// threads on a line buffer of M complex values in LDS.  Direct Stockham when
// n factors into the supported radices, otherwise Bluestein with an M-point
// smooth FFT.  Table pointers are cpx<T> device arrays inside the workspace.
struct LinePlan {
  int n;           // DFT length
  int M;           // FFT work length (== n when direct)
  int blue;        // 1: Bluestein
  int nstages;
  int radix[kMaxStages];
  int TL;          // threads per line the plan is sized for
  int pad;         // LDS padding shift of the line buffers (0: none)
  int wide;        // 1: sized for the wide butterfly rule (PPE kernels only)
  int spare;       // > 0: streamed stages (radix >= kStreamRadix) alternate between
                   // the line and positions [spare, spare + M) (a multiple of 16);
                   // the line buffer must hold them (PPE kernels only)
  const void *tw;     // [M]  exp(-2 pi i t / M)
  const void *chirp;  // [n]  exp(-pi i (t^2 mod 2n) / n)        (Bluestein)
  const void *filt;   // [M]  DFT_M(wrapped conj chirp) / M       (Bluestein)
};

// FC(Gram) maps of the two walls of one axis (C x d, row-major, FP64).
struct FcWalls {
  int on;              // axis is walled
  int C, d;
  const double *Mlo;   // map of the low wall (index 0)
  const double *Mhi;   // map of the high wall (index n-1)
  // placement on a transform line of length L: positions n .. n+head-1 hold
  // continuation values 0 .. head-1, positions L-tail .. L-1 hold the last
  // `tail` continuation values, every other position beyond n is zero
  // (whole extension: head = C, tail = 0, L = n + C)
  int head, tail;
};

// Continuation index stored at line position j >= n of a length-L line, or -1
// for a zero-padding position.
__host__ __device__ inline int fc_slot(const FcWalls &fc, int n, int L, int j) {
  const int r = j - n;
  if (r < fc.head) return r;
  const int t = L - j;
  return t <= fc.tail ? fc.C - t : -1;
}

// Spectral symbols: per-axis phase tables ph_a[k * (kSymR+1) + s] =
// exp(-2 pi i k s / E_a), s = 0..kSymR, for the sum along the line axis (the
// transverse sums are tabulated per plan, ColsArgs::symR).
struct SymTables {
  int ndim;
  int E[3];
  const double2 *ph[3];      // per axis phase table (FP64)
};

enum SymCode { SYM_GX = 0, SYM_GY = 1, SYM_GZ = 2, SYM_LAP = 3 };

// ---------------------------------------------------------------- x passes
struct RowsFwdArgs {
  LinePlan plan;
  int nlines;          // complex lines (row pairs)
  int nx, E, H;        // physical, extended, half-spectrum length (E/2+1)
  FcWalls fc;          // x-axis FC (on = 0 for a periodic x axis)
  const double *inA, *inB;   // real rows (inB may be null)
  long strideA, strideB;     // elements between consecutive lines
  int nB;              // lines [0, nB) have a B row
  void *outA, *outB;   // cpx<T> half-spectrum rows
  long ostrideA, ostrideB;   // complex elements between consecutive lines
  int B;               // line groups per workgroup
  int ldsM;            // complex slots per line buffer
  // map_per > 0: line l packs logical rows 2l, 2l+1 of inA, or (inB set)
  // logical row l of inA and of inB; logical row r of a field at
  // field + (r / map_per) * map_plane + (r % map_per) * nx (boundary-row blocks)
  int map_per;
  long map_plane;
  // edge_rows = d > 0 (FP32 kernels, 2D, line l = row l of inA and of inB):
  // the lines of rows y < d and y >= ny - d also run an FP64 pass with
  // plan64 (the FP64 plan of the same length) into the FP64 boundary-row
  // spectra edgeA, edgeB (row e = y, or d + y - (ny - d); pitch H), the
  // inputs of FC_y in the column pass, as a separate FP64 edge launch would
  int edge_rows;
  int ny;
  LinePlan plan64;
  void *edgeA, *edgeB;
};

enum RowsEpi {
  EPI_STORE = 0,       // store the two real outputs (scaled), T or double output
  EPI_STEP_A2 = 1,     // 2D: u* from (Gx u, Gy u), (Gx v, Gy v), (L u, L v)
  EPI_STEP_D2 = 2,     // 2D: projection from (Gx phi, Gy phi)
  EPI_STEP_A3 = 3,     // 3D: u* from 12 derivatives in 6 packed lines
  EPI_STEP_D3 = 4,     // 3D: projection from 3 gradients in 2 packed lines
  EPI_ADVECT2 = 5,     // 2D: RK3 sub-step of linear advection from (Gx u, Gy u)
  EPI_STEP_A3S = 6     // 3D: u* from 12 derivatives, one line group taking the
                       // 6 packed lines in turn (rows of at most 4 TL points)
};

struct WallInfo {
  int ndim;
  int n[3];
  int walled[3];
  int dir[3][2];       // 1 if the velocity wall is Dirichlet
};

// Terms of the intermediate velocity of a low-storage RK3 sub-step (eq.
// uStarRK3 with the RK3 coefficient table; the pressure term is dropped as in
// the first-order form):
//   u* = u - dt (g F + z F_prev - a f),   F = (u . grad) u - nu lap u.
// on == 0: the first-order form u* = u - dt (F - f) (g = a = 1, z = 0).
// F[c] holds F_prev of component c on entry (read only when z != 0) and F on
// exit (physical layout, FP64).
struct RkTerms {
  int on;
  double g, z, a;
  double *F[3];
};

// u* of one component; F is formed from the same expression as the
// first-order form, so on == 0 rounds exactly like it.
__device__ __forceinline__ double rk_ustar(const RkTerms &rk, double u, double adv, double nu, double lap,
                                           double f, double dt, size_t idx, int c) {
  if (!rk.on) return u - dt * (adv - nu * lap - f);
  const double F = adv - nu * lap;
  const double Fp = rk.z != 0.0 ? rk.F[c][idx] : 0.0;
  rk.F[c][idx] = F;
  return u - dt * (rk.g * F + rk.z * Fp - rk.a * f);
}

struct RowsInvArgs {
  LinePlan plan;
  int nrows;           // real rows handled (2D: ny, 3D: ny*nz)
  int nx, E, H;
  int B;               // line groups per workgroup
  int ldsM;
  // EPI_STORE: line l packs rows (2l, 2l+1) of one output spectrum array
  const void *spec[12]; // cpx<T> spectrum row arrays (row pitch H)
  long spec_pitch;     // complex elements per row
  // row r of a spectrum array starts at ((r / rpp) * prow + r % rpp) * spec_pitch:
  // rpp physical rows per plane, prow rows stored per plane (3D: y-extended
  // arrays hold E_y rows per z plane; 2D: prow = rpp)
  int rpp, prow;
  void *out[2];        // EPI_STORE outputs (row pitch nx)
  int out_is_double;
  double scale;
  // step epilogues
  const double *u[3], *f[3], *wall[3];
  double *ustar[3];
  double *unew[3];
  double dt, nu, dt_over_rho;
  RkTerms rk;
  WallInfo wi;
  // EPI_STEP_D2 / D3: 1 = the transformed values are the new velocity
  // (EXTENDED projection, no u* read), 0 = u* - (dt/rho) times them
  int assign;
  // EPI_STEP_A2: 1 = the row's u* and v* also go through the FP64 x forward
  // pass of the divergence that follows (FC along x with fwd_fc, the packed
  // real-to-complex DFT with plan64, the FP64 plan of the same length: plan
  // itself in FP64 kernels) into the FP64 half-spectrum rows fwd_out[0],
  // fwd_out[1] (row pitch H), as a separate FP64 rows-forward launch would
  // write them
  int fwd_fused;
  FcWalls fwd_fc;
  void *fwd_out[2];
  LinePlan plan64;
  // EPI_ADVECT2: F = adv_c[0] Gx u + adv_c[1] Gy u, u <- u - dt (g F + z F_prev)
  // (rk.g, rk.z, rk.F[0]: F_prev in, F out), u[0] read and unew[0] written;
  // wall points flagged in wi.dir take wall[0]
  double adv_c[2];
};

// ---------------------------------------------------------------- strided passes
// COLS_PROJ: projection on the extended periodic lattice (EXTENDED PPE
// domain): forward transforms of every velocity component, the pressure
// spectrum phi = (rho/dt) sum_a S_a e_a / sum_a S_a^2, corrected spectra
// e_a - (dt/rho) S_a phi, and inverse transforms of all of them.
enum ColsMode { COLS_FWD = 0, COLS_OP = 1, COLS_INV = 2, COLS_DIV = 3, COLS_PROJ = 4 };

struct ColsArgs {
  LinePlan plan;
  int mode;
  int ninner;          // contiguous index count (half spectrum in x)
  int nouter;          // outer lines (3D: the other transverse axis)
  long es;             // element stride along the line (complex elements)
  long os_in, os_out;  // outer stride of input / output arrays
  long es_out;         // element stride of the output
  int nload;           // values loaded per line (physical or extended length)
  int nstore;          // values stored per line
  FcWalls fc;          // FC along the line axis (COLS_FWD / COLS_OP / COLS_DIV)
  // inputs / outputs (cpx<T>); blockIdx.y selects an input field for COLS_OP
  const void *in[3];
  void *out[3][4];
  int nout;
  int sym[4];          // symbol code per output (COLS_OP)
  // symbol evaluation
  SymTables st;
  int line_axis;       // lattice axis of the line
  int inner_axis;      // lattice axis of the inner index (x)
  int outer_axis;      // lattice axis of the outer index (-1: none)
  int B;               // lines (adjacent inner indices) per workgroup
  int ldsM;
  // FP32 plans: FP64 x spectra of the d first and d last rows of every outer
  // plane, per input field: edge[f][((h * nouter + o) * d + r) * ninner + c]
  // (h = 0 low rows, 1 high rows), the inputs of FC along the line in FP64
  const double2 *edge[3];
  // symbol passes (OP, DIV): the line coefficients of every symbol at every
  // inner and outer wavenumber, symR[((q * ninner + k) * nouter + o) * kSymW
  // + sl + R], tabulated at plan creation (2D: one outer index)
  const double2 *symR;
  // kernels of unbounded support (Gaussian family): the symbols themselves,
  // symF[((q * ninner + c) * nouter + o) * plan.n + k]; when set, symR is not used
  const double2 *symF;
  // COLS_OP, one problem per launch: 0, or the number of workgroups that run
  // whole (f, panel) tasks; each later workgroup runs one output of one of
  // the remaining tasks (gridDim.y == 1, see launch_cols)
  int nfull;
  // COLS_PROJ (one line per workgroup): dt/rho; the modes whose symbol sum
  // |sum_a S_a^2| (table units) is at most proj_tol get a zero pressure; the
  // corrected spectra are scaled by proj_inv_norm and the pressure spectrum by
  // proj_inv_norm^2 (the transforms are unnormalised, the symbol tables carry
  // 1 / prod E)
  double proj_dtr, proj_tol, proj_inv_norm;
};

// ---------------------------------------------------------------- PPE passes
// Per-axis PPE transform.  With N = n - 1 intervals between the walls:
//  DCT1 (Neumann both walls) and DST1 (Dirichlet both walls): complex DFT of
//    the even / odd extension, length 2N;
//  QWS (Dirichlet at index 0, Neumann at n-1; basis sin(pi (2l+1) j / 2N),
//    unknowns j = 1..N) and QWC (Neumann at 0, Dirichlet at n-1; basis
//    cos(pi (2l+1) j / 2N), unknowns j = 0..N-1): the data extended to the
//    length-4N sequence that is odd / even about 0, even / odd about N and
//    anti-periodic with half period 2N has only odd frequencies 2l+1; those are
//    a length-2N DFT of the first 2N samples times exp(-i pi j / 2N)
//    (forward), and the inverse is the length-2N inverse DFT followed by
//    exp(+i pi j / 2N).  Stored coefficients are 4 sum_j w_j x_j basis_l(j)
//    (w = 1/2 at the Neumann end), so the synthesis scale is 1 / 2N as for
//    DCT1 and DST1.
enum TrigKind { TRIG_DFT = 0, TRIG_DCT1 = 1, TRIG_DST1 = 2, TRIG_QWS = 3, TRIG_QWC = 4 };

struct PpeRowsArgs {
  LinePlan plan;       // complex FFT of the extended trig length
  int kind;            // TrigKind of the x axis
  int inverse;         // 0: forward (real rows -> packed coefficients), 1: inverse
  int nrows, nx;
  int ncoef;           // coefficients per row (DCT1: n, DST1: n-2, DFT: n/2+1)
  int cpitch;          // complex elements per coefficient row
  const double *in_real;   // forward input (double), or null when in_float used
  const float *in_float;
  const void *qtw;     // QWS / QWC: cpx<T> exp(-i pi j / 2N), j < 2N
  const double2 *dcs;  // DCT1 at length N (plan.n == N): (cos, sin)(pi j / N), j <= N / 2; null: length 2N
  void *coef;          // cpx<T> coefficient rows
  double *out;         // inverse output (physical rows)
  double scale;
  int B, ldsM;
  // forward from an x half spectrum instead of real rows (spec non-null):
  // rows 2l, 2l+1 of spec (pitch spec_pitch) through the packed C2R of
  // xplan (extended length xE, xH coefficients), times in_scale, rounded to
  // FP32 first when round32 (the values the separate C2R store would write)
  const void *spec;
  long spec_pitch;
  LinePlan xplan;
  int xE, xH;
  double in_scale;
  int round32;
  // inverse, spec_out non-null: besides storing the rows, their x half
  // spectra (FC_x with the maps xfc, packed R2C of xplan) at rows 2l, 2l+1
  // of spec_out (pitch spec_pitch), the first pass of the projection gradient
  void *spec_out;
  FcWalls xfc;
};

struct PpeColsArgs {
  LinePlan plan;
  int kind;            // TrigKind of the line axis
  int ninner, nouter;
  long es, os;         // strides in complex elements
  int nline;           // physical points on the line axis
  int ncoef;           // modes on the line axis
  int solve;           // 1: forward, divide, inverse; 0: forward only; 2: inverse only
  const double *mu_line;   // eigenvalues along the line
  const double *mu_inner;  // eigenvalues along the inner axis
  int inner_packed;        // inner index c holds modes (2c, 2c+1) in (re, im)
  int inner_nmodes;
  const double *mu_outer;  // eigenvalues along the outer axis (or null)
  double scale;
  const void *qtw;     // QWS / QWC line axis: cpx<T> exp(-i pi j / 2N), j < 2N
  const double2 *dcs;  // DCT1 at length N, as for the rows
  void *data;          // cpx<T>, in place
  int B, ldsM;
  // SPH eigenvalue family (2D, every axis periodic): mu = sum_a sigma_a^2,
  // sigma_a = sph_norm Im S_a(inner, line) from the plan's symbol tables
  // (line coefficients symR per inner wavenumber, phase table ph_line); modes
  // with mu <= mu_tol get zero
  int sph;
  const double2 *symR;
  int sym_ninner;
  const double2 *ph_line;
  double sph_norm, mu_tol;
};

// ---------------------------------------------------------------- direct tap sums
// One tap of the compact kernel: lattice offset and the un-normalised weights
// dV d_x W, dV d_y W, dV d_z W, dV lap W at that offset.
struct Tap {
  int s[3];
  int pad;
  double w[4];
};

enum DirectMode {
  DIR_OPS = 0,       // grad / lap of one field into up to 4 outputs
  DIR_DIV = 1,       // scale * sum_a G_a u_a
  DIR_STEP_A = 2,    // u* (fused advection, viscosity, forcing, wall data)
  DIR_STEP_D = 3     // projection u = u* - dt/rho grad phi, wall reset
};

struct DirectArgs {
  int ndim;
  int n[3];
  int walled[3];
  int R;               // tap reach per axis (|s_a| <= R)
  FcWalls fc[3];       // per axis, for the field class being differentiated
  const Tap *taps;
  int ntaps;
  double wd[3][kSymW * kSymW];   // 2D dense weights (grad x, grad y, lap) at [(sy+R)*W + sx+R]
  const double *in[3]; // input fields (OPS: in[0]; DIV / STEP_A: velocity; STEP_D: phi)
  // outputs
  void *out[4];        // OPS: grad x, y, z, lap (null = skip); DIV: out[0]
  int out_is_double;
  double scale;
  // step
  const double *f[3], *wall[3], *ustar_in[3];
  double *ustar[3], *unew[3];
  double dt, nu, dt_over_rho;
  RkTerms rk;
  WallInfo wi;
  // FC ghost values of the inputs within R points of the lattice (2D):
  // gx[f] [ny][2R] (x = -R..-1, nx..nx+R-1), gy[f] [2R][nx+2R] (same slots in y,
  // column index x + R, corners included); filled by the ghost kernel
  double *gx[3], *gy[3];
};

hipError_t launch_direct(const DirectArgs &a, int mode, hipStream_t s);
hipError_t launch_ghost2d(const DirectArgs &a, int nfields, hipStream_t s);

// ---------------------------------------------------------------- FC standalone
struct FcExtArgs {
  const double *in;
  double *out;
  int axis_len;        // physical length along the axis
  long stride;         // element stride along the axis
  long nlines;         // number of lines
  long inner;          // lines are (outer, inner) with inner contiguous
  long outer_stride_in, outer_stride_out;
  long total_in_per_line_stride;
  FcWalls fc;
};

// ---------------------------------------------------------------- launch plumbing
// Kernel argument: the argument struct itself (one problem per launch), or a
// device array of them indexed by blockIdx.z (grouped launch: many problems
// with the same launch shape in one dispatch).
template <typename A, bool G>
struct KArg;
template <typename A>
struct KArg<A, false> {
  A a;
  // Read the fields through the kernel-argument segment pointer (this struct
  // is the kernel's only argument, at offset 0), as the grouped variant reads
  // its array: field loads then stay where they are used instead of the whole
  // struct being held in registers (which made the line kernels spill).
  __device__ __forceinline__ const A &get() const {
    return *(const A *)__builtin_amdgcn_kernarg_segment_ptr();
  }
};
template <typename A>
struct KArg<A, true> {
  const A *__restrict__ arr;
  __device__ __forceinline__ const A &get() const { return arr[blockIdx.z]; }
};

// One launch captured instead of issued: the grouped kernel, its per-problem
// launch shape and the bytes of its argument struct.
struct LaunchRecord {
  const void *gfunc;
  dim3 grid, block;
  size_t lds;
  std::vector<unsigned char> args;
};
struct Recorder {
  std::vector<LaunchRecord> recs;
};
// While non-null (per host thread), launchers append to it and issue nothing.
Recorder *&active_recorder();

template <typename K>
inline hipError_t set_kernel_lds(K kern, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Issue kernel `ks` on stream s, or record its grouped twin `kg`.
template <typename A, typename KS, typename KG>
inline hipError_t issue(KS ks, KG kg, const A &a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  if (Recorder *r = active_recorder()) {
    if (grid.z != 1) return hipErrorInvalidValue;
    hipError_t e = set_kernel_lds(kg, lds);
    if (e != hipSuccess) return e;
    LaunchRecord rec;
    rec.gfunc = reinterpret_cast<const void *>(kg);
    rec.grid = grid;
    rec.block = block;
    rec.lds = lds;
    rec.args.resize(sizeof(A));
    std::memcpy(rec.args.data(), &a, sizeof(A));
    r->recs.push_back(std::move(rec));
    return hipSuccess;
  }
  hipError_t e = set_kernel_lds(ks, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ks, grid, block, lds, s, KArg<A, false>{a});
  return hipGetLastError();
}

// LDS lines per column of the strided pass: OP and DIV keep a second line
// (the forward spectrum / the divergence accumulator).
inline int cols_lines_per_column(int mode, int ndim = 2) {
  return mode == COLS_PROJ ? ndim + 2 : (mode == COLS_OP || mode == COLS_DIV) ? 2 : 1;
}

// launchers (kernels.hip); return hipError_t
hipError_t launch_rows_fwd(const RowsFwdArgs &a, bool fp32, hipStream_t s);
hipError_t launch_rows_inv(const RowsInvArgs &a, int epi, bool fp32, hipStream_t s);
hipError_t launch_cols(const ColsArgs &a, int ninputs_grid, bool fp32, hipStream_t s);
hipError_t launch_ppe_rows(const PpeRowsArgs &a, bool fp32, hipStream_t s);
hipError_t launch_ppe_cols(const PpeColsArgs &a, bool fp32, hipStream_t s);
hipError_t launch_count_nonfinite(const double *x, size_t n, unsigned long long *counter, hipStream_t s);
hipError_t launch_fc_extend_axis(const double *in, double *out, int ndim, const int *shape_in,
                                 int axis, const FcWalls &fc, hipStream_t s);

}  // namespace fcsph
