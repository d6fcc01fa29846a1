// Direct evaluation of the spectral SPH operators for compact kernels.
//
// The operators are circular convolutions on the FC-extended periodic lattice
// (eq. circularConv): (G f)_i = sum_s w(s) e[(i - s) mod n_ext].  With a kernel
// whose support reaches R lattice points, an output at a physical point only
// needs the extended field within R points of the physical lattice: the
// physical values themselves and, across a wall, the first R continuation
// values of the periodic extension (the continuation wraps, so the points
// below the low wall are its last values).  Summing the taps directly gives
// the same result as the DFT route up to rounding, with one read of every
// input and one write of every output.
//
// Each workgroup stages a (TY + 2R) x (TX + 2R) tile of every input in LDS;
// values outside the physical lattice are produced on the fly: periodic axes
// wrap, walled axes evaluate the FC(Gram) continuation from the d values next
// to each wall (FP64), corners apply the two axes' continuations in order x
// then y (then z).
#include "fft_device.h"
#include "internal.h"

namespace fcsph {

namespace {

constexpr int TX = 64;       // tile width (x)
constexpr int NT = 256;      // threads per workgroup
constexpr int RMAX = kSymR;

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// continuation index (0-based, < C) of extended position g outside [0, n)
__device__ __forceinline__ int cont_index(int g, int n, int C) { return g >= n ? g - n : C + g; }

// FC continuation value of position g (outside [0,n)) of a line given by
// get(j).  The common d = 5 case is unrolled so that all 2d loads are in
// flight together.
template <int D, typename Get>
__device__ __forceinline__ double fc_at_d(const FcWalls &fc, int n, int i, Get get) {
  const double *hi = fc.Mhi + (size_t)i * D;
  const double *lo = fc.Mlo + (size_t)(fc.C - 1 - i) * D;
  double v[2 * D], m[2 * D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    v[j] = get(n - D + j);
    m[j] = hi[j];
    v[D + j] = get(D - 1 - j);
    m[D + j] = lo[j];
  }
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < 2 * D; ++j) acc = fma(m[j], v[j], acc);
  return acc;
}

template <typename Get>
__device__ __forceinline__ double fc_at(const FcWalls &fc, int n, int g, Get get) {
  const int i = cont_index(g, n, fc.C);
  if (fc.d == 5) return fc_at_d<5>(fc, n, i, get);
  const double *hi = fc.Mhi + (size_t)i * fc.d;
  const double *lo = fc.Mlo + (size_t)(fc.C - 1 - i) * fc.d;
  double acc = 0.0;
  for (int j = 0; j < fc.d; ++j) acc = fma(hi[j], get(n - fc.d + j), acc);
  for (int j = 0; j < fc.d; ++j) acc = fma(lo[j], get(fc.d - 1 - j), acc);
  return acc;
}

// Extended value of a 2D field at lattice position (x, y), |overshoot| <= R.
__device__ double ext2(const DirectArgs &a, const double *f, int x, int y) {
  const int nx = a.n[0], ny = a.n[1];
  if (!a.walled[0]) x = wrap(x, nx);
  if (!a.walled[1]) y = wrap(y, ny);
  const bool inx = x >= 0 && x < nx, iny = y >= 0 && y < ny;
  if (inx && iny) return f[(size_t)y * nx + x];
  if (!inx && iny) {
    const double *row = f + (size_t)y * nx;
    return fc_at(a.fc[0], nx, x, [&](int j) { return row[j]; });
  }
  if (inx && !iny) return fc_at(a.fc[1], ny, y, [&](int j) { return f[(size_t)j * nx + x]; });
  // corner: y continuation of the x-continued column
  return fc_at(a.fc[1], ny, y, [&](int j) {
    const double *row = f + (size_t)j * nx;
    return fc_at(a.fc[0], nx, x, [&](int jj) { return row[jj]; });
  });
}

// Ghost slot of an extended coordinate g outside [0, n): slots 0..R-1 hold
// g = -R..-1, slots R..2R-1 hold g = n..n+R-1.
__device__ __forceinline__ int ghost_slot(int g, int n, int R) { return g < 0 ? g + R : R + (g - n); }

// One thread per ghost value: x ghosts of every row, then y ghosts of every
// column of the x-extended lattice (corners: y continuation of x ghosts).
template <bool G>
__global__ void k_ghost2d(KArg<DirectArgs, G> ka) {
  const DirectArgs &a = ka.get();
  const int fi = blockIdx.y;
  const double *f = a.in[fi];
  const int nx = a.n[0], ny = a.n[1], R = a.R;
  const int nxg = a.walled[0] ? ny * 2 * R : 0;
  const int nyg = a.walled[1] ? 2 * R * (nx + 2 * R) : 0;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxg) {
    const int y = t / (2 * R), sl = t - y * 2 * R;
    const int x = sl < R ? sl - R : nx + (sl - R);
    const double *row = f + (size_t)y * nx;
    a.gx[fi][t] = fc_at(a.fc[0], nx, x, [&](int j) { return row[j]; });
  } else if (t < nxg + nyg) {
    const int u = t - nxg;
    const int sl = u / (nx + 2 * R), xc = u - sl * (nx + 2 * R);
    const int y = sl < R ? sl - R : ny + (sl - R);
    int x = xc - R;
    if (!a.walled[0]) x = wrap(x, nx);
    double v;
    if (x >= 0 && x < nx) {
      v = fc_at(a.fc[1], ny, y, [&](int j) { return f[(size_t)j * nx + x]; });
    } else {
      v = fc_at(a.fc[1], ny, y, [&](int j) {
        const double *row = f + (size_t)j * nx;
        return fc_at(a.fc[0], nx, x, [&](int jj) { return row[jj]; });
      });
    }
    a.gy[fi][u] = v;
  }
}

// Extended value at (x, y) from the field and its ghost arrays.
__device__ __forceinline__ double ext_g(const DirectArgs &a, int fi, int x, int y) {
  const int nx = a.n[0], ny = a.n[1], R = a.R;
  if (!a.walled[0]) x = wrap(x, nx);
  if (!a.walled[1]) y = wrap(y, ny);
  if (y >= 0 && y < ny) {
    if (x >= 0 && x < nx) return a.in[fi][(size_t)y * nx + x];
    return a.gx[fi][(size_t)y * 2 * R + ghost_slot(x, nx, R)];
  }
  return a.gy[fi][(size_t)ghost_slot(y, ny, R) * (nx + 2 * R) + (x + R)];
}

__device__ __forceinline__ bool dirichlet_pt(const WallInfo &w, int x, int y, int z) {
  const int c[3] = {x, y, z};
  for (int q = 0; q < w.ndim; ++q) {
    if (!w.walled[q]) continue;
    if (c[q] == 0 && w.dir[q][0]) return true;
    if (c[q] == w.n[q] - 1 && w.dir[q][1]) return true;
  }
  return false;
}

// Each thread computes RPT consecutive rows of one column; the input rows are
// streamed through a register window so that every LDS value read serves up
// to 2R+1 outputs.
constexpr int RPT = 4;                    // output rows per thread
constexpr int TYD = RPT * (NT / TX);      // tile height: 16 rows

template <int MODE, int R, bool G>
__global__ void __launch_bounds__(NT) k_direct2d(KArg<DirectArgs, G> ka) {
  const DirectArgs &a = ka.get();
  constexpr int NF = (MODE == DIR_DIV || MODE == DIR_STEP_A) ? 2 : 1;
  constexpr int W = TX + 2 * R, Hh = TYD + 2 * R;
  constexpr int SW = kSymW;
  __shared__ double tile[NF][Hh][W];
  const int nx = a.n[0], ny = a.n[1];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TYD;
  const bool interior = x0 - R >= 0 && x0 + TX + R <= nx && y0 - R >= 0 && y0 + TYD + R <= ny;
  if (interior) {
    constexpr int NIT = (W * Hh + NT - 1) / NT;
    double v[NF][NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < W * Hh) {
        const int ly = idx / W, lx = idx - ly * W;
        const size_t g = (size_t)(y0 + ly - R) * nx + (x0 + lx - R);
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) v[fi][it] = a.in[fi][g];
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < W * Hh) {
        const int ly = idx / W, lx = idx - ly * W;
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) tile[fi][ly][lx] = v[fi][it];
      }
    }
  } else {
    constexpr int NIT = (W * Hh + NT - 1) / NT;
    double v[NF][NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int ly = idx / W, lx = idx - ly * W;
      const int gx = x0 + lx - R, gy = y0 + ly - R;
      // positions beyond R of the lattice are never read
      if (idx < W * Hh && gx >= -R && gx < nx + R && gy >= -R && gy < ny + R) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) v[fi][it] = ext_g(a, fi, gx, gy);
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int ly = idx / W, lx = idx - ly * W;
      const int gx = x0 + lx - R, gy = y0 + ly - R;
      if (idx < W * Hh && gx >= -R && gx < nx + R && gy >= -R && gy < ny + R) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) tile[fi][ly][lx] = v[fi][it];
      }
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % TX, tg = threadIdx.x / TX;
  const int ty0 = tg * RPT;                 // first output row of this thread (tile coords)
  double acc[RPT][NF][3];
#pragma unroll
  for (int o = 0; o < RPT; ++o)
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) acc[o][fi][0] = acc[o][fi][1] = acc[o][fi][2] = 0.0;
  // (G e)_i = sum_s w(s) e[i - s]: output row ty0+o reads input tile row ty0+o+R-sy
#pragma unroll
  for (int iy = 0; iy < RPT + 2 * R; ++iy) {
    double row[NF][2 * R + 1];
#pragma unroll
    for (int fi = 0; fi < NF; ++fi)
#pragma unroll
      for (int sx = -R; sx <= R; ++sx) row[fi][sx + R] = tile[fi][ty0 + iy][tx + R - sx];
#pragma unroll
    for (int o = 0; o < RPT; ++o) {
      const int sy = o + R - iy;
      if (sy < -R || sy > R) continue;
#pragma unroll
      for (int sx = -R; sx <= R; ++sx) {
        const int wi = (sy + kSymR) * SW + (sx + kSymR);
        const double wx = a.wd[0][wi], wy = a.wd[1][wi], wl = a.wd[2][wi];
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          const double e = row[fi][sx + R];
          acc[o][fi][0] = fma(wx, e, acc[o][fi][0]);
          acc[o][fi][1] = fma(wy, e, acc[o][fi][1]);
          acc[o][fi][2] = fma(wl, e, acc[o][fi][2]);
        }
      }
    }
  }
  const int x = x0 + tx;
  if (x >= nx) return;
#pragma unroll
  for (int o = 0; o < RPT; ++o) {
    const int y = y0 + ty0 + o;
    if (y >= ny) break;
    const size_t off = (size_t)y * nx + x;
    if constexpr (MODE == DIR_OPS) {
      const double v[3] = {acc[o][0][0], acc[o][0][1], acc[o][0][2]};
      const int slot[3] = {0, 1, 3};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        void *dst = a.out[slot[q]];
        if (!dst) continue;
        if (a.out_is_double) static_cast<double *>(dst)[off] = v[q];
        else static_cast<float *>(dst)[off] = (float)v[q];
      }
    } else if constexpr (MODE == DIR_DIV) {
      const double dv = a.scale * (acc[o][0][0] + acc[o][1][1]);
      if (a.out_is_double) static_cast<double *>(a.out[0])[off] = dv;
      else static_cast<float *>(a.out[0])[off] = (float)dv;
    } else if constexpr (MODE == DIR_STEP_A) {
      const double u = tile[0][ty0 + o + R][tx + R], v = tile[1][ty0 + o + R][tx + R];
      const double fx = a.f[0] ? a.f[0][off] : 0.0, fy = a.f[1] ? a.f[1][off] : 0.0;
      double us = rk_ustar(a.rk, u, u * acc[o][0][0] + v * acc[o][0][1], a.nu, acc[o][0][2], fx, a.dt, off, 0);
      double vs = rk_ustar(a.rk, v, u * acc[o][1][0] + v * acc[o][1][1], a.nu, acc[o][1][2], fy, a.dt, off, 1);
      if (dirichlet_pt(a.wi, x, y, 0)) {
        us = a.wall[0] ? a.wall[0][off] : 0.0;
        vs = a.wall[1] ? a.wall[1][off] : 0.0;
      }
      a.ustar[0][off] = us;
      a.ustar[1][off] = vs;
    } else {   // DIR_STEP_D
      double un = a.ustar_in[0][off] - a.dt_over_rho * acc[o][0][0];
      double vn = a.ustar_in[1][off] - a.dt_over_rho * acc[o][0][1];
      if (dirichlet_pt(a.wi, x, y, 0)) {
        un = a.wall[0] ? a.wall[0][off] : 0.0;
        vn = a.wall[1] ? a.wall[1][off] : 0.0;
      }
      a.unew[0][off] = un;
      a.unew[1][off] = vn;
    }
  }
}

template <int MODE, int R>
hipError_t launch2d(const DirectArgs &a, hipStream_t s) {
  const dim3 grid((a.n[0] + TX - 1) / TX, (a.n[1] + TYD - 1) / TYD), block(NT);
  return issue(k_direct2d<MODE, R, false>, k_direct2d<MODE, R, true>, a, grid, block, 0, s);
}

template <int MODE>
hipError_t launch2d_r(const DirectArgs &a, hipStream_t s) {
  switch (a.R) {
    case 1: return launch2d<MODE, 1>(a, s);
    case 2: return launch2d<MODE, 2>(a, s);
    case 3: return launch2d<MODE, 3>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ghost2d(const DirectArgs &a, int nfields, hipStream_t s) {
  const int R = a.R;
  const int total = (a.walled[0] ? a.n[1] * 2 * R : 0) + (a.walled[1] ? 2 * R * (a.n[0] + 2 * R) : 0);
  if (total == 0) return hipSuccess;
  const dim3 grid((total + 255) / 256, nfields), block(256);
  return issue(k_ghost2d<false>, k_ghost2d<true>, a, grid, block, 0, s);
}

hipError_t launch_direct(const DirectArgs &a, int mode, hipStream_t s) {
  if (a.ndim != 2 || a.R < 1 || a.R > RMAX) return hipErrorInvalidValue;
  switch (mode) {
    case DIR_OPS: return launch2d_r<DIR_OPS>(a, s);
    case DIR_DIV: return launch2d_r<DIR_DIV>(a, s);
    case DIR_STEP_A: return launch2d_r<DIR_STEP_A>(a, s);
    case DIR_STEP_D: return launch2d_r<DIR_STEP_D>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcsph
