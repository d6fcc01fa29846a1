// HIP kernels of the FC(Gram)-based spectral ISPH step (gfx950).
//
// Pass structure of one spectral SPH operator on a 2D lattice (x fastest):
//   rows_fwd : FC along x (FP64) + real-to-complex DFT of every row, two real
//              rows packed into one complex line; writes the x half spectrum
//   cols OP  : per x wavenumber, FC along y (FP64, on complex data) + DFT along
//              y, multiplication by the operator symbol(s), inverse DFT along
//              y, restriction to the physical rows
//   rows_inv : inverse complex-to-real DFT along x, restriction to the
//              physical columns, fused point-wise epilogue
// 3D adds a forward and an inverse strided pass.  The PPE uses the same line
// engine with even / odd extensions (DCT-I / DST-I) or plain DFTs.
#include <algorithm>

#include "fft_device.h"
#include "internal.h"

namespace fcsph {

template <typename T>
__device__ __forceinline__ cpx<T> to_cpx(double r, double i) {
  return {static_cast<T>(r), static_cast<T>(i)};
}

// FC continuation value i (0-based, i < C) of a real line given by a
// callback returning line values as double.  d = 5 is unrolled so that the
// 2d loads are issued together.
template <typename Get>
__device__ __forceinline__ double fc_cont(const FcWalls &fc, int n, int i, Get get) {
  if (fc.d == 5) {
    const double *hi = fc.Mhi + (size_t)i * 5;
    const double *lo = fc.Mlo + (size_t)(fc.C - 1 - i) * 5;
    double v[10], m[10];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      v[j] = get(n - 5 + j);
      m[j] = hi[j];
      v[5 + j] = get(4 - j);
      m[5 + j] = lo[j];
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 10; ++j) acc = fma(m[j], v[j], acc);
    return acc;
  }
  const double *hi = fc.Mhi + (size_t)i * fc.d;
  const double *lo = fc.Mlo + (size_t)(fc.C - 1 - i) * fc.d;
  double acc = 0.0;
  for (int j = 0; j < fc.d; ++j) acc = fma(hi[j], get(n - fc.d + j), acc);
  for (int j = 0; j < fc.d; ++j) acc = fma(lo[j], get(fc.d - 1 - j), acc);
  return acc;
}

// ============================================================= rows forward
template <typename T, bool G>
__global__ void __launch_bounds__(kMaxThreads) k_rows_fwd(KArg<RowsFwdArgs, G> ka) {
  const RowsFwdArgs &a = ka.get();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *smem = reinterpret_cast<cpx<T> *>(smem_raw);
  const int TL = a.plan.TL;
  const int g = threadIdx.x / TL;
  const int lt = threadIdx.x - g * TL;
  const int line = blockIdx.x * a.B + g;
  Line<T> buf{smem + (size_t)g * a.ldsM};
  const bool active = line < a.nlines;
  const double *pa, *pb;
  if (a.map_per > 0) {
    // rows 2l, 2l+1 of inA, or (inB set) row l of inA and row l of inB
    const int rA = a.inB ? line : 2 * line, rB = a.inB ? line : 2 * line + 1;
    const double *srcB = a.inB ? a.inB : a.inA;
    pa = active ? a.inA + (size_t)(rA / a.map_per) * a.map_plane + (size_t)(rA % a.map_per) * a.nx : nullptr;
    pb = (active && line < a.nB) ? srcB + (size_t)(rB / a.map_per) * a.map_plane + (size_t)(rB % a.map_per) * a.nx
                                 : nullptr;
  } else {
    pa = active ? a.inA + (size_t)line * a.strideA : nullptr;
    pb = (active && line < a.nB && a.inB) ? a.inB + (size_t)line * a.strideB : nullptr;
  }
  batched<8, cpx<T>>(lt, a.nx, TL, [&](int j) { return to_cpx<T>(pa ? pa[j] : 0.0, pb ? pb[j] : 0.0); },
                     [&](int j, cpx<T> v) { buf[j] = v; });
  if (a.fc.on) {
    for (int j = a.nx + lt; j < a.E; j += TL) {
      const int i = fc_slot(a.fc, a.nx, a.E, j);
      double ra = (pa && i >= 0) ? fc_cont(a.fc, a.nx, i, [&](int q) { return pa[q]; }) : 0.0;
      double rb = (pb && i >= 0) ? fc_cont(a.fc, a.nx, i, [&](int q) { return pb[q]; }) : 0.0;
      buf[j] = to_cpx<T>(ra, rb);
    }
  }
  __syncthreads();
  line_dft<T>(buf, a.plan, lt, TL, false, false);
  if (active) {
    cpx<T> *oa = static_cast<cpx<T> *>(a.outA) + (size_t)line * a.ostrideA;
    cpx<T> *ob = pb ? static_cast<cpx<T> *>(a.outB) + (size_t)line * a.ostrideB : nullptr;
    const T half = T(0.5);
    for (int k = lt; k < a.H; k += TL) {
      const cpx<T> z = buf[k];
      const cpx<T> zc = cconj(buf[k == 0 ? 0 : a.E - k]);
      oa[k] = cscale(cadd(z, zc), half);
      if (ob) ob[k] = cscale(cmi(csub(z, zc)), half);
    }
  }
  if constexpr (sizeof(T) == 4) {
    if (a.edge_rows > 0) {
      // FP64 spectra of the boundary rows: every line group of a workgroup
      // that holds one runs the FP64 transform (the others inactive, through
      // the same barriers), on FP64 lines laid over the finished FP32 ones
      const int d = a.edge_rows;
      const int l0 = blockIdx.x * a.B, l1 = min(l0 + a.B, a.nlines);
      const bool wg_edge = l0 < d || l1 > a.ny - d;
      if (wg_edge) {
        const bool mine = active && (line < d || line >= a.ny - d);
        Line<double> b64{reinterpret_cast<cpx<double> *>(smem_raw) + (size_t)g * a.ldsM};
        __syncthreads();   // every group has read its FP32 line
        if (mine) {
          for (int j = lt; j < a.nx; j += TL) b64[j] = cpx<double>{pa[j], pb ? pb[j] : 0.0};
          if (a.fc.on)
            for (int j = a.nx + lt; j < a.E; j += TL) {
              const int i = fc_slot(a.fc, a.nx, a.E, j);
              const double ra = i >= 0 ? fc_cont(a.fc, a.nx, i, [&](int q) { return pa[q]; }) : 0.0;
              const double rb = (pb && i >= 0) ? fc_cont(a.fc, a.nx, i, [&](int q) { return pb[q]; }) : 0.0;
              b64[j] = cpx<double>{ra, rb};
            }
        }
        __syncthreads();
        line_dft<double>(b64, a.plan64, lt, TL, false, false, mine);
        if (mine) {
          const int e = line < d ? line : d + line - (a.ny - d);
          cpx<double> *oa = static_cast<cpx<double> *>(a.edgeA) + (size_t)e * a.H;
          cpx<double> *ob = pb ? static_cast<cpx<double> *>(a.edgeB) + (size_t)e * a.H : nullptr;
          for (int k = lt; k < a.H; k += TL) {
            const cpx<double> z = b64[k];
            const cpx<double> zc = cconj(b64[k == 0 ? 0 : a.E - k]);
            oa[k] = cscale(cadd(z, zc), 0.5);
            if (ob) ob[k] = cscale(cmi(csub(z, zc)), 0.5);
          }
        }
      }
    }
  }
}

// ============================================================= rows inverse
__device__ __forceinline__ bool is_dirichlet_point(const WallInfo &w, int x, int y, int z) {
  const int c[3] = {x, y, z};
  for (int a = 0; a < w.ndim; ++a) {
    if (!w.walled[a]) continue;
    if (c[a] == 0 && w.dir[a][0]) return true;
    if (c[a] == w.n[a] - 1 && w.dir[a][1]) return true;
  }
  return false;
}

// Load one packed complex line Z = A + i B from two half spectra (length H)
// of a real length-E signal: Z[k] = A[k] + i B[k], Z[E-k] = conj(A[k]) + i conj(B[k]).
template <typename T, bool CONJ = false>
__device__ __forceinline__ void load_packed_c2r(Line<T> buf, const cpx<T> *A, const cpx<T> *Bp,
                                                int E, int H, int lt, int TL) {
  struct AB {
    cpx<T> a, b;
  };
  batched<4, AB>(lt, H, TL,
                 [&](int k) {
                   return AB{A ? A[k] : cpx<T>{T(0), T(0)}, Bp ? Bp[k] : cpx<T>{T(0), T(0)}};
                 },
                 [&](int k, AB v) {
                   cpx<T> av = v.a, bv = v.b;
                   const bool selfconj = (k == 0) || (2 * k == E);
                   if (selfconj) {
                     av.i = T(0);
                     bv.i = T(0);
                   }
                   if (CONJ) {
                     // the input conjugation of an inverse DFT computed as
                     // conj(DFT(conj(.))); readers take -im of its output
                     buf[k] = {av.r - bv.i, -(av.i + bv.r)};
                     if (!selfconj) buf[E - k] = {av.r + bv.i, -(bv.r - av.i)};
                   } else {
                     buf[k] = {av.r - bv.i, av.i + bv.r};
                     if (!selfconj) buf[E - k] = {av.r + bv.i, bv.r - av.i};
                   }
                 });
}

__device__ __forceinline__ size_t spec_row(const RowsInvArgs &a, int r) {
  return ((size_t)(r / a.rpp) * a.prow + (r % a.rpp)) * (size_t)a.spec_pitch;
}

// At most 128 VGPRs (4 waves per SIMD): the 3D step epilogues run up to
// 512-thread workgroups, and at the compiler's own choice (137) only one of
// them fitted a CU; capped, two do (the 1024^2 step was 3 % faster when its
// epilogue had that form too).  The 2D step-A epilogue runs one 256-thread
// line group (four per CU, 113 VGPRs).
template <typename T, int EPI, bool GR>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_rows_inv(KArg<RowsInvArgs, GR> ka) {
  const RowsInvArgs &a = ka.get();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *smem = reinterpret_cast<cpx<T> *>(smem_raw);
  const int TL = a.plan.TL;
  const int g = threadIdx.x / TL;
  const int lt = threadIdx.x - g * TL;
  Line<T> buf{smem + (size_t)g * a.ldsM};
  const long P = a.spec_pitch;

  if constexpr (EPI == EPI_STORE) {
    // line = blockIdx.x * B + g; pack rows (2 line, 2 line + 1) of spec[0] when
    // spec[1] is null, otherwise row `line` of spec[0] and spec[1]
    const int line = blockIdx.x * a.B + g;
    const bool pair = a.spec[1] != nullptr;
    int rA = pair ? line : 2 * line;
    int rB = pair ? line : 2 * line + 1;
    const bool okA = rA < a.nrows, okB = rB < a.nrows;
    const cpx<T> *sA = okA ? static_cast<const cpx<T> *>(a.spec[0]) + spec_row(a, rA) : nullptr;
    const cpx<T> *sB = okB ? static_cast<const cpx<T> *>(pair ? a.spec[1] : a.spec[0]) + spec_row(a, rB) : nullptr;
    load_packed_c2r<T, true>(buf, sA, sB, a.E, a.H, lt, TL);
    __syncthreads();
    line_dft<T>(buf, a.plan, lt, TL, false, false);   // conjugated output: im = -z.i
    const int oB = pair ? 1 : 0;
    for (int x = lt; x < a.nx; x += TL) {
      const cpx<T> z = buf[x];
      if (a.out_is_double) {
        if (okA) static_cast<double *>(a.out[0])[(size_t)rA * a.nx + x] = a.scale * (double)z.r;
        if (okB) static_cast<double *>(a.out[oB])[(size_t)rB * a.nx + x] = a.scale * (double)(-z.i);
      } else {
        if (okA) static_cast<float *>(a.out[0])[(size_t)rA * a.nx + x] = (float)(a.scale * (double)z.r);
        if (okB) static_cast<float *>(a.out[oB])[(size_t)rB * a.nx + x] = (float)(a.scale * (double)(-z.i));
      }
    }
  } else if constexpr (EPI == EPI_ADVECT2) {
    const int row = blockIdx.x * a.B + g;
    const bool ok = row < a.nrows;
    const cpx<T> *sA = ok ? static_cast<const cpx<T> *>(a.spec[0]) + spec_row(a, row) : nullptr;
    const cpx<T> *sB = ok ? static_cast<const cpx<T> *>(a.spec[1]) + spec_row(a, row) : nullptr;
    load_packed_c2r<T, true>(buf, sA, sB, a.E, a.H, lt, TL);
    __syncthreads();
    line_dft<T>(buf, a.plan, lt, TL, false, false);   // conjugated output
    if (!ok) return;
    const size_t ro = (size_t)row * a.nx;
    for (int x = lt; x < a.nx; x += TL) {
      const double gx = (double)buf[x].r, gy = (double)(-buf[x].i);
      const double F = a.adv_c[0] * gx + a.adv_c[1] * gy;
      const double Fp = a.rk.z != 0.0 ? a.rk.F[0][ro + x] : 0.0;
      a.rk.F[0][ro + x] = F;
      double un = a.u[0][ro + x] - a.dt * (a.rk.g * F + a.rk.z * Fp);
      if (is_dirichlet_point(a.wi, x, row, 0)) un = a.wall[0] ? a.wall[0][ro + x] : 0.0;
      a.unew[0][ro + x] = un;
    }
  } else if constexpr (EPI == EPI_STEP_D2) {
    const int row = blockIdx.x * a.B + g;
    const bool ok = row < a.nrows;
    const cpx<T> *sA = ok ? static_cast<const cpx<T> *>(a.spec[0]) + spec_row(a, row) : nullptr;
    const cpx<T> *sB = ok ? static_cast<const cpx<T> *>(a.spec[1]) + spec_row(a, row) : nullptr;
    load_packed_c2r<T, true>(buf, sA, sB, a.E, a.H, lt, TL);
    __syncthreads();
    line_dft<T>(buf, a.plan, lt, TL, false, false);   // conjugated output
    if (!ok) return;
    const size_t ro = (size_t)row * a.nx;
    for (int x = lt; x < a.nx; x += TL) {
      double un = a.assign ? (double)buf[x].r : a.ustar[0][ro + x] - a.dt_over_rho * (double)buf[x].r;
      double vn = a.assign ? (double)(-buf[x].i) : a.ustar[1][ro + x] - a.dt_over_rho * (double)(-buf[x].i);
      if (is_dirichlet_point(a.wi, x, row, 0)) {
        un = a.wall[0] ? a.wall[0][ro + x] : 0.0;
        vn = a.wall[1] ? a.wall[1][ro + x] : 0.0;
      }
      a.unew[0][ro + x] = un;
      a.unew[1][ro + x] = vn;
    }
  } else if constexpr (EPI == EPI_STEP_A2) {
    // One row per workgroup and one line group: the three packed lines run in
    // turn through one LDS line, (L u, L v) first, then (Gx u, Gy u), then
    // (Gx v, Gy v).  Two real arrays after the line carry each thread's own
    // positions from one line to the next (L u then u*, and L v), so a
    // workgroup holds 1.4 lines of LDS instead of three and the 1024 rows of
    // a 1024^2 lattice are resident at once.  u* is stored only after the
    // last line has read u and v, which keeps an in-place call correct.
    const int row = blockIdx.x;
    const size_t ro_s = spec_row(a, row);
    const size_t ro = (size_t)row * a.nx;
    // the arrays start after one FP64 line, which the fused FP64 forward pass
    // of an FP32 kernel lays over its own (then finished) line
    double *keep_u = reinterpret_cast<double *>(smem_raw + (size_t)a.ldsM * sizeof(cpx<double>));   // L u, then u*
    double *keep_v = keep_u + a.nx;   // L v, then v* (FP32 kernels)
    constexpr int order[3] = {2, 0, 1};
    const int lt0 = lt;
#pragma unroll 1
    for (int s = 0; s < 3; ++s) {
      const int q = order[s];
      // a fresh copy of the lane index per line keeps the compiler from
      // hoisting the transform's lane-dependent LDS offsets out of this loop,
      // whose live ranges across the transforms spilled 52 B per lane to
      // scratch (13.6 MB of scratch writes per 1024^2 launch)
      int lt = lt0;
      asm volatile("" : "+v"(lt));
      load_packed_c2r<T, true>(buf, static_cast<const cpx<T> *>(a.spec[2 * q]) + ro_s,
                               static_cast<const cpx<T> *>(a.spec[2 * q + 1]) + ro_s, a.E, a.H, lt, TL);
      __syncthreads();
      line_dft<T>(buf, a.plan, lt, TL, false, false);   // conjugated output: im = -.i
      if (q == 2) {
        for (int x = lt; x < a.nx; x += TL) {
          keep_u[x] = (double)buf[x].r;
          keep_v[x] = (double)(-buf[x].i);
        }
      } else if (q == 0) {
        for (int x = lt; x < a.nx; x += TL) {
          const double u = a.u[0][ro + x], v = a.u[1][ro + x];
          const double gxu = buf[x].r, gyu = -buf[x].i;
          const double fx = a.f[0] ? a.f[0][ro + x] : 0.0;
          double us = rk_ustar(a.rk, u, u * gxu + v * gyu, a.nu, keep_u[x], fx, a.dt, ro + x, 0);
          if (is_dirichlet_point(a.wi, x, row, 0)) us = a.wall[0] ? a.wall[0][ro + x] : 0.0;
          keep_u[x] = us;
        }
      } else {
        for (int x = lt; x < a.nx; x += TL) {
          const double u = a.u[0][ro + x], v = a.u[1][ro + x];
          const double gxv = buf[x].r, gyv = -buf[x].i;
          const double fy = a.f[1] ? a.f[1][ro + x] : 0.0;
          double vs = rk_ustar(a.rk, v, u * gxv + v * gyv, a.nu, keep_v[x], fy, a.dt, ro + x, 1);
          if (is_dirichlet_point(a.wi, x, row, 0)) vs = a.wall[1] ? a.wall[1][ro + x] : 0.0;
          const double us = keep_u[x];
          a.ustar[0][ro + x] = us;
          a.ustar[1][ro + x] = vs;
          if constexpr (sizeof(T) == 8) {
            // position x of the line was read above by this thread only
            if (a.fwd_fused) buf[x] = to_cpx<T>(us, vs);
          } else {
            keep_v[x] = vs;   // position x of keep_v was read above by this thread only
          }
        }
      }
      __syncthreads();   // the line is read before the next load overwrites it
    }
    if (a.fwd_fused) {
      // the FP64 x forward pass of (u*, v*): FC along x, packed DFT, half
      // spectra (FP64 kernels: on buf itself, which holds (u*, v*) already;
      // FP32 kernels: on an FP64 line over the finished FP32 one, filled from
      // the arrays)
      Line<double> b64{reinterpret_cast<cpx<double> *>(smem_raw)};
      const LinePlan &plan64 = sizeof(T) == 8 ? a.plan : a.plan64;
      if constexpr (sizeof(T) == 4) {
        for (int x = lt; x < a.nx; x += TL) b64[x] = cpx<double>{keep_u[x], keep_v[x]};
        __syncthreads();
      }
      for (int j = a.nx + lt; j < a.E; j += TL) {
        const int i = fc_slot(a.fwd_fc, a.nx, a.E, j);
        double ra = 0.0, rb = 0.0;
        if (a.fwd_fc.on && i >= 0) {
          ra = fc_cont(a.fwd_fc, a.nx, i, [&](int q) { return b64[q].r; });
          rb = fc_cont(a.fwd_fc, a.nx, i, [&](int q) { return b64[q].i; });
        }
        b64[j] = cpx<double>{ra, rb};
      }
      __syncthreads();
      line_dft<double>(b64, plan64, lt, TL, false, false);
      cpx<double> *oa = static_cast<cpx<double> *>(a.fwd_out[0]) + (size_t)row * a.H;
      cpx<double> *ob = static_cast<cpx<double> *>(a.fwd_out[1]) + (size_t)row * a.H;
      for (int k = lt; k < a.H; k += TL) {
        const cpx<double> z = b64[k];
        const cpx<double> zc = cconj(b64[k == 0 ? 0 : a.E - k]);
        oa[k] = cscale(cadd(z, zc), 0.5);
        ob[k] = cscale(cmi(csub(z, zc)), 0.5);
      }
    }
  } else if constexpr (EPI == EPI_STEP_A3S) {
    // One row per workgroup and one line group: the six packed lines (Gx u,
    // Gy u), (Gz u, L u), (Gx v, Gy v), (Gz v, L v), (Gx w, Gy w), (Gz w, L w)
    // (spec[2q], spec[2q + 1]) run in turn through one LDS line.  Each thread
    // keeps its positions' u, v, w in registers (at most K positions:
    // nx <= K TL) and the partial advection sum and the finished u*, v* in
    // three real arrays after the line (its own positions only), so the
    // workgroup is one wave; u* is stored after the last line.
    constexpr int K = 4;
    const int row = blockIdx.x;
    const size_t ro_s = spec_row(a, row);
    const size_t ro = (size_t)row * a.nx;
    const int y = row % a.wi.n[1], z = row / a.wi.n[1];
    double *acc = reinterpret_cast<double *>(smem + (size_t)a.ldsM);   // u d/dx + v d/dy
    double *us = acc + a.nx, *vs = us + a.nx;                          // u*, v*
    double uu[K], vv[K], ww[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int x = lt + k * TL;
      const bool in = x < a.nx;
      uu[k] = in ? a.u[0][ro + x] : 0.0;
      vv[k] = in ? a.u[1][ro + x] : 0.0;
      ww[k] = in ? a.u[2][ro + x] : 0.0;
    }
    const int lt0 = lt;
#pragma unroll 1
    for (int q = 0; q < 6; ++q) {
      // a fresh copy of the lane index per line (no transform offsets hoisted
      // out of this loop, as in the 2D epilogue)
      int lt = lt0;
      asm volatile("" : "+v"(lt));
      load_packed_c2r<T, true>(buf, static_cast<const cpx<T> *>(a.spec[2 * q]) + ro_s,
                               static_cast<const cpx<T> *>(a.spec[2 * q + 1]) + ro_s, a.E, a.H, lt, TL);
      __syncthreads();
      line_dft<T>(buf, a.plan, lt, TL, false, false);   // conjugated output: im = -.i
      const int c = q >> 1;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int x = lt + k * TL;
        if (x >= a.nx) continue;
        const double re = (double)buf[x].r, im = (double)(-buf[x].i);
        if ((q & 1) == 0) {
          acc[x] = uu[k] * re + vv[k] * im;   // u d/dx + v d/dy of component c
          continue;
        }
        const double self = c == 0 ? uu[k] : (c == 1 ? vv[k] : ww[k]);
        const double f = a.f[c] ? a.f[c][ro + x] : 0.0;
        double st = rk_ustar(a.rk, self, acc[x] + ww[k] * re, a.nu, im, f, a.dt, ro + x, c);
        if (is_dirichlet_point(a.wi, x, y, z)) st = a.wall[c] ? a.wall[c][ro + x] : 0.0;
        if (c == 0) {
          us[x] = st;
        } else if (c == 1) {
          vs[x] = st;
        } else {
          a.ustar[0][ro + x] = us[x];
          a.ustar[1][ro + x] = vs[x];
          a.ustar[2][ro + x] = st;
        }
      }
      __syncthreads();   // the line is read before the next load overwrites it
    }
  } else {
    // One row per workgroup; NL packed lines, processed by the workgroup's
    // line groups in rounds (a group without a line in a round stays idle but
    // keeps the barriers).  Line buffers: NL consecutive slots of ldsM.
    //  A3: 0 (Gx u, Gy u) 1 (Gz u, Gx v) 2 (Gy v, Gz v) 3 (Gx w, Gy w) 4 (Gz w, L u) 5 (L v, L w)
    //      from spec[2q], spec[2q+1]
    //  D3: 0 (Gx p, Gy p) from spec[0], spec[1];  1 (Gz p, 0) from spec[2]
    constexpr int NL = EPI == EPI_STEP_A3 ? 6 : 2;
    const int G = blockDim.x / TL;
    const int row = blockIdx.x;
    const size_t ro_s = spec_row(a, row);
    for (int r0 = 0; r0 < NL; r0 += G) {
      const int q = r0 + g;
      const bool act = q < NL;
      Line<T> lb{smem + (size_t)(act ? q : 0) * a.ldsM};
      if (act) {
        const cpx<T> *sA, *sB;
        if constexpr (EPI == EPI_STEP_A3) {
          sA = static_cast<const cpx<T> *>(a.spec[2 * q]) + ro_s;
          sB = static_cast<const cpx<T> *>(a.spec[2 * q + 1]) + ro_s;
        } else {
          sA = static_cast<const cpx<T> *>(a.spec[q == 0 ? 0 : 2]) + ro_s;
          sB = q == 0 ? static_cast<const cpx<T> *>(a.spec[1]) + ro_s : nullptr;
        }
        load_packed_c2r<T, true>(lb, sA, sB, a.E, a.H, lt, TL);
      }
      __syncthreads();
      line_dft<T>(lb, a.plan, lt, TL, false, false, act);   // conjugated outputs: im = -.i
    }
    const size_t ro = (size_t)row * a.nx;
    if constexpr (EPI == EPI_STEP_A3) {
      Line<T> b[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) b[k] = Line<T>{smem + (size_t)k * a.ldsM};
      const int y = row % a.wi.n[1], z = row / a.wi.n[1];
      for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
        const double u = a.u[0][ro + x], v = a.u[1][ro + x], w = a.u[2][ro + x];
        const double gxu = b[0][x].r, gyu = -b[0][x].i, gzu = b[1][x].r;
        const double gxv = -b[1][x].i, gyv = b[2][x].r, gzv = -b[2][x].i;
        const double gxw = b[3][x].r, gyw = -b[3][x].i, gzw = b[4][x].r;
        const double lu = -b[4][x].i, lv = b[5][x].r, lw = -b[5][x].i;
        const double fx = a.f[0] ? a.f[0][ro + x] : 0.0;
        const double fy = a.f[1] ? a.f[1][ro + x] : 0.0;
        const double fz = a.f[2] ? a.f[2][ro + x] : 0.0;
        double us = rk_ustar(a.rk, u, u * gxu + v * gyu + w * gzu, a.nu, lu, fx, a.dt, ro + x, 0);
        double vs = rk_ustar(a.rk, v, u * gxv + v * gyv + w * gzv, a.nu, lv, fy, a.dt, ro + x, 1);
        double ws = rk_ustar(a.rk, w, u * gxw + v * gyw + w * gzw, a.nu, lw, fz, a.dt, ro + x, 2);
        if (is_dirichlet_point(a.wi, x, y, z)) {
          us = a.wall[0] ? a.wall[0][ro + x] : 0.0;
          vs = a.wall[1] ? a.wall[1][ro + x] : 0.0;
          ws = a.wall[2] ? a.wall[2][ro + x] : 0.0;
        }
        a.ustar[0][ro + x] = us;
        a.ustar[1][ro + x] = vs;
        a.ustar[2][ro + x] = ws;
      }
    } else {
      const Line<T> b0{smem}, b1{smem + a.ldsM};
      const int y = row % a.wi.n[1], z = row / a.wi.n[1];
      for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
        double un = a.assign ? (double)b0[x].r : a.ustar[0][ro + x] - a.dt_over_rho * (double)b0[x].r;
        double vn = a.assign ? (double)(-b0[x].i) : a.ustar[1][ro + x] - a.dt_over_rho * (double)(-b0[x].i);
        double wn = a.assign ? (double)b1[x].r : a.ustar[2][ro + x] - a.dt_over_rho * (double)b1[x].r;
        if (is_dirichlet_point(a.wi, x, y, z)) {
          un = a.wall[0] ? a.wall[0][ro + x] : 0.0;
          vn = a.wall[1] ? a.wall[1][ro + x] : 0.0;
          wn = a.wall[2] ? a.wall[2][ro + x] : 0.0;
        }
        a.unew[0][ro + x] = un;
        a.unew[1][ro + x] = vn;
        a.unew[2][ro + x] = wn;
      }
    }
  }
}

// ============================================================= strided passes
// Coefficients R[s] (s = -kSymR..kSymR along the line axis) of the symbol of
// operator q at fixed wavenumbers of the transverse axes,
//   S(k) = sum_s R[s] exp(-2 pi i k_line s / E_line),
// read from the plan's table (tabulated at plan creation: R[s] is the sum over
// the other offsets of the tap weight times the phases of the other axes'
// wavenumbers).  Uniform across a column's workgroup.
__device__ __forceinline__ void line_coeffs(const ColsArgs &a, int q, int kin, int kout, double2 *R) {
  const double2 *t = a.symR + (((size_t)q * a.ninner + kin) * a.nouter + (kout < 0 ? 0 : kout)) * kSymW;
#pragma unroll
  for (int s = 0; s < kSymW; ++s) R[s] = t[s];
}

// The symbol from the line coefficients R and the first phase factor
// p1 = exp(-2 pi i k / E) of line wavenumber k (from the plan's phase table,
// rounded once from extended precision); the powers s = 2, 3 by products (a
// few ulp on the symbol).
__device__ __forceinline__ double2 sym_from_phase(const double2 *R, double2 p1) {
  double2 p[kSymR + 1];
  p[1] = p1;
#pragma unroll
  for (int s = 2; s <= kSymR; ++s)
    p[s] = make_double2(p[s - 1].x * p[1].x - p[s - 1].y * p[1].y, p[s - 1].x * p[1].y + p[s - 1].y * p[1].x);
  double2 acc = R[kSymR];
#pragma unroll
  for (int s = 1; s <= kSymR; ++s) {
    const double2 rp = R[kSymR + s], rm = R[kSymR - s];
    // rp * p + rm * conj(p)
    acc.x += (rp.x + rm.x) * p[s].x - (rp.y - rm.y) * p[s].y;
    acc.y += (rp.x - rm.x) * p[s].y + (rp.y + rm.y) * p[s].x;
  }
  return acc;
}

__device__ __forceinline__ double2 line_phase(const double2 *ph_line, int k) {
  return ph_line[(size_t)k * (kSymR + 1) + 1];
}

__device__ __forceinline__ double2 sym_eval(const double2 *R, const double2 *ph_line, int k) {
  return sym_from_phase(R, line_phase(ph_line, k));
}


// Symbol q at inner wavenumber c, outer index o and line wavenumber k: from
// the plan's full table (kernels of unbounded support) or from the line
// coefficients R of the compact kernel.
// SF: the kernel instantiation that reads full symbol tables (kept separate,
// so the compact-kernel instantiations carry no extra registers for it).
template <bool SF>
__device__ __forceinline__ double2 sym_value(const ColsArgs &a, int q, int c, int o, const double2 *R,
                                             const double2 *ph_line, int k) {
  if constexpr (SF) return a.symF[(((size_t)q * a.ninner + c) * a.nouter + (o < 0 ? 0 : o)) * a.plan.n + k];
  else return sym_eval(R, ph_line, k);
}
// The same in two steps, so that a loop can issue the loads of several
// wavenumbers before it uses them: sym_load (one table read) and sym_finish.
template <bool SF>
__device__ __forceinline__ double2 sym_load(const ColsArgs &a, int q, int c, int o, const double2 *ph_line, int k) {
  if constexpr (SF) return a.symF[(((size_t)q * a.ninner + c) * a.nouter + (o < 0 ? 0 : o)) * a.plan.n + k];
  else return line_phase(ph_line, k);
}
template <bool SF>
__device__ __forceinline__ double2 sym_finish(const double2 *R, double2 v) {
  if constexpr (SF) return v;
  else return sym_from_phase(R, v);
}

template <bool SF>
__device__ __forceinline__ void line_coeffs_if(const ColsArgs &a, int q, int kin, int kout, double2 *R) {
  if constexpr (!SF) line_coeffs(a, q, kin, kout, R);
}

// CONJ loads the complex conjugate (the input conjugation of an inverse
// transform computed as conj(DFT(conj(x))), folded into the load).
template <typename T, bool CONJ = false>
__device__ __forceinline__ void cols_load(const ColsArgs &a, cpx<T> *smem, const cpx<T> *in,
                                          int c0, size_t obase, int n) {
  if (a.B == 1) {
    // one column per workgroup (the default): no division by the panel width
    const bool ok = c0 < a.ninner;
    batched<8, cpx<T>>(threadIdx.x, n, blockDim.x,
                       [&](int j) { return ok ? in[obase + (size_t)j * a.es + c0] : cpx<T>{T(0), T(0)}; },
                       [&](int j, cpx<T> v) { Line<T>{smem}[j] = CONJ ? cconj(v) : v; });
    return;
  }
  batched<8, cpx<T>>(threadIdx.x, a.B * n, blockDim.x,
                     [&](int idx) {
                       const int l = idx % a.B, j = idx / a.B;
                       const int c = c0 + l;
                       return c < a.ninner ? in[obase + (size_t)j * a.es + c] : cpx<T>{T(0), T(0)};
                     },
                     [&](int idx, cpx<T> v) {
                       const int l = idx % a.B, j = idx / a.B;
                       Line<T>{smem + (size_t)l * a.ldsM}[j] = CONJ ? cconj(v) : v;
                     });
}

// CONJ stores the complex conjugate (the output conjugation of an inverse
// transform computed as conj(DFT(conj(x))), folded into the store).
template <typename T, bool CONJ = false>
__device__ __forceinline__ void cols_store(const ColsArgs &a, const cpx<T> *smem, cpx<T> *out,
                                           int c0, size_t obase, int n) {
  auto val = [](cpx<T> v) { return CONJ ? cconj(v) : v; };
  if (a.B == 1) {
    if (c0 < a.ninner)
      for (int j = threadIdx.x; j < n; j += blockDim.x)
        out[obase + (size_t)j * a.es_out + c0] = val(Line<T>{const_cast<cpx<T> *>(smem)}[j]);
    return;
  }
  for (int idx = threadIdx.x; idx < a.B * n; idx += blockDim.x) {
    const int l = idx % a.B, j = idx / a.B;
    const int c = c0 + l;
    if (c < a.ninner)
      out[obase + (size_t)j * a.es_out + c] = val(Line<T>{const_cast<cpx<T> *>(smem) + (size_t)l * a.ldsM}[j]);
  }
}

template <typename T>
__device__ __forceinline__ void cols_fc(const ColsArgs &a, Line<T> buf, int lt, int TL, int f, int c, int o) {
  const int n = a.nload, L = a.plan.n;
  const double2 *edge = a.edge[f];
  const int d = a.fc.d;
  // FP64 boundary rows when the plan keeps them (FP32 spectra would carry
  // their rounding, amplified by the continuation maps, into the extension)
  auto val = [&](int q) -> double2 {
    if (edge) {
      const int h = q < d ? 0 : 1, r = q < d ? q : q - (n - d);
      return edge[(((size_t)h * a.nouter + o) * d + r) * a.ninner + (c < a.ninner ? c : 0)];
    }
    return make_double2((double)buf[q].r, (double)buf[q].i);
  };
  for (int j = n + lt; j < L; j += TL) {
    const int i = fc_slot(a.fc, n, L, j);
    double re = 0.0, im = 0.0;
    if (i >= 0) {
      re = fc_cont(a.fc, n, i, [&](int q) { return val(q).x; });
      im = fc_cont(a.fc, n, i, [&](int q) { return val(q).y; });
    }
    buf[j] = to_cpx<T>(re, im);
  }
}

// At most 128 VGPRs (4 waves per SIMD): with the symbol coefficients read from
// the plan's table the column kernels need 105-137; capped, only the FP64
// operator form spills (12 B per lane), and the 1024^2 step gains 1 %, the
// 256^3 step 2.5 % (four 4-wave workgroups per CU, as the LDS allows).  The
// FP32 operator form (single-problem launch) is held to 96 VGPRs, 5 waves per
// SIMD: its two FP32 lines of LDS per workgroup let five workgroups share a
// CU, so the 1122 (field, column) tasks of the 1024^2 stage-A pass run in one
// round instead of two (no spill; the grouped batch form would spill and
// keeps 4).
template <typename T, int MODE, bool G, bool SF = false>
__global__ void __launch_bounds__(kMaxThreads)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MODE == COLS_OP && !G) ? 5 : 4)))
k_cols(KArg<ColsArgs, G> ka) {
  const ColsArgs &a = ka.get();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *smem = reinterpret_cast<cpx<T> *>(smem_raw);
  const int TL = a.plan.TL;
  const int g = threadIdx.x / TL;
  const int lt = threadIdx.x - g * TL;
  Line<T> buf{smem + (size_t)g * a.ldsM};
  const int npanel = (a.ninner + a.B - 1) / a.B;
  // task = (input field f, panel); normally f = blockIdx.y.  A split launch
  // (COLS_OP only) numbers the tasks linearly, field-major: workgroup b <
  // nfull runs task b whole, a later one runs output qsel of task
  // nfull + (b - nfull) / nout.  Every output is formed by the same code
  // either way.
  int f = blockIdx.y, bx = blockIdx.x, nbx = gridDim.x, qsel = -1;
  if constexpr (!G && MODE == COLS_OP) {
    if (a.nfull > 0) {
      const int npo = npanel * a.nouter;
      int t = blockIdx.x;
      if (t >= a.nfull) {
        const int r = t - a.nfull, q = r / a.nout;
        t = a.nfull + q;
        qsel = r - q * a.nout;
      }
      f = t / npo;
      bx = t - f * npo;
      nbx = npo;
    }
  }
  const int bid = xcd_panel(bx, nbx);
  const int o = bid / npanel;
  const int c0 = (bid - o * npanel) * a.B;
  const int c = c0 + g;
  const size_t obase_in = (size_t)o * a.os_in, obase_out = (size_t)o * a.os_out;
  const int E = a.plan.n;
  const double2 *ph_line = a.st.ph[a.line_axis];

  if constexpr (MODE == COLS_FWD || MODE == COLS_INV) {
    // COLS_INV loads the whole line (nload == plan length) and computes the
    // inverse as conj(DFT(conj(.))) with the conjugations in the load and store
    constexpr bool inv = MODE == COLS_INV;
    const cpx<T> *in = static_cast<const cpx<T> *>(a.in[f]);
    cols_load<T, inv>(a, smem, in, c0, obase_in, a.nload);
    __syncthreads();
    if (MODE == COLS_FWD && a.fc.on) {
      cols_fc<T>(a, buf, lt, TL, f, c, o);
      __syncthreads();
    }
    line_dft<T>(buf, a.plan, lt, TL, false, false);
    cols_store<T, inv>(a, smem, static_cast<cpx<T> *>(a.out[f][0]), c0, obase_out, a.nstore);
  } else if constexpr (MODE == COLS_OP) {
    // pass 0: FC + forward DFT in place (the spectrum stays in buf); pass
    // q + 1: symbol q times buf into a second LDS line (xb), inverse DFT
    // there, store.  One transform call site (on a line chosen per pass)
    // keeps the kernel's register footprint at that of a single transform.
    Line<T> xb{smem + (size_t)(a.B + g) * a.ldsM};
    for (int pass = 0; pass <= a.nout; ++pass) {
      if (pass > 0 && qsel >= 0 && pass != qsel + 1) continue;   // uniform per workgroup
      if (pass == 0) {
        cols_load<T>(a, smem, static_cast<const cpx<T> *>(a.in[f]), c0, obase_in, a.nload);
        __syncthreads();
        if (a.fc.on) {
          cols_fc<T>(a, buf, lt, TL, f, c, o);
          __syncthreads();
        }
      } else {
        double2 R[kSymW];
        const int cq = c < a.ninner ? c : 0;
        line_coeffs_if<SF>(a, a.sym[pass - 1], cq, o, R);
        __syncthreads();   // the previous output's store has finished reading xb
        // the inverse DFT is conj(DFT(conj(.))): the input conjugation is
        // folded into the symbol product, the output one into the store
        const int q = a.sym[pass - 1];
        batched<5, double2>(lt, E, TL, [&](int k) { return sym_load<SF>(a, q, cq, o, ph_line, k); },
                            [&](int k, double2 v) {
                              const double2 sv = sym_finish<SF>(R, v);
                              xb[k] = cconj(cmul(to_cpx<T>(sv.x, sv.y), buf[k]));
                            });
        __syncthreads();
      }
      line_dft<T>(pass == 0 ? buf : xb, a.plan, lt, TL, false, false);
      if (pass > 0)
        cols_store<T, true>(a, smem + (size_t)a.B * a.ldsM, static_cast<cpx<T> *>(a.out[f][pass - 1]), c0,
                            obase_out, a.nstore);
    }
  } else if constexpr (MODE == COLS_PROJ) {
    // One column per workgroup (B == 1).  Lines 0..nin-1: the spectra e_a of
    // the velocity components (FC along the line); line nin: the pressure
    // spectrum; line nin + 1: the divergence D = sum_a S_a e_a.
    const int nin = a.st.ndim;
    const int cc = c < a.ninner ? c : 0;
    Line<T> P{smem + (size_t)nin * a.ldsM}, D{smem + (size_t)(nin + 1) * a.ldsM};
    for (int f = 0; f < nin; ++f) {
      Line<T> Lf{smem + (size_t)f * a.ldsM};
      cols_load<T>(a, smem + (size_t)f * a.ldsM, static_cast<const cpx<T> *>(a.in[f]), c0, obase_in, a.nload);
      __syncthreads();
      if (a.fc.on) {
        cols_fc<T>(a, Lf, lt, TL, f, c, o);
        __syncthreads();
      }
      line_dft<T>(Lf, a.plan, lt, TL, false, false);
    }
    // D and sum_a S_a^2 (real part of the squares: the symbols are odd, so
    // purely imaginary up to rounding), accumulated symbol by symbol
    for (int f = 0; f < nin; ++f) {
      double2 R[kSymW];
      line_coeffs_if<SF>(a, a.sym[f], cc, o, R);
      const Line<T> Lf{smem + (size_t)f * a.ldsM};
      for (int k = lt; k < E; k += TL) {
        const double2 sv = sym_value<SF>(a, a.sym[f], cc, o, R, ph_line, k);
        const cpx<T> e = Lf[k];
        const cpx<T> t = cmul(to_cpx<T>(sv.x, sv.y), e);
        const T sq = T(sv.x * sv.x - sv.y * sv.y);
        if (f == 0) {
          D[k] = t;
          P[k] = {sq, T(0)};
        } else {
          D[k] = cadd(D[k], t);
          P[k].r += sq;
        }
      }
    }
    // phi = D / (dt/rho sum S^2) (table units), zero where the sum vanishes
    for (int k = lt; k < E; k += TL) {
      const T sq = P[k].r;
      const cpx<T> d = D[k];
      const bool ok = fabs((double)sq) > a.proj_tol;
      const T den = T(a.proj_dtr) * (ok ? sq : T(1));
      P[k] = ok ? cpx<T>{d.r / den, d.i / den} : cpx<T>{T(0), T(0)};
    }
    // corrected spectra e_a - (dt/rho) S_a phi; the inverse transforms are
    // conj(DFT(conj(.))), the input conjugation folded in here
    const T s1 = T(a.proj_inv_norm);
    for (int f = 0; f < nin; ++f) {
      double2 R[kSymW];
      line_coeffs_if<SF>(a, a.sym[f], cc, o, R);
      Line<T> Lf{smem + (size_t)f * a.ldsM};
      for (int k = lt; k < E; k += TL) {
        const double2 sv = sym_value<SF>(a, a.sym[f], cc, o, R, ph_line, k);
        const cpx<T> corr = cmul(to_cpx<T>(sv.x, sv.y), P[k]);
        const cpx<T> e = Lf[k];
        const cpx<T> v = {e.r - T(a.proj_dtr) * corr.r, e.i - T(a.proj_dtr) * corr.i};
        Lf[k] = cconj(cscale(v, s1));
      }
    }
    for (int k = lt; k < E; k += TL) P[k] = cconj(cscale(P[k], T(a.proj_inv_norm * a.proj_inv_norm)));
    __syncthreads();
    for (int f = 0; f <= nin; ++f) {
      line_dft<T>(Line<T>{smem + (size_t)f * a.ldsM}, a.plan, lt, TL, false, false);
      cols_store<T, true>(a, smem + (size_t)f * a.ldsM, static_cast<cpx<T> *>(a.out[0][f]), c0, obase_out,
                          a.nstore);
    }
  } else {
    // COLS_DIV: out = sum_f S_f DFT(FC(in_f)), one output; passes 0..nin-1
    // transform input f and accumulate in a second LDS line (each thread owns
    // its positions), the last pass inverts the sum
    Line<T> acc{smem + (size_t)(a.B + g) * a.ldsM};
    for (int k = lt; k < E; k += TL) acc[k] = {T(0), T(0)};
    const int nin = a.st.ndim;
    for (int pass = 0; pass <= nin; ++pass) {
      __syncthreads();
      if (pass < nin) {
        cols_load<T>(a, smem, static_cast<const cpx<T> *>(a.in[pass]), c0, obase_in, a.nload);
        __syncthreads();
        if (a.fc.on) {
          cols_fc<T>(a, buf, lt, TL, pass, c, o);
          __syncthreads();
        }
      } else {
        // inverse as conj(DFT(conj(.))), conjugations folded into this copy and the store
        for (int k = lt; k < E; k += TL) buf[k] = cconj(acc[k]);
        __syncthreads();
      }
      line_dft<T>(buf, a.plan, lt, TL, false, false);
      if (pass < nin) {
        double2 R[kSymW];
        const int cq = c < a.ninner ? c : 0;
        line_coeffs_if<SF>(a, a.sym[pass], cq, o, R);
        for (int k = lt; k < E; k += TL) {
          const double2 sv = sym_value<SF>(a, a.sym[pass], cq, o, R, ph_line, k);
          acc[k] = cadd(acc[k], cmul(to_cpx<T>(sv.x, sv.y), buf[k]));
        }
      }
    }
    cols_store<T, true>(a, smem, static_cast<cpx<T> *>(a.out[0][0]), c0, obase_out, a.nstore);
  }
}

// ============================================================= DCT-I / DST-I at length N
// The DFT of the even (DCT-I) or odd (DST-I) extension of length 2N of the
// N + 1 values f = buf[0..N] of a complex line,
//   DCT-I: Z_k = f_0 + (-1)^k f_N + 2 sum_{j=1}^{N-1} f_j cos(pi j k / N),
//   DST-I: Z_k = -2i sum_{j=1}^{N-1} f_j sin(pi j k / N)   (f_0 = f_N = 0),
// k = 0..N, computed from one DFT of length N (Y = DFT_N(y), j < N):
//   DCT-I: y_j = (f_j + f_{N-j}) / 2 - sin(pi j / N) (f_j - f_{N-j});
//          Z_{2k} = Y_k + Y_{N-k},  Z_{2k+1} = Z_{2k-1} + i (Y_k - Y_{N-k}),
//          started at Z_1 = f_0 - f_N + 2 sum_{j=1}^{N-1} f_j cos(pi j / N);
//   DST-I: y_j = sin(pi j / N) (f_j + f_{N-j}) + (f_j - f_{N-j}) / 2;
//          Z_{2k} = Y_k - Y_{N-k},  Z_{2k+1} = -i W_{2k+1} with
//          W_{2k+1} = W_{2k-1} + Y_k + Y_{N-k}, started at W_1 = Y_0.
// (The symmetric / antisymmetric parts of y under j -> N - j carry the even
// and odd outputs.)  trig1_pre forms y in place and returns the DCT-I start
// Z_1 (every thread of the line group holds it); the caller runs the
// length-N transform (plan p) on buf; trig1_post forms Z into buf[0..N].
// Line buffer: [0, M) transform, [M + 1, M + N + 2) the result (clear of
// buf[0..N] also when M == N), then 8 slots for per-wave partial sums.
// cs[j] = (cos, sin)(pi j / N) for j <= N / 2.  Line groups are whole waves
// (TL is a multiple of 64).
template <typename T>
__device__ __forceinline__ cpx<T> wave_incl_scan(cpx<T> v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T r = __shfl_up(v.r, d, 64), i = __shfl_up(v.i, d, 64);
    if (lane >= d) {
      v.r += r;
      v.i += i;
    }
  }
  return v;
}

template <typename T>
__device__ __forceinline__ cpx<T> trig1_pre(Line<T> buf, const LinePlan &p, const double2 *cs, bool sine,
                                            int lt, int TL) {
  const int N = p.n, H = N / 2;
  const int tail = p.M + N + 2;
  cpx<T> z = {T(0), T(0)};
  for (int j = lt; j <= H; j += TL) {
    if (j == 0) {
      const cpx<T> a = buf[0], b = buf[N];
      buf[0] = cscale(sine ? csub(a, b) : cadd(a, b), T(0.5));
      z = csub(a, b);
    } else if (2 * j != N) {
      // positions j and N - j belong to this thread only
      const cpx<T> a = buf[j], b = buf[N - j];
      const double2 w = cs[j];
      const T s = T(w.y), c2 = T(2.0 * w.x);
      const cpx<T> h = cscale(cadd(a, b), T(0.5)), d = csub(a, b);
      if (sine) {
        const T s2 = s + s;
        const cpx<T> u = {s2 * h.r, s2 * h.i}, v = cscale(d, T(0.5));
        buf[j] = cadd(u, v);
        buf[N - j] = csub(u, v);
      } else {
        buf[j] = {h.r - s * d.r, h.i - s * d.i};
        buf[N - j] = {h.r + s * d.r, h.i + s * d.i};
        z = {z.r + c2 * d.r, z.i + c2 * d.i};
      }
    } else if (sine) {
      buf[j] = cscale(buf[j], T(2));     // sin(pi / 2) (f + f)
    }
  }
  z = wave_incl_scan(z);
  if ((threadIdx.x & 63) == 63) buf[tail + (lt >> 6)] = z;
  __syncthreads();
  cpx<T> z1 = {T(0), T(0)};
  if (!sine)
    for (int w = 0; w < (TL >> 6); ++w) z1 = cadd(z1, buf[tail + w]);
  return z1;
}

template <typename T>
__device__ __forceinline__ void trig1_post(Line<T> buf, const LinePlan &p, cpx<T> z1, bool sine, int lt,
                                           int TL) {
  const int N = p.n, H = N / 2, O = p.M + 1;
  const int tail = O + N + 1;
  // k = 0..H in contiguous chunks per thread: even output 2k, odd output
  // 2k + 1 (while 2k + 1 <= N) as a chunk-local running sum first
  const int q = (H + TL) / TL;
  const int k0 = lt * q, k1 = min(k0 + q, H + 1);
  cpx<T> run = {T(0), T(0)};
  for (int k = k0; k < k1; ++k) {
    const cpx<T> yk = buf[k], ynk = buf[k == 0 ? 0 : N - k];
    if (sine) {
      buf[O + 2 * k] = k == 0 ? cpx<T>{T(0), T(0)} : csub(yk, ynk);
      run = cadd(run, k == 0 ? yk : cadd(yk, ynk));
    } else {
      buf[O + 2 * k] = cadd(yk, ynk);
      if (k > 0) run = cadd(run, cpi(csub(yk, ynk)));
    }
    if (2 * k + 1 <= N) buf[O + 2 * k + 1] = run;
  }
  // offsets: the start value + the sums of the chunks before this thread's
  const cpx<T> incl = wave_incl_scan(run);
  if ((threadIdx.x & 63) == 63) buf[tail + (lt >> 6)] = incl;
  __syncthreads();
  cpx<T> off = cadd(z1, csub(incl, run));
  for (int w = 0; w < (lt >> 6); ++w) off = cadd(off, buf[tail + w]);
  for (int k = k0; k < k1; ++k)
    if (2 * k + 1 <= N) {
      const cpx<T> v = cadd(buf[O + 2 * k + 1], off);
      buf[O + 2 * k + 1] = sine ? cmi(v) : v;
    }
  __syncthreads();
  for (int k = lt; k <= N; k += TL) buf[k] = buf[O + k];
  __syncthreads();
}

// ============================================================= PPE rows
// Coefficient row layout: DCT-I / DST-I rows are real; coefficient m of a row
// is stored in component (m & 1) of complex slot m >> 1.  DFT rows are complex
// half spectra.
template <typename T>
__device__ __forceinline__ void put_real_coef(cpx<T> *row, int m, T v) {
  T *p = reinterpret_cast<T *>(row + (m >> 1));
  p[m & 1] = v;
}
template <typename T>
__device__ __forceinline__ T get_real_coef(const cpx<T> *row, int m) {
  const T *p = reinterpret_cast<const T *>(row + (m >> 1));
  return p[m & 1];
}

template <typename T, bool G, bool W>
__global__ void __launch_bounds__(kMaxThreads) k_ppe_rows(KArg<PpeRowsArgs, G> ka) {
  const PpeRowsArgs &a = ka.get();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *smem = reinterpret_cast<cpx<T> *>(smem_raw);
  const int TL = a.plan.TL;
  const int g = threadIdx.x / TL;
  const int lt = threadIdx.x - g * TL;
  Line<T> buf{smem + (size_t)g * a.ldsM};
  const int line = blockIdx.x * a.B + g;
  const int rA = 2 * line, rB = 2 * line + 1;
  const bool okA = rA < a.nrows, okB = rB < a.nrows;
  const int n = a.nx, L = a.plan.n;
  cpx<T> *cA = static_cast<cpx<T> *>(a.coef) + (size_t)rA * a.cpitch;
  cpx<T> *cB = static_cast<cpx<T> *>(a.coef) + (size_t)rB * a.cpitch;
  auto val = [&](int r, int j) -> double {
    const size_t o = (size_t)r * n + j;
    return a.in_real ? a.in_real[o] : (double)a.in_float[o];
  };

  // ---- line set-up: values (forward) or coefficients (inverse), extended
  const bool qw = a.kind == TRIG_QWS || a.kind == TRIG_QWC;
  const cpx<T> *qtw = static_cast<const cpx<T> *>(a.qtw);
  if (!a.inverse && a.spec) {
    // the rows from their x half spectrum (the divergence's last pass fused
    // in): packed C2R, then the values the C2R store would have written
    // (conjugated output: row A = Re z, row B = -Im z), unknowns only
    const cpx<T> *sp = static_cast<const cpx<T> *>(a.spec);
    load_packed_c2r<T, true>(buf, okA ? sp + (size_t)rA * a.spec_pitch : nullptr,
                             okB ? sp + (size_t)rB * a.spec_pitch : nullptr, a.xE, a.xH, lt, TL);
    __syncthreads();
    line_dft<T>(buf, a.xplan, lt, TL, false, false);
    const int jl = a.kind == TRIG_DST1 || a.kind == TRIG_QWS ? 1 : 0;
    const int jh = a.kind == TRIG_DST1 || a.kind == TRIG_QWC ? n - 2 : n - 1;
    for (int j = lt; j < n; j += TL) {
      const cpx<T> z = buf[j];
      double va = a.in_scale * (double)z.r, vb = a.in_scale * (double)(-z.i);
      if (a.round32) {
        va = (double)(float)va;
        vb = (double)(float)vb;
      }
      const bool in = j >= jl && j <= jh;
      buf[j] = to_cpx<T>(okA && in ? va : 0.0, okB && in ? vb : 0.0);
    }
  } else if (!a.inverse) {
    if (a.kind == TRIG_DST1 || qw) {
      // unknowns only: DST1 1..n-2, QWS 1..n-1, QWC 0..n-2 (wall values are
      // zero); the extension is formed in LDS below
      const int jl = a.kind == TRIG_QWC ? 0 : 1;
      const int jh = a.kind == TRIG_QWS ? n - 1 : n - 2;
      batched<8, cpx<T>>(lt, n, TL,
                         [&](int j) {
                           const bool in = j >= jl && j <= jh;
                           return to_cpx<T>(okA && in ? val(rA, j) : 0.0, okB && in ? val(rB, j) : 0.0);
                         },
                         [&](int j, cpx<T> v) { buf[j] = v; });
    } else {
      batched<8, cpx<T>>(lt, n, TL, [&](int j) { return to_cpx<T>(okA ? val(rA, j) : 0.0, okB ? val(rB, j) : 0.0); },
                         [&](int j, cpx<T> v) { buf[j] = v; });
    }
  } else {
    if (a.kind == TRIG_DFT) {
      load_packed_c2r<T>(buf, okA ? cA : nullptr, okB ? cB : nullptr, n, a.ncoef, lt, TL);
    } else if (a.kind == TRIG_DCT1) {
      for (int j = lt; j < n; j += TL)
        buf[j] = {okA ? get_real_coef<T>(cA, j) : T(0), okB ? get_real_coef<T>(cB, j) : T(0)};
    } else if (qw) {
      for (int j = lt; j < n - 1; j += TL)
        buf[j] = {okA ? get_real_coef<T>(cA, j) : T(0), okB ? get_real_coef<T>(cB, j) : T(0)};
    } else {
      for (int j = lt; j < n; j += TL) {
        const bool in = j > 0 && j < n - 1;
        buf[j] = {okA && in ? get_real_coef<T>(cA, j - 1) : T(0), okB && in ? get_real_coef<T>(cB, j - 1) : T(0)};
      }
    }
  }
  __syncthreads();
  const bool half = (a.kind == TRIG_DCT1 || a.kind == TRIG_DST1) && a.dcs;
  if (a.kind == TRIG_DCT1) {
    if (!half)
      for (int j = n + lt; j < L; j += TL) buf[j] = buf[L - j];           // even extension
  } else if (a.kind == TRIG_DST1) {
    if (!half)
      for (int j = n + lt; j < L; j += TL) buf[j] = cscale(buf[L - j], T(-1));   // odd extension
  } else if (qw && !a.inverse) {
    // samples N+1 .. 2N-1 of the quarter-wave extension: +x (QWS) / -x (QWC) at 2N - j
    const T sg = a.kind == TRIG_QWS ? T(1) : T(-1);
    for (int j = n + lt; j < L; j += TL) buf[j] = cscale(buf[L - j], sg);
    __syncthreads();
    for (int j = lt; j < L; j += TL) buf[j] = cmul(buf[j], qtw[j]);
  } else if (qw) {
    // odd-frequency coefficients 2N-1-l mirror l: -F (QWS) / +F (QWC)
    const T sg = a.kind == TRIG_QWS ? T(-1) : T(1);
    for (int j = n - 1 + lt; j < L; j += TL) buf[j] = cscale(buf[L - 1 - j], sg);
  }
  __syncthreads();
  cpx<T> z1 = {T(0), T(0)};
  if (half) z1 = trig1_pre<T>(buf, a.plan, a.dcs, a.kind == TRIG_DST1, lt, TL);
  const bool cj = a.inverse && (a.kind == TRIG_DFT || qw);
  // streamed radix stages in the single-problem kernel only (batched plans
  // never use them), which keeps the grouped kernel's registers
  line_dft<T, !G, W>(buf, a.plan, lt, TL, cj, cj);
  if (half) trig1_post<T>(buf, a.plan, z1, a.kind == TRIG_DST1, lt, TL);

  // ---- results
  if (!a.inverse) {
    if (a.kind == TRIG_DFT) {
      const T half = T(0.5);
      for (int k = lt; k < a.ncoef; k += TL) {
        const cpx<T> z = buf[k], zc = cconj(buf[k == 0 ? 0 : n - k]);
        if (okA) cA[k] = cscale(cadd(z, zc), half);
        if (okB) cB[k] = cscale(cmi(csub(z, zc)), half);
      }
    } else if (a.kind == TRIG_DCT1) {
      for (int k = lt; k < a.ncoef; k += TL) {
        if (okA) put_real_coef<T>(cA, k, buf[k].r);
        if (okB) put_real_coef<T>(cB, k, buf[k].i);
      }
    } else if (a.kind == TRIG_QWS) {
      // W = -2i S_a + 2 S_b; stored 4 S
      for (int k = lt; k < a.ncoef; k += TL) {
        const cpx<T> z = buf[k];
        if (okA) put_real_coef<T>(cA, k, T(-2) * z.i);
        if (okB) put_real_coef<T>(cB, k, T(2) * z.r);
      }
    } else if (a.kind == TRIG_QWC) {
      // W = 2 C_a + 2i C_b; stored 4 C
      for (int k = lt; k < a.ncoef; k += TL) {
        const cpx<T> z = buf[k];
        if (okA) put_real_coef<T>(cA, k, T(2) * z.r);
        if (okB) put_real_coef<T>(cB, k, T(2) * z.i);
      }
    } else {
      // Z = -i S_a + S_b: S_a = -Im Z, S_b = Re Z, modes 1..n-2 stored at m - 1
      for (int k = lt; k < a.ncoef; k += TL) {
        const cpx<T> z = buf[k + 1];
        if (okA) put_real_coef<T>(cA, k, -z.i);
        if (okB) put_real_coef<T>(cB, k, z.r);
      }
    }
    // an odd coefficient count leaves the last real slot of the packed row
    // unused: write zero, since the column transforms round the two slots of
    // a complex element together
    if (a.kind != TRIG_DFT && (a.ncoef & 1) && lt == 0) {
      if (okA) put_real_coef<T>(cA, a.ncoef, T(0));
      if (okB) put_real_coef<T>(cB, a.ncoef, T(0));
    }
    return;
  }
  for (int x = lt; x < n; x += TL) {
    double va, vb;
    if (a.kind == TRIG_DST1) {
      const bool wall = (x == 0 || x == n - 1);
      va = wall ? 0.0 : -(double)buf[x].i;
      vb = wall ? 0.0 : (double)buf[x].r;
    } else if (qw) {
      // R = exp(i pi x / 2N) IDFT: QWS R = 2i y_a - 2 y_b, QWC R = 2 y_a + 2i y_b
      const cpx<T> R = cmul(buf[x], cconj(qtw[x]));
      const bool wall = a.kind == TRIG_QWS ? x == 0 : x == n - 1;
      va = wall ? 0.0 : 0.5 * (a.kind == TRIG_QWS ? (double)R.i : (double)R.r);
      vb = wall ? 0.0 : 0.5 * (a.kind == TRIG_QWS ? -(double)R.r : (double)R.i);
    } else {
      va = (double)buf[x].r;
      vb = (double)buf[x].i;
    }
    const double pa = a.scale * va, pb = a.scale * vb;
    if (okA) a.out[(size_t)rA * n + x] = pa;
    if (okB) a.out[(size_t)rB * n + x] = pb;
    // (each position is read and rewritten by its own thread only)
    if (a.spec_out) buf[x] = to_cpx<T>(okA ? pa : 0.0, okB ? pb : 0.0);
  }
  if (!a.spec_out) return;
  // the projection gradient's x pass fused in: FC_x of the two rows just
  // stored (from LDS), packed R2C, half spectra of rows rA, rB
  __syncthreads();
  if (a.xfc.on)
    for (int j = n + lt; j < a.xE; j += TL) {
      const int i = fc_slot(a.xfc, n, a.xE, j);
      const double ra = (okA && i >= 0) ? fc_cont(a.xfc, n, i, [&](int q) { return (double)buf[q].r; }) : 0.0;
      const double rb = (okB && i >= 0) ? fc_cont(a.xfc, n, i, [&](int q) { return (double)buf[q].i; }) : 0.0;
      buf[j] = to_cpx<T>(ra, rb);
    }
  __syncthreads();
  line_dft<T>(buf, a.xplan, lt, TL, false, false);
  if (!okA) return;
  cpx<T> *so = static_cast<cpx<T> *>(a.spec_out);
  cpx<T> *oa = so + (size_t)rA * a.spec_pitch;
  cpx<T> *ob = okB ? so + (size_t)rB * a.spec_pitch : nullptr;
  const T hf = T(0.5);
  for (int k = lt; k < a.xH; k += TL) {
    const cpx<T> z = buf[k];
    const cpx<T> zc = cconj(buf[k == 0 ? 0 : a.xE - k]);
    oa[k] = cscale(cadd(z, zc), hf);
    if (ob) ob[k] = cscale(cmi(csub(z, zc)), hf);
  }
}

// ============================================================= PPE strided pass
// Symmetric extension of buf[0..n) to length L and transform.  Coefficients
// (is_values = false) or values (true) of the complex line end up in buf[0..n).
template <typename T, bool W, bool BIG>
__device__ __forceinline__ void ppe_line_transform(Line<T> buf, const PpeColsArgs &a, int lt, int TL,
                                                   bool is_values) {
  // extension / twiddle before, one transform, mode extraction after
  const int n = a.nline, L = a.plan.n;
  const bool qw = a.kind == TRIG_QWS || a.kind == TRIG_QWC;
  const bool qws = a.kind == TRIG_QWS;
  const cpx<T> *qtw = static_cast<const cpx<T> *>(a.qtw);
  if (qw && !is_values) {
    // values at 0..N: zero the Dirichlet wall, extend, pre-twiddle
    if (lt == 0) buf[qws ? 0 : n - 1] = {T(0), T(0)};
    const T sg = qws ? T(1) : T(-1);
    for (int j = n + lt; j < L; j += TL) buf[j] = cscale(buf[L - j], sg);
    __syncthreads();
    for (int j = lt; j < L; j += TL) buf[j] = cmul(buf[j], qtw[j]);
  } else if (qw) {
    // coefficients at 0..N-1: mirror to 2N-1-l
    const T sg = qws ? T(-1) : T(1);
    for (int j = n - 1 + lt; j < L; j += TL) buf[j] = cscale(buf[L - 1 - j], sg);
  } else if (a.kind == TRIG_DCT1 && !a.dcs) {
    for (int j = n + lt; j < L; j += TL) buf[j] = buf[L - j];
  } else if (a.kind == TRIG_DST1) {
    // odd extension: positions 0 and n-1 are zero, j > n-1 holds -buf[L-j]
    // (none at length N)
    if (lt == 0) {
      buf[0] = {T(0), T(0)};
      buf[n - 1] = {T(0), T(0)};
    }
    if (!a.dcs)
      for (int j = n + lt; j < L; j += TL) buf[j] = cscale(buf[L - j], T(-1));
  }
  __syncthreads();
  const bool half = (a.kind == TRIG_DCT1 || a.kind == TRIG_DST1) && a.dcs;
  cpx<T> z1 = {T(0), T(0)};
  if (half) z1 = trig1_pre<T>(buf, a.plan, a.dcs, a.kind == TRIG_DST1, lt, TL);
  const bool cj = (a.kind == TRIG_DFT || qw) && is_values;
  line_dft<T, BIG, W>(buf, a.plan, lt, TL, cj, cj);
  if (half) trig1_post<T>(buf, a.plan, z1, a.kind == TRIG_DST1, lt, TL);
  if (qw && !is_values) {
    // F = 2i W (QWS), 2 W (QWC); position N holds no mode
    for (int j = lt; j < n; j += TL) {
      const cpx<T> w = buf[j];
      buf[j] = j == n - 1 ? cpx<T>{T(0), T(0)} : (qws ? cscale(cpi(w), T(2)) : cscale(w, T(2)));
    }
    __syncthreads();
  } else if (qw) {
    // y = -(i/2) R (QWS), R / 2 (QWC), R = exp(i pi j / 2N) IDFT; wall value 0
    for (int j = lt; j < n; j += TL) {
      const cpx<T> R = cmul(buf[j], cconj(qtw[j]));
      const bool wall = qws ? j == 0 : j == n - 1;
      buf[j] = wall ? cpx<T>{T(0), T(0)} : (qws ? cscale(cmi(R), T(0.5)) : cscale(R, T(0.5)));
    }
    __syncthreads();
  } else if (a.kind == TRIG_DST1) {
    // the DST-I of the complex line is i Z; wall values are zero (each
    // position written by the thread that owns it)
    for (int j = lt; j < n; j += TL)
      buf[j] = (is_values && (j == 0 || j == n - 1)) ? cpx<T>{T(0), T(0)} : cpi(buf[j]);
    __syncthreads();
  }
}

template <typename T, bool G, bool W>
__global__ void __launch_bounds__(kMaxThreads) k_ppe_cols(KArg<PpeColsArgs, G> ka) {
  const PpeColsArgs &a = ka.get();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *smem = reinterpret_cast<cpx<T> *>(smem_raw);
  const int TL = a.plan.TL;
  const int g = threadIdx.x / TL;
  const int lt = threadIdx.x - g * TL;
  Line<T> buf{smem + (size_t)g * a.ldsM};
  const int npanel = (a.ninner + a.B - 1) / a.B;
  const int bid = xcd_panel(blockIdx.x, gridDim.x);
  const int o = bid / npanel;
  const int c0 = (bid - o * npanel) * a.B;
  const int c = c0 + g;
  cpx<T> *data = static_cast<cpx<T> *>(a.data) + (size_t)o * a.os;
  const int n = a.nline;

  if (a.B == 1) {
    // one column pair per workgroup (the default): no division by the panel width
    const bool ok = c0 < a.ninner;
    batched<8, cpx<T>>(threadIdx.x, n, blockDim.x,
                       [&](int j) { return ok ? data[(size_t)j * a.es + c0] : cpx<T>{T(0), T(0)}; },
                       [&](int j, cpx<T> v) { Line<T>{smem}[j] = v; });
  } else {
    batched<8, cpx<T>>(threadIdx.x, a.B * n, blockDim.x,
                       [&](int idx) {
                         const int l = idx % a.B, j = idx / a.B;
                         const int cc = c0 + l;
                         return cc < a.ninner ? data[(size_t)j * a.es + cc] : cpx<T>{T(0), T(0)};
                       },
                       [&](int idx, cpx<T> v) {
                         const int l = idx % a.B, j = idx / a.B;
                         Line<T>{smem + (size_t)l * a.ldsM}[j] = v;
                       });
  }
  __syncthreads();
  // solve == 0: forward only; 1: forward, divide, inverse; 2: inverse only
  const int npass = a.solve == 1 ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const bool values = a.solve == 2 || pass == 1;
    ppe_line_transform<T, W, !G>(buf, a, lt, TL, values);
    if (a.solve == 1 && pass == 0) {
      // divide by -(mu_inner + mu_line + mu_outer) in FP64; a vanishing sum
      // (the constant mode) gives zero
      const double mo = a.mu_outer ? a.mu_outer[o] : 0.0;
      double mir = 0.0, mii = 0.0;
      if (c < a.ninner) {
        if (a.inner_packed) {
          mir = a.mu_inner[2 * c];
          mii = (2 * c + 1 < a.inner_nmodes) ? a.mu_inner[2 * c + 1] : 1.0;
        } else {
          mir = mii = a.mu_inner[c];
        }
      }
      if (a.sph) {
        // SPH family: mu = sum_a sigma_a^2 at (inner, line) wavenumbers
        double2 Rx[kSymW], Ry[kSymW];
        const int ci = c < a.ninner ? c : 0;
#pragma unroll
        for (int q = 0; q < kSymW; ++q) {
          Rx[q] = a.symR[((size_t)SYM_GX * a.sym_ninner + ci) * kSymW + q];
          Ry[q] = a.symR[((size_t)SYM_GY * a.sym_ninner + ci) * kSymW + q];
        }
        for (int k = lt; k < n; k += TL) {
          const double sx = a.sph_norm * sym_eval(Rx, a.ph_line, k).y;
          const double sy = a.sph_norm * sym_eval(Ry, a.ph_line, k).y;
          const double mu = sx * sx + sy * sy;
          const cpx<T> v = buf[k];
          const bool ok = mu > a.mu_tol;
          const double vr = ok ? -(double)v.r / mu : 0.0;
          const double vi = ok ? -(double)v.i / mu : 0.0;
          buf[k] = to_cpx<T>(vr * a.scale, vi * a.scale);
        }
      } else {
        for (int k = lt; k < n; k += TL) {
          const bool valid = a.kind == TRIG_DST1 ? (k >= 1 && k <= n - 2)
                             : (a.kind == TRIG_QWS || a.kind == TRIG_QWC) ? k < n - 1 : true;
          const double ml = valid ? a.mu_line[k] + mo : 0.0;
          const double sr = mir + ml, si = mii + ml;
          const cpx<T> v = buf[k];
          const double vr = (valid && sr != 0.0) ? -(double)v.r / sr : 0.0;
          const double vi = (valid && si != 0.0) ? -(double)v.i / si : 0.0;
          buf[k] = to_cpx<T>(vr * a.scale, vi * a.scale);
        }
      }
      __syncthreads();
    }
  }
  if (a.B == 1) {
    if (c0 < a.ninner)
      for (int j = threadIdx.x; j < n; j += blockDim.x) data[(size_t)j * a.es + c0] = Line<T>{smem}[j];
    return;
  }
  for (int idx = threadIdx.x; idx < a.B * n; idx += blockDim.x) {
    const int l = idx % a.B, j = idx / a.B;
    const int cc = c0 + l;
    if (cc < a.ninner) data[(size_t)j * a.es + cc] = Line<T>{smem + (size_t)l * a.ldsM}[j];
  }
}

// ============================================================= FC standalone
// Array viewed as [outer][len][inner]; output [outer][len + C][inner].
__global__ void k_fc_extend(const double *in, double *out, long outer, int len, long inner,
                            FcWalls fc) {
  const long Lo = len + fc.C;
  const long total = outer * Lo * inner;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long c = idx % inner;
    const long j = (idx / inner) % Lo;
    const long o = idx / (inner * Lo);
    const double *line = in + o * len * inner + c;
    double v;
    if (j < len) {
      v = line[j * inner];
    } else {
      v = fc_cont(fc, len, (int)(j - len), [&](int jj) { return line[(long)jj * inner]; });
    }
    out[idx] = v;
  }
}

// ============================================================= finiteness check
// counter[0] <- 0 (a kernel, not a memset: safe under graph capture), then
// counter[0] += the number of NaN / infinite values of x[0..n).
__global__ void k_zero_counter(unsigned long long *counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) counter[0] = 0ull;
}

__global__ void __launch_bounds__(256) k_count_nonfinite(const double *x, size_t n, unsigned long long *counter) {
  unsigned int c = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    c += isfinite(x[i]) ? 0u : 1u;
  // wave reduction, one atomic per wave
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_down(c, d, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(counter, (unsigned long long)c);
}

hipError_t launch_count_nonfinite(const double *x, size_t n, unsigned long long *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  size_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)nb), dim3(256), 0, s, x, n, counter);
  return hipGetLastError();
}

// ============================================================= launchers
Recorder *&active_recorder() {
  static thread_local Recorder *r = nullptr;
  return r;
}

static size_t lds_bytes(int B, int ldsM, bool fp32) {
  return (size_t)B * ldsM * (fp32 ? sizeof(cpx<float>) : sizeof(cpx<double>));
}

hipError_t launch_rows_fwd(const RowsFwdArgs &a, bool fp32, hipStream_t s) {
  const dim3 grid((a.nlines + a.B - 1) / a.B), block(a.B * a.plan.TL);
  // the fused FP64 boundary-row pass of FP32 kernels lays FP64 lines over the FP32 ones
  const bool edge = fp32 && a.edge_rows > 0;
  if (edge && (a.plan64.TL != a.plan.TL || a.plan64.M != a.plan.M || a.map_per != 0 || !a.edgeA ||
               (a.inB && !a.edgeB)))
    return hipErrorInvalidValue;
  const size_t lds = lds_bytes(a.B, a.ldsM, fp32 && !edge);
  if (fp32) return issue(k_rows_fwd<float, false>, k_rows_fwd<float, true>, a, grid, block, lds, s);
  return issue(k_rows_fwd<double, false>, k_rows_fwd<double, true>, a, grid, block, lds, s);
}

template <typename T, int EPI>
static hipError_t rows_inv_t(const RowsInvArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  return issue(k_rows_inv<T, EPI, false>, k_rows_inv<T, EPI, true>, a, grid, block, lds, s);
}

template <typename T>
static hipError_t rows_inv_dispatch(const RowsInvArgs &a, int epi, hipStream_t s) {
  const int TL = a.plan.TL;
  dim3 grid, block;
  size_t lds;
  switch (epi) {
    case EPI_STORE: {
      const bool pair = a.spec[1] != nullptr;
      const int nl = pair ? a.nrows : (a.nrows + 1) / 2;
      grid = dim3((nl + a.B - 1) / a.B);
      block = dim3(a.B * TL);
      lds = lds_bytes(a.B, a.ldsM, sizeof(T) == 4);
      return rows_inv_t<T, EPI_STORE>(a, grid, block, lds, s);
    }
    case EPI_STEP_D2:
      grid = dim3((a.nrows + a.B - 1) / a.B);
      block = dim3(a.B * TL);
      lds = lds_bytes(a.B, a.ldsM, sizeof(T) == 4);
      return rows_inv_t<T, EPI_STEP_D2>(a, grid, block, lds, s);
    case EPI_ADVECT2:
      grid = dim3((a.nrows + a.B - 1) / a.B);
      block = dim3(a.B * TL);
      lds = lds_bytes(a.B, a.ldsM, sizeof(T) == 4);
      return rows_inv_t<T, EPI_ADVECT2>(a, grid, block, lds, s);
    case EPI_STEP_A2:
      // one line group, one FP64 line (the FP32 line and, in FP32 kernels,
      // the fused FP64 forward pass's line) and two real arrays of the row
      if (a.fwd_fused && sizeof(T) == 4 && (a.plan64.TL != TL || a.plan64.M != a.plan.M)) return hipErrorInvalidValue;
      grid = dim3(a.nrows);
      block = dim3(TL);
      lds = lds_bytes(1, a.ldsM, false) + 2 * (size_t)a.nx * sizeof(double);
      if (lds > (size_t)kMaxLds) return hipErrorInvalidValue;
      return rows_inv_t<T, EPI_STEP_A2>(a, grid, block, lds, s);
    case EPI_STEP_A3S:
      // one line group, one line and three real arrays of the row; rows of at
      // most 4 TL points
      if (a.nx > 4 * TL) return hipErrorInvalidValue;
      grid = dim3(a.nrows);
      block = dim3(TL);
      lds = lds_bytes(1, a.ldsM, sizeof(T) == 4) + 3 * (size_t)a.nx * sizeof(double);
      if (lds > (size_t)kMaxLds) return hipErrorInvalidValue;
      return rows_inv_t<T, EPI_STEP_A3S>(a, grid, block, lds, s);
    case EPI_STEP_A3:
    case EPI_STEP_D3: {
      const int NL = epi == EPI_STEP_A3 ? 6 : 2;
      // step D (two lines): one line group taking them in turn (one-wave
      // workgroups, twice as many rows resident as with a group per line)
      const int G = epi == EPI_STEP_D3 ? 1 : std::max(1, std::min(NL, kMaxThreads / TL));
      grid = dim3(a.nrows);
      block = dim3(G * TL);
      lds = lds_bytes(NL, a.ldsM, sizeof(T) == 4);
      if (lds > (size_t)kMaxLds) return hipErrorInvalidValue;
      if (epi == EPI_STEP_A3) return rows_inv_t<T, EPI_STEP_A3>(a, grid, block, lds, s);
      return rows_inv_t<T, EPI_STEP_D3>(a, grid, block, lds, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rows_inv(const RowsInvArgs &a, int epi, bool fp32, hipStream_t s) {
  return fp32 ? rows_inv_dispatch<float>(a, epi, s) : rows_inv_dispatch<double>(a, epi, s);
}

template <typename T, int MODE>
static hipError_t cols_t(const ColsArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  constexpr bool SYM = MODE == COLS_OP || MODE == COLS_DIV || MODE == COLS_PROJ;
  if constexpr (SYM) {
    if (a.symF) return issue(k_cols<T, MODE, false, true>, k_cols<T, MODE, true, true>, a, grid, block, lds, s);
  }
  return issue(k_cols<T, MODE, false>, k_cols<T, MODE, true>, a, grid, block, lds, s);
}

template <typename T>
static hipError_t cols_dispatch(const ColsArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  switch (a.mode) {
    case COLS_FWD: return cols_t<T, COLS_FWD>(a, grid, block, lds, s);
    case COLS_INV: return cols_t<T, COLS_INV>(a, grid, block, lds, s);
    case COLS_OP: return cols_t<T, COLS_OP>(a, grid, block, lds, s);
    case COLS_DIV: return cols_t<T, COLS_DIV>(a, grid, block, lds, s);
    case COLS_PROJ: return cols_t<T, COLS_PROJ>(a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

// Workgroups of the one-problem COLS_OP kernel resident on the whole device
// at once (0 if unknown).  Cached per host thread for the last shape asked.
template <typename T>
static int cols_op_slots(int block, size_t lds) {
  struct Entry {
    int dev = -1, block = 0, slots = 0;
    size_t lds = 0;
  };
  thread_local Entry e;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (e.dev == dev && e.block == block && e.lds == lds) return e.slots;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (set_kernel_lds(k_cols<T, COLS_OP, false>, lds) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cols<T, COLS_OP, false>, block, lds) !=
      hipSuccess)
    return 0;
  e = Entry{dev, block, per * cus, lds};
  return e.slots;
}

hipError_t launch_cols(const ColsArgs &a, int ngrid_y, bool fp32, hipStream_t s) {
  const int npanel = (a.ninner + a.B - 1) / a.B;
  const dim3 grid(npanel * a.nouter, ngrid_y), block(a.B * a.plan.TL);
  const size_t lds = lds_bytes(a.B * cols_lines_per_column(a.mode, a.st.ndim), a.ldsM, fp32);
  if (lds > (size_t)kMaxLds) return hipErrorInvalidValue;
  if (a.mode == COLS_PROJ && (a.B != 1 || (!a.symR && !a.symF))) return hipErrorInvalidValue;
  // the symbol passes read their line coefficients from the plan's table
  if ((a.mode == COLS_OP || a.mode == COLS_DIV) && !a.symR && !a.symF) return hipErrorInvalidValue;
  if (a.nfull != 0) return hipErrorInvalidValue;
  // the inverse pass conjugates on load: it must load every line position
  if (a.mode == COLS_INV && a.nload != a.plan.n) return hipErrorInvalidValue;
  // Tail split: when the tasks (field, panel) exceed the resident workgroups
  // by at most a third of them divided by the outputs, the leftover tasks
  // would run as a second, nearly empty round of whole tasks (forward + nout
  // inverse transforms).  Their outputs go to separate workgroups instead
  // (forward + one inverse each), which fill one round after the first.
  // The 1024^2 stage-A pass has 1122 tasks for 1024 resident workgroups.
  if (a.mode == COLS_OP && a.nout > 1 && !active_recorder() && !a.symF) {
    const long tasks = (long)grid.x * ngrid_y;
    const int slots = fp32 ? cols_op_slots<float>(block.x, lds) : cols_op_slots<double>(block.x, lds);
    const long rest = tasks - slots;
    if (slots > 0 && rest > 0 && rest * a.nout <= slots) {
      ColsArgs b = a;
      b.nfull = slots;
      const dim3 g2((unsigned)(slots + rest * a.nout), 1);
      return fp32 ? cols_dispatch<float>(b, g2, block, lds, s) : cols_dispatch<double>(b, g2, block, lds, s);
    }
  }
  return fp32 ? cols_dispatch<float>(a, grid, block, lds, s) : cols_dispatch<double>(a, grid, block, lds, s);
}

hipError_t launch_ppe_rows(const PpeRowsArgs &a, bool fp32, hipStream_t s) {
  const int nl = (a.nrows + 1) / 2;
  const dim3 grid((nl + a.B - 1) / a.B), block(a.B * a.plan.TL);
  const size_t lds = lds_bytes(a.B, a.ldsM, fp32);
  // plans whose lines do not fit the narrow butterfly rule run the wide kernels
  if (a.plan.wide) {
    if (fp32) return issue(k_ppe_rows<float, false, true>, k_ppe_rows<float, true, true>, a, grid, block, lds, s);
    return issue(k_ppe_rows<double, false, true>, k_ppe_rows<double, true, true>, a, grid, block, lds, s);
  }
  if (fp32) return issue(k_ppe_rows<float, false, false>, k_ppe_rows<float, true, false>, a, grid, block, lds, s);
  return issue(k_ppe_rows<double, false, false>, k_ppe_rows<double, true, false>, a, grid, block, lds, s);
}

hipError_t launch_ppe_cols(const PpeColsArgs &a, bool fp32, hipStream_t s) {
  const int npanel = (a.ninner + a.B - 1) / a.B;
  const dim3 grid(npanel * a.nouter), block(a.B * a.plan.TL);
  const size_t lds = lds_bytes(a.B, a.ldsM, fp32);
  if (a.plan.wide) {
    if (fp32) return issue(k_ppe_cols<float, false, true>, k_ppe_cols<float, true, true>, a, grid, block, lds, s);
    return issue(k_ppe_cols<double, false, true>, k_ppe_cols<double, true, true>, a, grid, block, lds, s);
  }
  if (fp32) return issue(k_ppe_cols<float, false, false>, k_ppe_cols<float, true, false>, a, grid, block, lds, s);
  return issue(k_ppe_cols<double, false, false>, k_ppe_cols<double, true, false>, a, grid, block, lds, s);
}

hipError_t launch_fc_extend_axis(const double *in, double *out, int ndim, const int *shape_in,
                                 int axis, const FcWalls &fc, hipStream_t s) {
  // shape_in in lattice order (x, y, z); axis in lattice order
  long inner = 1, outer = 1;
  for (int a = 0; a < axis; ++a) inner *= shape_in[a];
  for (int a = axis + 1; a < ndim; ++a) outer *= shape_in[a];
  const int len = shape_in[axis];
  const long total = outer * (long)(len + fc.C) * inner;
  const int block = 256;
  long nblk = (total + block - 1) / block;
  if (nblk > 65535L * 16) nblk = 65535L * 16;
  hipLaunchKernelGGL(k_fc_extend, dim3((unsigned)nblk), dim3(block), 0, s, in, out, outer, len,
                     inner, fc);
  return hipGetLastError();
}

}  // namespace fcsph
