// Device-side line FFT engine for gfx950: mixed-radix Stockham stages on a
// line buffer in LDS, executed cooperatively by a group of TL threads, plus a
// Bluestein (chirp-z) wrapper for lengths with large prime factors.
//
// Stockham stage with radix R on length N, after stages whose radices
// multiply to Ns: butterfly j (0 <= j < N/R) reads x[j + r N/R], applies the
// twiddles w^(r k) with k = j mod Ns and w = exp(-2 pi i / (Ns R)), takes the
// length-R DFT, and writes to (j - k) R + k + r Ns.  Output is in natural
// order after the last stage.  Each thread keeps its butterflies of the stage
// in registers between the read and write phases, so a single LDS buffer per
// line suffices (read phase, barrier, write phase, barrier).
//
// Every line group of a workgroup runs the same plan, so the barriers are
// uniform across the workgroup.
#pragma once
#include "internal.h"

namespace fcsph {

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.r, -a.i}; }
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.r * s, a.i * s}; }
// multiply by -i and +i
template <typename T>
__device__ __forceinline__ cpx<T> cmi(cpx<T> a) { return {a.i, -a.r}; }
template <typename T>
__device__ __forceinline__ cpx<T> cpi(cpx<T> a) { return {-a.i, a.r}; }

// Strided loop that keeps up to U loads in flight: ld(i) for U indices, then
// use(i, value) for them.  A plain loop that stores each loaded value to LDS
// waits for every load in turn.
template <int U, typename V, typename Ld, typename Use>
__device__ __forceinline__ void batched(int start, int end, int step, Ld ld, Use use) {
  for (int base = start; base < end; base += U * step) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * step;
      if (i < end) v[u] = ld(i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * step;
      if (i < end) use(i, v[u]);
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8).  Remapping b so that every XCD receives a contiguous range of
// panels makes neighbouring panels - which share cache lines - meet in the
// same L2.  The map is a bijection of [0, nb).
__device__ __forceinline__ int xcd_panel(int b, int nb) {
  constexpr int NX = 8;
  const int per = nb / NX, rem = nb % NX;
  const int x = b % NX, k = b / NX;
  return x * per + (x < rem ? x : rem) + k;
}

// ---- radix-R DFTs (forward, exp(-2 pi i j k / R)) on a register array ----
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
  __device__ __forceinline__ static void run(cpx<T> *x, const cpx<T> *, int) {
    cpx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <typename T>
struct Dft<T, 3> {
  __device__ __forceinline__ static void run(cpx<T> *x, const cpx<T> *, int) {
    const T c = T(-0.5);
    const T s = T(0.86602540378443864676372317075294);   // sin(2 pi / 3)
    cpx<T> t = cadd(x[1], x[2]);
    cpx<T> m = {x[0].r + c * t.r, x[0].i + c * t.i};
    cpx<T> d = csub(x[1], x[2]);
    cpx<T> sd = {s * d.r, s * d.i};
    x[0] = cadd(x[0], t);
    x[1] = cadd(m, cmi(sd));
    x[2] = cadd(m, cpi(sd));
  }
};

template <typename T>
struct Dft<T, 4> {
  __device__ __forceinline__ static void run(cpx<T> *x, const cpx<T> *, int) {
    cpx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cpx<T> b0 = cadd(x[1], x[3]), b1 = cmi(csub(x[1], x[3]));
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  }
};

template <typename T>
struct Dft<T, 8> {
  __device__ __forceinline__ static void run(cpx<T> *x, const cpx<T> *, int) {
    const T h = T(0.70710678118654752440084436210485);
    cpx<T> a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = cadd(x[j], x[j + 4]);
      b[j] = csub(x[j], x[j + 4]);
    }
    // b_j *= exp(-2 pi i j / 8)
    b[1] = {h * (b[1].r + b[1].i), h * (b[1].i - b[1].r)};
    b[2] = cmi(b[2]);
    b[3] = {h * (b[3].i - b[3].r), -h * (b[3].r + b[3].i)};
    Dft<T, 4>::run(a, nullptr, 0);
    Dft<T, 4>::run(b, nullptr, 0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      x[2 * m] = a[m];
      x[2 * m + 1] = b[m];
    }
  }
};

// Odd radix, computed in place and stored as it goes:
//   X_k     = x0 + sum_{j=1..h} (x_j + x_{R-j}) cos(2 pi j k/R) - i sum_j (x_j - x_{R-j}) sin(2 pi j k/R)
//   X_{R-k} = the same with +i,   X_0 = sum_j x_j.
// x[j] is overwritten by x_j + x_{R-j} and x[R-j] by x_j - x_{R-j}; each pair
// of outputs is handed to put(r, value) as soon as it is formed, so the
// registers hold the R inputs and two accumulators only.  cs_sn(m, c, s)
// gives cos / sin(2 pi m / R).
template <typename T, int R, typename CS, typename Put>
__device__ __forceinline__ void dft_odd_store(cpx<T> *x, CS cs_sn, Put put) {
  constexpr int h = (R - 1) / 2;
#pragma unroll
  for (int j = 1; j <= h; ++j) {
    const cpx<T> a = x[j], b = x[R - j];
    x[j] = cadd(a, b);
    x[R - j] = csub(a, b);
  }
  const cpx<T> x0 = x[0];
  cpx<T> tot = x0;
#pragma unroll
  for (int j = 1; j <= h; ++j) tot = cadd(tot, x[j]);
  put(0, tot);
#pragma unroll
  for (int k = 1; k <= h; ++k) {
    cpx<T> A = x0, Bv = {T(0), T(0)};
#pragma unroll
    for (int j = 1; j <= h; ++j) {
      const int m = (j * k) % R;
      T c, sn;
      cs_sn(m, c, sn);
      A.r += x[j].r * c;
      A.i += x[j].i * c;
      Bv.r += x[R - j].r * sn;
      Bv.i += x[R - j].i * sn;
    }
    put(k, cadd(A, cmi(Bv)));
    put(R - k, cadd(A, cpi(Bv)));
  }
}

template <typename T>
struct Dft<T, 5> {
  template <typename Put>
  __device__ __forceinline__ static void run_store(cpx<T> *x, const cpx<T> *, int, Put put) {
    dft_odd_store<T, 5>(x, [](int m, T &c, T &s) {
      constexpr double C1 = 0.30901699437494742410229341718282, C2 = -0.80901699437494742410229341718282;
      constexpr double S1 = 0.95105651629515357211643933337938, S2 = 0.58778525229247312916870595463907;
      c = T(m == 1 || m == 4 ? C1 : C2);
      s = T(m == 1 ? S1 : m == 2 ? S2 : m == 3 ? -S2 : -S1);
    }, put);
  }
};

template <typename T>
struct Dft<T, 7> {
  template <typename Put>
  __device__ __forceinline__ static void run_store(cpx<T> *x, const cpx<T> *, int, Put put) {
    dft_odd_store<T, 7>(x, [](int m, T &c, T &s) {
      constexpr double C1 = 0.62348980185873353052500488400424, C2 = -0.22252093395631440428890256449679,
                       C3 = -0.90096886790241912623610231950745;
      constexpr double S1 = 0.78183148246802980870844452667406, S2 = 0.97492791218182360701813168299393,
                       S3 = 0.43388373911755812047576833284836;
      const int mm = m <= 3 ? m : 7 - m;
      const double sg = m <= 3 ? 1.0 : -1.0;
      c = T(mm == 1 ? C1 : mm == 2 ? C2 : C3);
      s = T(sg * (mm == 1 ? S1 : mm == 2 ? S2 : S3));
    }, put);
  }
};

// Larger odd radices read cos / sin(2 pi m / R) from the line's root table:
// tw[m N / R] = exp(-2 pi i m / R).
template <typename T, int R>
struct Dft {
  template <typename Put>
  __device__ __forceinline__ static void run_store(cpx<T> *x, const cpx<T> *tw, int base, Put put) {
    dft_odd_store<T, R>(x, [&](int m, T &c, T &s) {
      const cpx<T> w = tw[m * base];
      c = w.r;
      s = -w.i;
    }, put);
  }
};

// j mod Ns for 0 <= j < 2^13, 1 <= Ns <= 2^13 (line work lengths stay below
// 8192): a float quotient with rns = 1 / Ns is off by at most one and one
// correction step in each direction makes it exact (checked for every pair
// in range).  Full-rate float and 24-bit integer operations instead of the
// runtime integer division (quarter-rate 32-bit multiplies).
__device__ __forceinline__ int mod_small(int j, int Ns, float rns) {
  const int q = (int)((float)j * rns);
  int k = j - __mul24(q, Ns);
  k = k >= Ns ? k - Ns : k;
  k = k < 0 ? k + Ns : k;
  return k;
}

// Radices 2, 4 and 8 compute in registers and then store.
template <typename T, int R>
__device__ __forceinline__ constexpr bool is_pow2_radix() { return R == 2 || R == 3 || R == 4 || R == 8; }

// One Stockham stage.  N: work length; Ns: product of previous radices.
template <typename T, int R, bool WIDE = false>
__device__ __forceinline__ void stockham_stage(Line<T> buf, int N, int Ns, const cpx<T> *tw,
                                               int lt, int TL, bool active) {
  constexpr int NB = nb_max(R, WIDE);
  const int NR = N / R;
  const int tstride = N / (Ns * R);
  const float rns = 1.0f / (float)Ns;
  cpx<T> v[NB][R];
  cpx<T> w1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lt + b * TL;
    if (active && j < NR) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[j + __mul24(r, NR)];
      // radix <= 8: one twiddle per butterfly, loaded before the barrier (its
      // latency hides behind the barrier), its powers formed by products of
      // depth <= 3; larger radices load each twiddle
      if constexpr (R <= 8) w1[b] = tw[__mul24(mod_small(j, Ns, rns), tstride)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lt + b * TL;
    if (active && j < NR) {
      const int k = mod_small(j, Ns, rns);
      if (k != 0) {
        if constexpr (R <= 4) {
          cpx<T> t = w1[b];
          v[b][1] = cmul(v[b][1], t);
#pragma unroll
          for (int r = 2; r < R; ++r) {
            t = cmul(t, w1[b]);
            v[b][r] = cmul(v[b][r], t);
          }
        } else if constexpr (R <= 8) {
          // w^2 = w w, w^3 = w^2 w, w^4 = w^2 w^2, w^{4+q} = w^4 w^q
          const cpx<T> t1 = w1[b];
          const cpx<T> t2 = cmul(t1, t1);
          const cpx<T> t3 = cmul(t2, t1);
          const cpx<T> t4 = cmul(t2, t2);
          v[b][1] = cmul(v[b][1], t1);
          v[b][2] = cmul(v[b][2], t2);
          v[b][3] = cmul(v[b][3], t3);
          v[b][4] = cmul(v[b][4], t4);
          if constexpr (R > 5) v[b][5] = cmul(v[b][5], cmul(t4, t1));
          if constexpr (R > 6) v[b][6] = cmul(v[b][6], cmul(t4, t2));
          if constexpr (R > 7) v[b][7] = cmul(v[b][7], cmul(t4, t3));
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[r * k * tstride]);
        }
      }
      const int o = __mul24(j - k, R) + k;
      if constexpr (is_pow2_radix<T, R>()) {
        Dft<T, R>::run(v[b], tw, NR);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[o + __mul24(r, Ns)] = v[b][r];
      } else {
        Dft<T, R>::run_store(v[b], tw, NR, [&](int r, cpx<T> val) { buf[o + __mul24(r, Ns)] = val; });
      }
    }
  }
  __syncthreads();
}

// Forward FFT of length N = prod(radix) in place on buf (natural order).
// BIG enables the odd radices 11..31 (held whole in registers); no kernel
// instantiates it at present, which keeps every kernel's register budget at
// that of radices <= 8.
template <typename T, bool BIG = false, bool WIDE = false>
__device__ __forceinline__ void fft_stockham(Line<T> buf, const LinePlan &p, int N, int lt, int TL,
                                             bool active) {
  const cpx<T> *tw = static_cast<const cpx<T> *>(p.tw);
  int Ns = 1;
  for (int s = 0; s < p.nstages; ++s) {
    const int R = p.radix[s];
    switch (R) {
      case 2: stockham_stage<T, 2, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
      case 3: stockham_stage<T, 3, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
      case 4: stockham_stage<T, 4, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
      case 5: stockham_stage<T, 5, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
      case 7: stockham_stage<T, 7, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
      case 8: stockham_stage<T, 8, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
      default:
        if constexpr (BIG) {
          switch (R) {
            case 11: stockham_stage<T, 11, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            case 13: stockham_stage<T, 13, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            case 17: stockham_stage<T, 17, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            case 19: stockham_stage<T, 19, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            case 23: stockham_stage<T, 23, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            case 29: stockham_stage<T, 29, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            case 31: stockham_stage<T, 31, WIDE>(buf, N, Ns, tw, lt, TL, active); break;
            default: break;
          }
        }
        break;   // the host never builds other radices
    }
    Ns *= R;
  }
}

// Forward DFT of length p.n on buf[0..n) (in place, result in buf[0..n)).
// conj_in / conj_out conjugate the input / output, which turns the forward
// transform into the unnormalised inverse.  Ends with a barrier.  An inactive
// line group touches no memory but executes the same barriers.
template <typename T, bool BIG = false, bool WIDE = false>
__device__ __forceinline__ void line_dft(Line<T> buf, const LinePlan &p, int lt, int TL, bool conj_in,
                                         bool conj_out, bool active = true) {
  if (!active) {
    lt = 1 << 30;           // every index loop below starts past its bound
  }
  // one Stockham call site (two passes for Bluestein) keeps the inlined code
  // and its registers at those of a single transform
  const int len = p.blue ? p.M : p.n;
  const cpx<T> *chirp = static_cast<const cpx<T> *>(p.chirp);
  const cpx<T> *filt = static_cast<const cpx<T> *>(p.filt);
  if (!p.blue) {
    if (conj_in) {
      for (int j = lt; j < p.n; j += TL) buf[j].i = -buf[j].i;
      __syncthreads();
    }
  } else {
    // a_j = x_j w_j (zero padded to M)
    for (int j = lt; j < p.M; j += TL) {
      cpx<T> v = {T(0), T(0)};
      if (j < p.n) {
        v = buf[j];
        if (conj_in) v.i = -v.i;
        v = cmul(v, chirp[j]);
      }
      buf[j] = v;
    }
    __syncthreads();
  }
  const int npass = p.blue ? 2 : 1;
#pragma unroll 1
  for (int pass = 0; pass < npass; ++pass) {
    fft_stockham<T, BIG, WIDE>(buf, p, len, lt, TL, active);
    if (pass == 0 && p.blue) {
      // pointwise product with the filter spectrum; conjugate for the inverse FFT
      for (int j = lt; j < p.M; j += TL) buf[j] = cconj(cmul(buf[j], filt[j]));
      __syncthreads();
    }
  }
  if (!p.blue) {
    if (conj_out) {
      for (int j = lt; j < p.n; j += TL) buf[j].i = -buf[j].i;
      __syncthreads();
    }
  } else {
    for (int k = lt; k < p.n; k += TL) {
      cpx<T> v = cmul(cconj(buf[k]), chirp[k]);
      if (conj_out) v.i = -v.i;
      buf[k] = v;
    }
    __syncthreads();
  }
}

}  // namespace fcsph
