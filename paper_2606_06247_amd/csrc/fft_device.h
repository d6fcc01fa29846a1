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

// Larger odd radices: cos / sin(2 pi m / R), m = 1 .. (R - 1) / 2, as
// literals (40-digit values rounded to double), the source of the streamed
// stages' root tables.
template <int R>
struct OddRoots;
template <> struct OddRoots<11> {
  static constexpr double c[5] = {8.41253532831181168862e-1, 4.15415013001886425529e-1, -1.42314838273285140444e-1, -6.54860733945285064057e-1, -9.5949297361449738989e-1};
  static constexpr double s[5] = {5.40640817455597582108e-1, 9.09631995354518371412e-1, 9.89821441880932732376e-1, 7.55749574354258283774e-1, 2.81732556841429697711e-1};
};
template <> struct OddRoots<13> {
  static constexpr double c[6] = {8.854560256532098959e-1, 5.68064746731155802512e-1, 1.20536680255323053349e-1, -3.5460488704253562597e-1, -7.48510748171101098635e-1, -9.70941817426052027157e-1};
  static constexpr double s[6] = {4.64723172043768545656e-1, 8.2298386589365639458e-1, 9.92708874098053992801e-1, 9.3501624268541482344e-1, 6.63122658240795202377e-1, 2.39315664287557767149e-1};
};
template <> struct OddRoots<17> {
  static constexpr double c[8] = {9.32472229404355804573e-1, 7.39008917220659115925e-1, 4.45738355776538267396e-1, 9.22683594633019952397e-2, -2.73662990072082863539e-1, -6.02634636379256389179e-1, -8.50217135729614152134e-1, -9.82973099683901778282e-1};
  static constexpr double s[8] = {3.61241666187152948745e-1, 6.73695643646557211713e-1, 8.95163291355062322067e-1, 9.95734176295034521871e-1, 9.61825643172819070409e-1, 7.98017227280239503333e-1, 5.26432162877355800245e-1, 1.83749517816570331574e-1};
};
template <> struct OddRoots<19> {
  static constexpr double c[9] = {9.4581724170063467902e-1, 7.89140509396393599219e-1, 5.46948158122426874712e-1, 2.45485487140799148922e-1, -8.25793454723323246003e-2, -4.01695424652969457517e-1, -6.77281571625741074762e-1, -8.79473751206489071391e-1, -9.86361303402722373603e-1};
  static constexpr double s[9] = {3.24699469204683487408e-1, 6.14212712689667817444e-1, 8.37166478262528574806e-1, 9.69400265939330416736e-1, 9.96584493006669849819e-1, 9.15773326655057439919e-1, 7.35723910673131624774e-1, 4.75947393037073544431e-1, 1.64594590280733894144e-1};
};
template <> struct OddRoots<23> {
  static constexpr double c[11] = {9.62917287347799295015e-1, 8.54419404546488552548e-1, 6.82553143218654082875e-1, 4.60065037731152126042e-1, 2.03456013052633789878e-1, -6.82424133646709759212e-2, -3.34879612170986151958e-1, -5.76680322114867141251e-1, -7.75711290704419807041e-1, -9.17211301505453017844e-1, -9.90685946036330752342e-1};
  static constexpr double s[11] = {2.69796771157024271245e-1, 5.19583950035433578133e-1, 7.30835964278124101651e-1, 8.87885218402375234984e-1, 9.79084087682322875633e-1, 9.97668769190539198454e-1, 9.42260922118820495618e-1, 8.16969893010442016973e-1, 6.31087944326052789367e-1, 3.98401089846241457998e-1, 1.36166649096246590761e-1};
};
template <> struct OddRoots<29> {
  static constexpr double c[14] = {9.76620555710086683208e-1, 9.0757541967095705362e-1, 7.96093065705643745998e-1, 6.47386284781827639182e-1, 4.68408440699790139216e-1, 2.67528338529220821195e-1, 5.41389085854175261499e-2, -1.61781996552764726544e-1, -3.70138155339914356864e-1, -5.6118706536238236927e-1, -7.25995491923130858138e-1, -8.56857176167589244523e-1, -9.47653171182802444274e-1, -9.94137957154359608955e-1};
  static constexpr double s[14] = {2.14970440211024067182e-1, 4.19889101560264576974e-1, 6.05174215193765165924e-1, 7.62162055127636463256e-1, 8.83512044446022922827e-1, 9.63549992519222960043e-1, 9.98533413851123864572e-1, 9.86826522541526151769e-1, 9.2897671981679144179e-1, 8.27688998156890556136e-1, 6.87699458853423293084e-1, 5.1555385717702173971e-1, 3.19301530135979973197e-1, 1.08119018423941763031e-1};
};
template <> struct OddRoots<31> {
  static constexpr double c[15] = {9.79529941252494493938e-1, 9.18957811620230629127e-1, 8.20763441207276326364e-1, 6.88966919075686567801e-1, 5.28964010326962457365e-1, 3.47305252844820285542e-1, 1.51427777504576663657e-1, -5.06491688387127122788e-2, -2.50652532258720539315e-1, -4.40394151557634309516e-1, -6.12105982547662844147e-1, -7.58758122692790901913e-1, -8.74346616144582118827e-1, -9.54139256400048851476e-1, -9.94869323391895146321e-1};
  static constexpr double s[15] = {2.01298520088660079142e-1, 3.94355855113318580102e-1, 5.71268215094792279157e-1, 7.24792787229119958865e-1, 8.48644257494750950464e-1, 9.37752132147080458429e-1, 9.88468324328111399162e-1, 9.98716507171052807146e-1, 9.68077118866204305153e-1, 8.97804539570741657137e-1, 7.90775736937698582078e-1, 6.51372482722222207454e-1, 4.85301962531081025215e-1, 2.99363122973357954008e-1, 1.01168321987432177786e-1};
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

// Stockham stage of a large odd radix R (>= kStreamRadix), streamed through
// LDS from the line `in` to the separate region `out`: no thread holds the R
// inputs at once.  Phase 1: the kStreamThreads threads of butterfly j
// (k = j mod Ns) twiddle its inputs, y_r = x_r w^{rk}, and replace x_m,
// x_{R-m} in the butterfly's own slots by s_m = y_m + y_{R-m} and
// d_m = y_m - y_{R-m}.  Phase 2: thread g of the butterfly forms the output
// pairs of its block,
//   X_q = y_0 + sum_m s_m cos(2 pi m q / R) - i sum_m d_m sin(2 pi m q / R),
// and X_{R-q} (+i), from those slots (block 0 also X_0 = y_0 + sum_m s_m),
// and writes X_r to out[(j - k) R + k + r Ns], the stage's output positions,
// which in place would be other butterflies' inputs.  Each wave of the line
// group takes one block for 64 butterflies at a time, so the block (and with
// it the root table row) is uniform across the wave and the roots come in
// through scalar loads; the loop over m keeps only the block's accumulators
// and one pair live.
template <int R>
struct StreamRoots {
  static constexpr int h = (R - 1) / 2;
  static constexpr int KB = (h + kStreamThreads - 1) / kStreamThreads;
  // [block][m - 1][q]: cos / sin(2 pi m k / R) for k = block KB + 1 + q
  // (zero past h)
  double c[kStreamThreads][h][KB];
  double s[kStreamThreads][h][KB];
  constexpr StreamRoots() : c(), s() {
    for (int g = 0; g < kStreamThreads; ++g)
      for (int m = 1; m <= h; ++m)
        for (int q = 0; q < KB; ++q) {
          const int k = g * KB + 1 + q;
          if (k > h) continue;
          const int mk = (m * k) % R;
          const int mm = mk <= h ? mk : R - mk;
          c[g][m - 1][q] = OddRoots<R>::c[mm - 1];
          s[g][m - 1][q] = mk <= h ? OddRoots<R>::s[mm - 1] : -OddRoots<R>::s[mm - 1];
        }
  }
};
template <int R>
__device__ constexpr StreamRoots<R> kStreamRoots{};

template <typename T, int R>
__device__ __forceinline__ void stockham_streamed(Line<T> in, Line<T> out, int N, int Ns, const cpx<T> *tw,
                                                  int lt, int TL, bool active) {
  using SR = StreamRoots<R>;
  constexpr int h = SR::h, KB = SR::KB;
  const int NR = N / R;
  const int tstride = N / (Ns * R);
  const float rns = 1.0f / (float)Ns;
  // wave w of the line group: block g = w mod kStreamThreads, chunks of 64
  // butterflies w / kStreamThreads, + cstep, ...
  const int w = __builtin_amdgcn_readfirstlane(lt >> 6);
  const int g = w % kStreamThreads;
  const int cstep = (TL >> 6) / kStreamThreads;
  const int nch = (NR + 63) >> 6;
  const bool on = active && w < kStreamThreads * cstep;
  if (on)
    for (int ch = w / kStreamThreads; ch < nch; ch += cstep) {
      const int j = (ch << 6) + (lt & 63);
      if (j >= NR) continue;
      const int k = mod_small(j, Ns, rns);
      for (int m = g + 1; m <= h; m += kStreamThreads) {
        cpx<T> a = in[j + m * NR], b = in[j + (R - m) * NR];
        if (k != 0) {
          a = cmul(a, tw[m * k * tstride]);
          b = cmul(b, tw[(R - m) * k * tstride]);
        }
        in[j + m * NR] = cadd(a, b);
        in[j + (R - m) * NR] = csub(a, b);
      }
    }
  __syncthreads();
  if (on) {
    const int k0 = g * KB + 1;
    const int nk = min(KB, h - k0 + 1);
    const double *cr = &kStreamRoots<R>.c[g][0][0];
    const double *sr = &kStreamRoots<R>.s[g][0][0];
    for (int ch = w / kStreamThreads; ch < nch; ch += cstep) {
      const int j = (ch << 6) + (lt & 63);
      if (j >= NR) continue;
      const cpx<T> x0 = in[j];
      cpx<T> A[KB], B[KB];
      cpx<T> tot = x0;
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        A[q] = x0;
        B[q] = {T(0), T(0)};
      }
#pragma unroll 1
      for (int m = 1; m <= h; ++m) {
        const cpx<T> sm = in[j + m * NR], dm = in[j + (R - m) * NR];
        tot = cadd(tot, sm);
#pragma unroll
        for (int q = 0; q < KB; ++q) {
          const T c = T(cr[(m - 1) * KB + q]), sn = T(sr[(m - 1) * KB + q]);
          A[q].r += sm.r * c;
          A[q].i += sm.i * c;
          B[q].r += dm.r * sn;
          B[q].i += dm.i * sn;
        }
      }
      const int k = mod_small(j, Ns, rns);
      const int o = (j - k) * R + k;
      if (g == 0) out[o] = tot;
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (q < nk) {
          out[o + (k0 + q) * Ns] = cadd(A[q], cmi(B[q]));
          out[o + (R - k0 - q) * Ns] = cadd(A[q], cpi(B[q]));
        }
    }
  }
  __syncthreads();
}

// Forward FFT of length N = prod(radix) in place on buf (natural order).
// BIG enables the odd radices 11 .. 31 as streamed stages that alternate
// between buf and the plan's spare region; only the PPE kernels instantiate
// it, which keeps the operator kernels' register budget at that of radices
// <= 8.  The result ends in buf.
template <typename T, bool BIG = false, bool WIDE = false>
__device__ __forceinline__ void fft_stockham(Line<T> buf, const LinePlan &p, int N, int lt, int TL,
                                             bool active) {
  const cpx<T> *tw = static_cast<const cpx<T> *>(p.tw);
  int Ns = 1;
  Line<T> line = buf;
  // spare is a multiple of the padding period, so this view indexes the same
  // slots as buf[spare + i]
  Line<T> other{buf.p + p.spare + (p.spare >> kLdsPadShift)};
  for (int s = 0; s < p.nstages; ++s) {
    const int R = p.radix[s];
    switch (R) {
      case 2: stockham_stage<T, 2, WIDE>(line, N, Ns, tw, lt, TL, active); break;
      case 3: stockham_stage<T, 3, WIDE>(line, N, Ns, tw, lt, TL, active); break;
      case 4: stockham_stage<T, 4, WIDE>(line, N, Ns, tw, lt, TL, active); break;
      case 5: stockham_stage<T, 5, WIDE>(line, N, Ns, tw, lt, TL, active); break;
      case 7: stockham_stage<T, 7, WIDE>(line, N, Ns, tw, lt, TL, active); break;
      case 8: stockham_stage<T, 8, WIDE>(line, N, Ns, tw, lt, TL, active); break;
      default:
        if constexpr (BIG) {
          switch (R) {
            case 11: stockham_streamed<T, 11>(line, other, N, Ns, tw, lt, TL, active); break;
            case 13: stockham_streamed<T, 13>(line, other, N, Ns, tw, lt, TL, active); break;
            case 17: stockham_streamed<T, 17>(line, other, N, Ns, tw, lt, TL, active); break;
            case 19: stockham_streamed<T, 19>(line, other, N, Ns, tw, lt, TL, active); break;
            case 23: stockham_streamed<T, 23>(line, other, N, Ns, tw, lt, TL, active); break;
            case 29: stockham_streamed<T, 29>(line, other, N, Ns, tw, lt, TL, active); break;
            case 31: stockham_streamed<T, 31>(line, other, N, Ns, tw, lt, TL, active); break;
            default: break;
          }
          const Line<T> t = line;
          line = other;
          other = t;
        }
        break;   // the host never builds other radices
    }
    Ns *= R;
  }
  if constexpr (BIG) {
    if (line.p != buf.p) {
      // back from the spare region
      if (active)
        for (int j = lt; j < N; j += TL) buf[j] = line[j];
      __syncthreads();
    }
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
