// Host side of the library: C ABI, argument validation, plan construction
// (tables computed in long double and rounded once), workspace layout and the
// launch sequences of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fcsph.h"
#include "internal.h"

using namespace fcsph;

struct TimedLaunch {
  const char *name;
  hipEvent_t start, stop;
};

struct fcsph_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  bool timing = false;
  std::string timing_only;               // time only this kernel kind (empty: all)
  std::vector<TimedLaunch> launches;     // recorded while timing is on
  std::vector<hipEvent_t> event_pool;    // reusable events
};

namespace {
hipEvent_t pool_event(fcsph_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  // timing only (read after the caller's synchronisation): no system-scope
  // fence at record time, so an event between two kernels neither writes
  // back nor invalidates the caches the next kernel reads
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when the context records timings.
struct LaunchTimer {
  fcsph_ctx *c;
  const char *name;
  hipEvent_t a = nullptr, b = nullptr;
  LaunchTimer(fcsph_ctx *ctx, const char *n) : c(ctx), name(n) {
    if (c && c->timing && !active_recorder() && (c->timing_only.empty() || c->timing_only == n)) {
      a = pool_event(c);
      b = pool_event(c);
      if (a) hipEventRecord(a, c->stream);
    }
  }
  ~LaunchTimer() {
    if (a && b) {
      hipEventRecord(b, c->stream);
      c->launches.push_back({name, a, b});
    }
  }
};
}  // namespace

// ------------------------------------------------------ static device scratch
// Scratch of the no-allocation entry point (fcsph_spectral_lap_noalloc): a
// file-scope device array of fixed size, one copy per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it names a stand-in, not device memory): each device's address comes
// from hipGetSymbolAddress, taken once per device with that device current
// (at context creation) and kept in g_scratch.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// With `device` current: record this device's address of the scratch array.
void register_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) g_scratch[device] = ptr;
  else g_scratch_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

void *scratch_of(int device, hipError_t *err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  *err = g_scratch[device] ? hipSuccess : g_scratch_err[device];
  return g_scratch[device];
}
}  // namespace

namespace {

typedef long double LD;
const LD kPi = 3.141592653589793238462643383279502884L;

// ----------------------------------------------------------------- workspace
struct Bump {
  char *base = nullptr;   // null: dry run (size only)
  size_t off = 0;
  void *take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    void *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

// Host staging of a table before copy to the workspace.
struct Upload {
  void *dst;
  std::vector<char> data;
};

// ----------------------------------------------------------------- line plans
bool factor_direct(int n, std::vector<int> &rad, bool big = false) {
  rad.clear();
  int m = n;
  if (big) {
    // large odd primes (streamed stages) first, largest first: the first
    // stage takes no twiddles
    const int odd_big[] = {31, 29, 23, 19, 17, 13, 11};
    for (int p : odd_big)
      while (m % p == 0) { rad.push_back(p); m /= p; }
  }
  while (m % 8 == 0 && m > 8) { rad.push_back(8); m /= 8; }
  if (m % 8 == 0) { rad.push_back(8); m /= 8; }
  while (m % 4 == 0) { rad.push_back(4); m /= 4; }
  while (m % 2 == 0) { rad.push_back(2); m /= 2; }
  const int odd[] = {3, 5, 7};
  for (int p : odd)
    while (m % p == 0) { rad.push_back(p); m /= p; }
  if (m != 1) return false;
  if (rad.empty()) rad.push_back(1);
  return (int)rad.size() <= kMaxStages;
}

bool smooth7(int m) {
  const int ps[] = {2, 3, 5, 7};
  for (int p : ps)
    while (m % p == 0) m /= p;
  return m == 1;
}

// Threads per line group (a multiple of 64) that a Stockham plan with these
// radices needs on a work length M, or 0 if it exceeds the workgroup bound.
int line_threads(int M, const std::vector<int> &rad, int min_TL = 64, bool wide = false) {
  int tl = std::max(64, min_TL);
  for (int R : rad) {
    if (R <= 1) continue;
    if (R >= kStreamRadix) {
      tl = std::max(tl, stream_threads(M, R));   // streamed stage
      continue;
    }
    tl = std::max(tl, (M / R + nb_max(R, wide) - 1) / nb_max(R, wide));
  }
  tl = (tl + 63) / 64 * 64;
  return tl > kMaxThreads ? 0 : tl;
}

// Transform length of a windowed walled axis: the cheapest L >= n + 2 R whose
// factors are all radices with straight-line butterflies (2, 3, 4, 5, 7, 8).
// Cost model per point: a fixed HBM term plus a per-stage butterfly term.
// FCSPH_WINDOW_L=<L> overrides (used by the schedule tuner).
int window_length(int n, int R) {
  const int lo = n + 2 * R;
  if (const char *e = getenv("FCSPH_WINDOW_L")) {
    const int L = atoi(e);
    std::vector<int> rad;
    if (L >= lo && factor_direct(L, rad) && line_threads(L, rad)) return L;
  }
  double best = 1e300;
  int bestL = -1;
  for (int L = lo; L <= 2 * lo + 8; ++L) {
    std::vector<int> rad;
    if (!factor_direct(L, rad) || !line_threads(L, rad)) continue;
    double c = 4.0;
    bool ok = true;
    for (int r : rad) {
      switch (r) {
        case 1: break;
        case 2: c += 1.0; break;
        case 3: c += 1.35; break;
        case 4: c += 1.1; break;
        case 5: c += 1.7; break;
        case 7: c += 2.4; break;
        case 8: c += 1.4; break;
        default: ok = false;
      }
    }
    if (!ok) continue;
    const double cost = c * L;
    if (cost < best) {
      best = cost;
      bestL = L;
    }
  }
  return bestL;
}

template <typename T>
void put_cpx(std::vector<char> &v, size_t idx, LD re, LD im) {
  cpx<T> c = {static_cast<T>(re), static_cast<T>(im)};
  std::memcpy(v.data() + idx * sizeof(cpx<T>), &c, sizeof(c));
}

struct LineSpec {
  LinePlan p{};
  size_t bytes_tables = 0;
};

// Build a line plan for length n.  min_TL forces a minimum thread count per
// line (used where the kernel keeps E / TL spectrum values in registers).
bool make_line_plan(int n, bool fp32, int min_TL, Bump &ws, std::vector<Upload> &up, LinePlan &p,
                    bool big = false, bool wide = false, int order = 0) {
  std::memset(&p, 0, sizeof(p));
  p.n = n;
  std::vector<int> rad;
  int M = n;
  int tl = 0;
  if (n == 1) {
    rad = {};
    tl = std::max(64, (min_TL + 63) / 64 * 64);
  } else if (factor_direct(n, rad, big) && (tl = line_threads(n, rad, min_TL, wide)) > 0) {
    p.blue = 0;
  } else {
    // Bluestein: the smallest 7-smooth M >= 2n - 1 whose stages fit one
    // workgroup's line group (a direct length too long for it comes here too)
    p.blue = 1;
    for (M = 2 * n - 1; M <= 8 * n; ++M)
      if (smooth7(M) && factor_direct(M, rad) && (tl = line_threads(M, rad, min_TL, wide)) > 0) break;
    if (tl <= 0 || tl > kMaxThreads) return false;
  }
  // schedule hint: the ((order - 1) mod m)-th distinct ordering of the radices
  // (lexicographic from the ascending one); the twiddle table serves any order
  if (order > 0 && !big && rad.size() > 1) {
    std::sort(rad.begin(), rad.end());
    int m = 0;
    std::vector<int> r = rad;
    do ++m; while (std::next_permutation(r.begin(), r.end()));
    for (int k = (order - 1) % m; k > 0; --k) std::next_permutation(rad.begin(), rad.end());
  }
  p.M = M;
  p.wide = wide ? 1 : 0;
  p.nstages = (int)rad.size();
  if (n == 1) p.nstages = 0;
  for (int s = 0; s < p.nstages; ++s) p.radix[s] = rad[s];
  // streamed stages write to a second region of the line buffer, starting at
  // a multiple of the LDS padding period
  p.spare = 0;
  for (int s = 0; s < p.nstages; ++s)
    if (p.radix[s] >= kStreamRadix) p.spare = (M + 1 + 15) & ~15;
  p.TL = tl;
  // LDS padding (one slot every 16 elements): a sweep of 0..5 on the 1024^2
  // step put 3..5 ahead of none by 2-4 %; the device code uses the fixed shift
  p.pad = kLdsPadShift;
  const size_t es = fp32 ? sizeof(cpx<float>) : sizeof(cpx<double>);
  // twiddles exp(-2 pi i t / M)
  {
    Upload u;
    u.data.resize((size_t)M * es);
    for (int t = 0; t < M; ++t) {
      const LD a = -2.0L * kPi * (LD)t / (LD)M;
      if (fp32) put_cpx<float>(u.data, t, cosl(a), sinl(a));
      else put_cpx<double>(u.data, t, cosl(a), sinl(a));
    }
    u.dst = ws.take(u.data.size());
    p.tw = u.dst;
    up.push_back(std::move(u));
  }
  if (p.blue) {
    // chirp w_j = exp(-pi i (j^2 mod 2n) / n)
    std::vector<LD> cr(n), ci(n);
    for (int j = 0; j < n; ++j) {
      const long long q = ((long long)j * j) % (2LL * n);
      const LD a = -kPi * (LD)q / (LD)n;
      cr[j] = cosl(a);
      ci[j] = sinl(a);
    }
    Upload uc;
    uc.data.resize((size_t)n * es);
    for (int j = 0; j < n; ++j) {
      if (fp32) put_cpx<float>(uc.data, j, cr[j], ci[j]);
      else put_cpx<double>(uc.data, j, cr[j], ci[j]);
    }
    uc.dst = ws.take(uc.data.size());
    p.chirp = uc.dst;
    up.push_back(std::move(uc));
    // filter b_m = conj(w_m) for |m| < n (wrapped mod M); filt = DFT_M(b) / M
    std::vector<LD> br(M, 0.0L), bi(M, 0.0L);
    for (int m = 0; m < n; ++m) {
      br[m] = cr[m];
      bi[m] = -ci[m];
      if (m > 0) {
        br[M - m] = cr[m];
        bi[M - m] = -ci[m];
      }
    }
    // the O(M^2) long-double DFT of the filter is cached per (n, M): plans of
    // the same line length (batches, served requests) reuse it
    static std::mutex filt_mu;
    static std::map<std::pair<int, int>, std::vector<LD>> filt_cache;
    std::vector<LD> spec;
    {
      std::lock_guard<std::mutex> lock(filt_mu);
      auto it = filt_cache.find({n, M});
      if (it != filt_cache.end()) spec = it->second;
    }
    if (spec.empty()) {
      std::vector<LD> twr(M), twi(M);
      for (int t = 0; t < M; ++t) {
        const LD a = -2.0L * kPi * (LD)t / (LD)M;
        twr[t] = cosl(a);
        twi[t] = sinl(a);
      }
      spec.assign(2 * (size_t)M, 0.0L);
      for (int k = 0; k < M; ++k) {
        LD sr = 0.0L, si = 0.0L;
        long long idx = 0;
        for (int m = 0; m < M; ++m) {
          if (br[m] != 0.0L || bi[m] != 0.0L) {
            sr += br[m] * twr[idx] - bi[m] * twi[idx];
            si += br[m] * twi[idx] + bi[m] * twr[idx];
          }
          idx += k;
          if (idx >= M) idx -= M;
        }
        spec[2 * (size_t)k] = sr / M;
        spec[2 * (size_t)k + 1] = si / M;
      }
      std::lock_guard<std::mutex> lock(filt_mu);
      filt_cache[{n, M}] = spec;
    }
    Upload uf;
    uf.data.resize((size_t)M * es);
    for (int k = 0; k < M; ++k) {
      if (fp32) put_cpx<float>(uf.data, k, spec[2 * (size_t)k], spec[2 * (size_t)k + 1]);
      else put_cpx<double>(uf.data, k, spec[2 * (size_t)k], spec[2 * (size_t)k + 1]);
    }
    uf.dst = ws.take(uf.data.size());
    p.filt = uf.dst;
    up.push_back(std::move(uf));
  }
  return true;
}

// Workgroup line count for a plan and per-line buffer size.
int pick_B(const LinePlan &p, bool fp32, int want, int nbuf = 1, int len = 0) {
  const size_t es = fp32 ? sizeof(cpx<float>) : sizeof(cpx<double>);
  const int m = len > 0 ? len : p.M;
  int B = want;
  while (B > 1 && ((size_t)B * nbuf * padded_len(m, p.pad) * es > (size_t)kMaxLds || B * p.TL > kMaxThreads)) --B;
  return B;
}

bool is_gaussian(int k) {
  return k == FCSPH_KERNEL_GAUSSIAN_G2 || k == FCSPH_KERNEL_GAUSSIAN_G4 || k == FCSPH_KERNEL_GAUSSIAN_G6 ||
         k == FCSPH_KERNEL_GAUSSIAN_G8 || k == FCSPH_KERNEL_GAUSSIAN_G10;
}

// ----------------------------------------------------------------- Gaussian symbols
// The Gaussian of order 2n (2D): W = (1/(pi h^2)) P(s) exp(-s), s = q^2, with
// P(s) = sum_{m<n} A_m s^m solving sum_m A_m m+j! = delta_{j0}, j < n (the
// moment conditions with I_k = k!).  Its taps (dV times the gradient and the
// Laplacian at the minimum-image displacement x, y) are
//   d_x W = (2 a / h^2) x Q1(s) e^-s,   lap W = (4 a / h^2) Q3(s) e^-s,
//   Q1 = P' - P,  Q3 = s (P'' - 2 P' + P) + Q1,  a = 1 / (pi h^2),
// and with s = u + v (u = x^2/h^2, v = y^2/h^2), s^m = sum_i C(m,i) u^i v^(m-i):
// every symbol (the DFT of the sampled taps over the extended lattice) is a
// sum of products of one-dimensional DFTs of x^e u^i e^-u (e = 0, 1).  An
// offset at exactly half a period averages its two images: the odd factors
// vanish there, the even ones keep their value.
std::vector<LD> gaussian_coeffs(int order) {
  const int n = order / 2;
  std::vector<std::vector<LD>> M(n, std::vector<LD>(n + 1, 0.0L));
  auto fact = [](int k) {
    LD f = 1.0L;
    for (int i = 2; i <= k; ++i) f *= (LD)i;
    return f;
  };
  for (int j = 0; j < n; ++j) {
    for (int m = 0; m < n; ++m) M[j][m] = fact(m + j);
    M[j][n] = j == 0 ? 1.0L : 0.0L;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(M[r][c]) > fabsl(M[piv][c])) piv = r;
    std::swap(M[c], M[piv]);
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const LD f = M[r][c] / M[c][c];
        for (int q = c; q <= n; ++q) M[r][q] -= f * M[c][q];
      }
  }
  std::vector<LD> A(n);
  for (int i = 0; i < n; ++i) A[i] = M[i][n] / M[i][i];
  return A;
}

// 1D DFTs over the minimum-image offsets of a period-E axis (spacing dx,
// smoothing length h): F[e][i][k] = sum_s g(s dx) exp(-2 pi i k s / E),
// g(x) = x^e (x^2/h^2)^i exp(-x^2/h^2), e = 0, 1, i = 0..imax.
void gaussian_axis_dfts(int E, LD dx, LD h, int imax, std::vector<std::vector<std::vector<std::pair<LD, LD>>>> &F) {
  F.assign(2, std::vector<std::vector<std::pair<LD, LD>>>(imax + 1, std::vector<std::pair<LD, LD>>(E, {0.0L, 0.0L})));
  std::vector<LD> ct(E), st(E);
  for (int t = 0; t < E; ++t) {
    const LD ang = -2.0L * kPi * (LD)t / (LD)E;
    ct[t] = cosl(ang);
    st[t] = sinl(ang);
  }
  for (int s = -((E - 1) / 2); s <= E / 2; ++s) {
    const bool tie = 2 * s == E;
    const LD x = (LD)s * dx, u = x * x / (h * h), g0 = expl(-u);
    LD up = 1.0L;
    for (int i = 0; i <= imax; ++i) {
      const LD ev = up * g0, od = tie ? 0.0L : x * up * g0;
      const int sm = ((s % E) + E) % E;
      long long idx = 0;
      for (int k = 0; k < E; ++k) {
        F[0][i][k].first += ev * ct[idx];
        F[0][i][k].second += ev * st[idx];
        F[1][i][k].first += od * ct[idx];
        F[1][i][k].second += od * st[idx];
        idx += sm;
        if (idx >= E) idx -= E;
      }
      up *= u;
    }
  }
}

// Full symbol table symF[q][kx][ky] (q = SYM_GX, SYM_GY, unused, SYM_LAP;
// kx < Ex/2 + 1, ky < Ey), in the library's convention of weights divided by
// Ex Ey.  Also returns max_k sum_a sigma_a(k)^2 (unnormalised).
std::vector<double2> gaussian_symbols_2d(int order, double dx_, double hod, int Ex, int Ey, double &sig2max) {
  const LD dx = dx_, h = (LD)hod * dx;
  const std::vector<LD> A = gaussian_coeffs(order);
  const int n = (int)A.size();
  // P, P', P'' coefficients; Q1 = P' - P, Q3 = s (P'' - 2P' + P) + Q1 (degree <= n)
  std::vector<LD> P(n + 2, 0.0L), dP(n + 2, 0.0L), ddP(n + 2, 0.0L);
  for (int m = 0; m < n; ++m) P[m] = A[m];
  for (int m = 1; m < n; ++m) dP[m - 1] = (LD)m * A[m];
  for (int m = 2; m < n; ++m) ddP[m - 2] = (LD)m * (LD)(m - 1) * A[m];
  std::vector<LD> Q1(n + 2, 0.0L), Q3(n + 2, 0.0L);
  for (int m = 0; m <= n; ++m) Q1[m] = dP[m] - P[m];
  for (int m = 0; m <= n; ++m) {
    const LD q2 = ddP[m] - 2.0L * dP[m] + P[m];
    Q3[m + 1] += q2;
    Q3[m] += Q1[m];
  }
  const LD a = 1.0L / (kPi * h * h), dV = dx * dx;
  const LD K1 = dV * 2.0L * a / (h * h), K3 = dV * 4.0L * a / (h * h);
  std::vector<std::vector<std::vector<std::pair<LD, LD>>>> FX, FY;
  gaussian_axis_dfts(Ex, dx, h, n + 1, FX);
  gaussian_axis_dfts(Ey, dx, h, n + 1, FY);
  std::vector<LD> binom((n + 2) * (n + 2), 0.0L);
  for (int m = 0; m <= n + 1; ++m) {
    binom[m * (n + 2)] = 1.0L;
    for (int i = 1; i <= m; ++i) binom[m * (n + 2) + i] = binom[(m - 1) * (n + 2) + i - 1] + (i <= m - 1 ? binom[(m - 1) * (n + 2) + i] : 0.0L);
  }
  const int Hx = Ex / 2 + 1;
  const LD norm = (LD)Ex * (LD)Ey;
  std::vector<double2> out((size_t)4 * Hx * Ey, make_double2(0.0, 0.0));
  LD s2max = 0.0L;
  auto cm = [](std::pair<LD, LD> p, std::pair<LD, LD> q) {
    return std::make_pair(p.first * q.first - p.second * q.second, p.first * q.second + p.second * q.first);
  };
  for (int kx = 0; kx < Hx; ++kx)
    for (int ky = 0; ky < Ey; ++ky) {
      std::pair<LD, LD> gx{0.0L, 0.0L}, gy{0.0L, 0.0L}, lp{0.0L, 0.0L};
      for (int m = 0; m <= n; ++m)
        for (int i = 0; i <= m; ++i) {
          const LD b = binom[m * (n + 2) + i];
          if (Q1[m] != 0.0L) {
            const auto tx = cm(FX[1][i][kx], FY[0][m - i][ky]);
            const auto ty = cm(FX[0][i][kx], FY[1][m - i][ky]);
            gx.first += K1 * Q1[m] * b * tx.first;
            gx.second += K1 * Q1[m] * b * tx.second;
            gy.first += K1 * Q1[m] * b * ty.first;
            gy.second += K1 * Q1[m] * b * ty.second;
          }
          if (Q3[m] != 0.0L) {
            const auto tl = cm(FX[0][i][kx], FY[0][m - i][ky]);
            lp.first += K3 * Q3[m] * b * tl.first;
            lp.second += K3 * Q3[m] * b * tl.second;
          }
        }
      const size_t base = (size_t)kx * Ey + ky;
      out[(size_t)SYM_GX * Hx * Ey + base] = make_double2((double)(gx.first / norm), (double)(gx.second / norm));
      out[(size_t)SYM_GY * Hx * Ey + base] = make_double2((double)(gy.first / norm), (double)(gy.second / norm));
      out[(size_t)SYM_LAP * Hx * Ey + base] = make_double2((double)(lp.first / norm), (double)(lp.second / norm));
      const LD s2 = gx.second * gx.second + gy.second * gy.second;
      if (s2 > s2max) s2max = s2;
    }
  sig2max = (double)s2max;
  return out;
}

// ----------------------------------------------------------------- kernel taps
// Wendland C2 (q = r/h, s = 1 - q/2):  grad W = -(5 alpha/h^2) s^3 x,
// lap W = -(5 alpha/h^2) s^2 (2 - 5q/2) in 2D, (3 - 3q) in 3D.
void wendland_taps(int ndim, double dx, double hod, const int *E, std::vector<double> W[4]) {
  const int cube = ndim == 2 ? kSymW * kSymW : kSymW * kSymW * kSymW;
  for (int q = 0; q < 4; ++q) W[q].assign(cube, 0.0);
  const LD h = (LD)hod * (LD)dx;
  const LD alpha = ndim == 2 ? 7.0L / (4.0L * kPi * h * h) : 21.0L / (16.0L * kPi * h * h * h);
  const LD dV = ndim == 2 ? (LD)dx * dx : (LD)dx * dx * dx;
  LD norm = 1.0L;
  for (int a = 0; a < ndim; ++a) norm *= (LD)E[a];
  const int zr = ndim == 3 ? kSymR : 0;
  for (int sz = -zr; sz <= zr; ++sz)
    for (int sy = -kSymR; sy <= kSymR; ++sy)
      for (int sx = -kSymR; sx <= kSymR; ++sx) {
        const LD r2 = (LD)(sx * sx + sy * sy + sz * sz);
        const LD r = sqrtl(r2) * (LD)dx;
        const LD q = r / h;
        if (!(q < 2.0L)) continue;
        const LD s = 1.0L - q / 2.0L;
        const LD pre = -5.0L * alpha / (h * h);
        const LD g = pre * s * s * s * dV;
        const LD lap = pre * s * s * (ndim == 2 ? (2.0L - 2.5L * q) : (3.0L - 3.0L * q)) * dV;
        const int idx = ndim == 2 ? (sy + kSymR) * kSymW + (sx + kSymR)
                                  : ((sz + kSymR) * kSymW + (sy + kSymR)) * kSymW + (sx + kSymR);
        W[0][idx] = (double)(g * (LD)sx * (LD)dx / norm);
        W[1][idx] = (double)(g * (LD)sy * (LD)dx / norm);
        if (ndim == 3) W[2][idx] = (double)(g * (LD)sz * (LD)dx / norm);
        W[3][idx] = (double)(lap / norm);
      }
}

// Compact tap list for the direct evaluation (un-normalised weights).
std::vector<Tap> wendland_tap_list(int ndim, double dx, double hod, int &reach) {
  std::vector<Tap> out;
  const LD h = (LD)hod * (LD)dx;
  const LD alpha = ndim == 2 ? 7.0L / (4.0L * kPi * h * h) : 21.0L / (16.0L * kPi * h * h * h);
  const LD dV = ndim == 2 ? (LD)dx * dx : (LD)dx * dx * dx;
  const int zr = ndim == 3 ? kSymR : 0;
  reach = 0;
  for (int sz = -zr; sz <= zr; ++sz)
    for (int sy = -kSymR; sy <= kSymR; ++sy)
      for (int sx = -kSymR; sx <= kSymR; ++sx) {
        const LD q = sqrtl((LD)(sx * sx + sy * sy + sz * sz)) * (LD)dx / h;
        if (!(q < 2.0L)) continue;
        const LD s = 1.0L - q / 2.0L;
        const LD pre = -5.0L * alpha / (h * h);
        const LD g = pre * s * s * s * dV;
        Tap t{};
        t.s[0] = sx;
        t.s[1] = sy;
        t.s[2] = sz;
        t.w[0] = (double)(g * (LD)sx * (LD)dx);
        t.w[1] = (double)(g * (LD)sy * (LD)dx);
        t.w[2] = (double)(g * (LD)sz * (LD)dx);
        t.w[3] = (double)(pre * s * s * (ndim == 2 ? (2.0L - 2.5L * q) : (3.0L - 3.0L * q)) * dV);
        out.push_back(t);
        reach = std::max(reach, std::max(std::abs(sx), std::max(std::abs(sy), std::abs(sz))));
      }
  return out;
}

}  // namespace

// ----------------------------------------------------------------- the plan
struct fcsph_plan {
  fcsph_ctx *ctx = nullptr;
  fcsph_desc d{};
  bool fp32 = false;
  int nd = 2;
  int n[3] = {1, 1, 1};
  int E[3] = {1, 1, 1};     // operator transform length per axis
  int Efc[3] = {1, 1, 1};   // FC-extended period per axis (n + C on walled axes)
  bool window = false;      // windowed operator transforms
  int want_B = 4;           // lines per workgroup of the line kernels (upper bound)
  int walled[3] = {0, 0, 0};
  int H = 0;            // x half spectrum
  // FC maps (device)
  const double *M_dir = nullptr, *M_neu = nullptr;
  // line plans
  LinePlan op[3];       // operator DFT along each axis (length E[a])
  LinePlan op64[3];     // FP32-mixed plans: FP64 twins for the PPE right-hand side
  LinePlan trig[3];     // PPE transform along each axis
  bool ppe_streamed = false;   // some trig plan has streamed stages (no batches)
  int trig_kind[3] = {0, 0, 0};
  int ncoef[3] = {0, 0, 0};
  const double *mu[3] = {nullptr, nullptr, nullptr};
  const void *qtw[3] = {nullptr, nullptr, nullptr};   // quarter-wave pre-twiddles
  const double2 *dcs[3] = {nullptr, nullptr, nullptr};  // DCT-I at length N: (cos, sin)(pi j / N)
  const double2 *symR2 = nullptr;   // 2D: tabulated symbol line coefficients (y lines)
  const double2 *symR3 = nullptr;   // 3D: the same for the z lines (inner x, outer y)
  const double2 *symF2 = nullptr;   // 2D Gaussian kernels: the full symbols [q][kx][ky]
  // symbols
  SymTables st{};
  // scratch
  void *S[3] = {nullptr, nullptr, nullptr};   // input spectra
  void *O[12] = {};                            // output spectra
  void *Y[3] = {nullptr, nullptr, nullptr};    // 3D: y-extended spectra
  size_t spec_elems = 0;
  double *ustar[3] = {nullptr, nullptr, nullptr};
  void *rhs = nullptr;          // PPE right-hand side (output type)
  double *phi = nullptr;        // pressure scratch
  void *coef = nullptr;         // PPE coefficient rows
  int cpitch = 0;
  double *ext_scratch = nullptr;  // intermediate of a multi-axis FC extension
  void *edge[3] = {nullptr, nullptr, nullptr};   // FP32 plans: FP64 boundary-row x spectra per field
  bool direct = false;            // operators as direct tap sums
  double wd2[3][kSymW * kSymW] = {};   // 2D dense tap weights (grad x, grad y, lap)
  double *ghx[3] = {}, *ghy[3] = {};    // FC ghost values of up to 3 direct-pass inputs
  const Tap *taps = nullptr;
  int ntaps = 0, reach = 0;
  // upper bound of sum_a sigma_a(k)^2 over every wavenumber (sum over the axes
  // of the squared l1 norm of the gradient taps), for the zero-mode tolerance
  // of the SPH family and the EXTENDED projection
  double sigma2_bound = 0.0;
  unsigned long long *counter = nullptr;   // device counter of fcsph_check_finite
  size_t ws_bytes = 0;
};

namespace {
// Line buffer elements of the PPE transform along axis a: the transform work
// length, plus the result and 8 partial-sum slots for the length-N DCT-I.
int ppe_line_len(const fcsph_plan *p, int a) {
  const LinePlan &t = p->trig[a];
  const int len = p->dcs[a] ? t.M + 1 + t.n + 1 + 8 : t.M;
  return t.spare ? std::max(len, t.spare + t.M) : len;
}
}  // namespace

namespace {

fcsph_status fail(fcsph_ctx *c, fcsph_status s, const std::string &msg) {
  if (c) c->last_error = msg;
  return s;
}

fcsph_status hip_fail(fcsph_ctx *c, hipError_t e, const char *where) {
  return fail(c, FCSPH_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Field class of a transported scalar (FC with the value map on every wall).
constexpr int kFieldScalar = 2;

FcWalls walls_for(const fcsph_plan *p, int axis, int fc) {
  FcWalls w{};
  w.on = p->walled[axis];
  w.C = p->d.fc_C;
  w.d = p->d.fc_d;
  w.head = w.C;
  w.tail = 0;
  if (w.on && p->window) {
    w.head = p->reach;
    w.tail = p->reach;
  }
  if (w.on && fc == kFieldScalar) {
    // a transported scalar: the plain (value) continuation on every wall
    w.Mlo = w.Mhi = p->M_dir;
  } else if (w.on) {
    const int(*bc)[2] = fc == FCSPH_FIELD_VELOCITY ? p->d.vel_bc : p->d.prs_bc;
    w.Mlo = bc[axis][0] == FCSPH_BC_NEUMANN ? p->M_neu : p->M_dir;
    w.Mhi = bc[axis][1] == FCSPH_BC_NEUMANN ? p->M_neu : p->M_dir;
  }
  return w;
}

fcsph_status validate(const fcsph_desc *d, std::string &msg) {
  if (!d) { msg = "null descriptor"; return FCSPH_E_INVALID; }
  if (d->ndim != 2 && d->ndim != 3) { msg = "ndim must be 2 or 3"; return FCSPH_E_INVALID; }
  if (!(d->dx > 0.0) || !std::isfinite(d->dx)) { msg = "dx must be positive"; return FCSPH_E_INVALID; }
  const bool gauss = is_gaussian(d->kernel);
  if (d->kernel != FCSPH_KERNEL_WENDLAND_C2 && !gauss) { msg = "unknown kernel"; return FCSPH_E_INVALID; }
  if (gauss) {
    if (!(d->h_over_dx > 0.0) || !std::isfinite(d->h_over_dx)) { msg = "h_over_dx must be positive"; return FCSPH_E_INVALID; }
    if (d->ndim != 2 || d->op_eval != FCSPH_OPS_FFT || d->eig == FCSPH_EIG_SPH) {
      msg = "the Gaussian kernels (unbounded support) are built for 2D lattices on the whole-period route "
            "(op_eval FCSPH_OPS_FFT) with the SPECTRAL or FD2 PPE";
      return FCSPH_E_UNSUPPORTED;
    }
  } else if (!(d->h_over_dx > 0.0) || 2.0 * d->h_over_dx >= kSymR + 1) {
    msg = "h_over_dx must be in (0, " + std::to_string((kSymR + 1) / 2.0) + ")";
    return FCSPH_E_UNSUPPORTED;
  }
  if (d->prec != FCSPH_FP64 && d->prec != FCSPH_FP32_MIXED) { msg = "bad precision"; return FCSPH_E_INVALID; }
  if (d->op_eval != FCSPH_OPS_FFT && d->op_eval != FCSPH_OPS_DIRECT && d->op_eval != FCSPH_OPS_FFT_WINDOW) {
    msg = "bad op_eval";
    return FCSPH_E_INVALID;
  }
  if (d->op_eval == FCSPH_OPS_DIRECT && d->ndim != 2) { msg = "direct evaluation is built for 2D"; return FCSPH_E_UNSUPPORTED; }
  if (d->ppe_domain != FCSPH_PPE_PHYSICAL && d->ppe_domain != FCSPH_PPE_EXTENDED) { msg = "bad PPE domain"; return FCSPH_E_INVALID; }
  if (d->ppe_domain == FCSPH_PPE_EXTENDED && (d->op_eval != FCSPH_OPS_FFT || d->prec != FCSPH_FP64)) {
    msg = "the EXTENDED projection is a division in the spectrum of the whole extended period: it needs "
          "op_eval FCSPH_OPS_FFT and FP64";
    return FCSPH_E_UNSUPPORTED;
  }
  if (d->eig != FCSPH_EIG_SPECTRAL && d->eig != FCSPH_EIG_FD2 && d->eig != FCSPH_EIG_SPH) { msg = "bad eigenvalue family"; return FCSPH_E_INVALID; }
  if (d->eig == FCSPH_EIG_SPH) {
    bool periodic = d->ndim == 2;
    for (int a = 0; a < d->ndim; ++a) periodic = periodic && d->axis[a] == FCSPH_AXIS_PERIODIC;
    if (!periodic || d->op_eval == FCSPH_OPS_DIRECT) {
      msg = "the SPH eigenvalue family diagonalises the PPE on 2D lattices periodic on every axis (FFT routes)";
      return FCSPH_E_UNSUPPORTED;
    }
  }
  if (!(d->rho > 0.0)) { msg = "rho must be positive"; return FCSPH_E_INVALID; }
  if (d->lines_per_group < 0 || d->lines_per_group > 16) { msg = "lines_per_group must be in 0..16"; return FCSPH_E_INVALID; }
  if (d->radix_order < 0) { msg = "radix_order must be >= 0"; return FCSPH_E_INVALID; }
  if (d->batched != 0 && d->batched != 1) { msg = "batched must be 0 or 1"; return FCSPH_E_INVALID; }
  bool any_wall = false;
  for (int a = 0; a < d->ndim; ++a) {
    if (d->n[a] < 2) { msg = "n must be >= 2"; return FCSPH_E_INVALID; }
    if (d->axis[a] != FCSPH_AXIS_PERIODIC && d->axis[a] != FCSPH_AXIS_WALLED) { msg = "bad axis kind"; return FCSPH_E_INVALID; }
    if (d->axis[a] == FCSPH_AXIS_WALLED) {
      any_wall = true;
      if (d->n[a] < 2 * d->fc_d) { msg = "walled axis needs n >= 2 fc_d"; return FCSPH_E_INVALID; }
      for (int s = 0; s < 2; ++s) {
        if ((d->vel_bc[a][s] != 0 && d->vel_bc[a][s] != 1) || (d->prs_bc[a][s] != 0 && d->prs_bc[a][s] != 1)) {
          msg = "bad wall type";
          return FCSPH_E_INVALID;
        }
      }
    }
    const int E = d->n[a] + (d->axis[a] == FCSPH_AXIS_WALLED ? d->fc_C : 0);
    if (!gauss && 2.0 * 2.0 * d->h_over_dx >= (double)E) {
      msg = "kernel support exceeds half the extended period";
      return FCSPH_E_INVALID;
    }
  }
  if (any_wall) {
    if (d->fc_d < 1 || d->fc_C < 2 || d->fc_d > 16 || d->fc_C > 4096) { msg = "bad FC sizes"; return FCSPH_E_INVALID; }
    if (!d->fc_M_dir || !d->fc_M_neu) { msg = "FC maps required for walled axes"; return FCSPH_E_INVALID; }
  }
  if (d->ndim == 3) {
    if (d->axis[0] != FCSPH_AXIS_PERIODIC || d->axis[2] != FCSPH_AXIS_PERIODIC || d->axis[1] != FCSPH_AXIS_WALLED) {
      msg = "3D lattices are built for walls in y only";
      return FCSPH_E_UNSUPPORTED;
    }
  }
  return FCSPH_OK;
}

// Lay out the plan in the workspace (dry run when ws.base is null).
fcsph_status layout(fcsph_plan *p, const fcsph_desc *d, Bump &ws, std::vector<Upload> &up, std::string &msg) {
  p->d = *d;
  p->fp32 = d->prec == FCSPH_FP32_MIXED;
  p->nd = d->ndim;
  p->window = d->op_eval == FCSPH_OPS_FFT_WINDOW;
  // one line per workgroup unless asked: the schedule tuner picked it at
  // every lattice size it timed (more workgroups in flight per CU)
  p->want_B = d->lines_per_group > 0 ? d->lines_per_group : 1;
  {
    std::vector<Tap> tl = wendland_tap_list(d->ndim, d->dx, d->h_over_dx, p->reach);
  }
  for (int a = 0; a < 3; ++a) {
    p->n[a] = a < p->nd ? d->n[a] : 1;
    p->walled[a] = a < p->nd ? (d->axis[a] == FCSPH_AXIS_WALLED) : 0;
    p->Efc[a] = p->n[a] + (p->walled[a] ? d->fc_C : 0);
    p->E[a] = p->Efc[a];
    if (p->window && p->walled[a]) {
      p->E[a] = window_length(p->n[a], p->reach);
      if (d->window_len[a] > 0) {
        std::vector<int> rad;
        if (d->window_len[a] < p->n[a] + 2 * p->reach || !factor_direct(d->window_len[a], rad) ||
            !line_threads(d->window_len[a], rad)) {
          msg = "window_len must be >= n + 2 R, a product of radices 2, 3, 4, 5, 7, 8, and fit 512 threads per line";
          return FCSPH_E_INVALID;
        }
        p->E[a] = d->window_len[a];
      }
    }
    if (p->E[a] <= 0) {
      msg = "no transform length for the window of axis " + std::to_string(a);
      return FCSPH_E_UNSUPPORTED;
    }
  }
  p->H = p->E[0] / 2 + 1;
  const bool f32 = p->fp32;
  const size_t ce = f32 ? sizeof(cpx<float>) : sizeof(cpx<double>);
  const size_t te = f32 ? sizeof(float) : sizeof(double);
  bool any_wall = p->walled[0] || p->walled[1] || p->walled[2];
  // FC maps
  if (any_wall) {
    const size_t mb = (size_t)d->fc_C * d->fc_d * sizeof(double);
    Upload a, b;
    a.data.assign((const char *)d->fc_M_dir, (const char *)d->fc_M_dir + mb);
    b.data.assign((const char *)d->fc_M_neu, (const char *)d->fc_M_neu + mb);
    a.dst = ws.take(mb);
    b.dst = ws.take(mb);
    p->M_dir = (const double *)a.dst;
    p->M_neu = (const double *)b.dst;
    up.push_back(std::move(a));
    up.push_back(std::move(b));
  }
  // operator line plans
  for (int a = 0; a < p->nd; ++a) {
    const int minTL = 64;
    if (!make_line_plan(p->E[a], f32, minTL, ws, up, p->op[a], false, false, d->radix_order) ||
        (f32 && !make_line_plan(p->E[a], false, minTL, ws, up, p->op64[a], false, false, d->radix_order))) {
      msg = "cannot plan a DFT of length " + std::to_string(p->E[a]);
      return FCSPH_E_UNSUPPORTED;
    }
  }
  // direct tap list
  p->direct = d->op_eval == FCSPH_OPS_DIRECT;
  {
    std::vector<Tap> tl = wendland_tap_list(p->nd, d->dx, d->h_over_dx, p->reach);
    Upload u;
    u.data.assign((const char *)tl.data(), (const char *)(tl.data() + tl.size()));
    u.dst = ws.take(u.data.size());
    p->taps = (const Tap *)u.dst;
    p->ntaps = (int)tl.size();
    double l1[3] = {0.0, 0.0, 0.0};
    for (const Tap &t : tl)
      for (int a = 0; a < 3; ++a) l1[a] += std::fabs(t.w[a]);
    p->sigma2_bound = l1[0] * l1[0] + l1[1] * l1[1] + l1[2] * l1[2];
    up.push_back(std::move(u));
    if (p->nd == 2)
      for (const Tap &t : tl) {
        const int wi = (t.s[1] + kSymR) * kSymW + (t.s[0] + kSymR);
        p->wd2[0][wi] = t.w[0];
        p->wd2[1][wi] = t.w[1];
        p->wd2[2][wi] = t.w[3];
      }
  }
  // symbols
  {
    std::vector<double> W[4];
    wendland_taps(p->nd, d->dx, d->h_over_dx, p->E, W);
    p->st.ndim = p->nd;
    for (int a = 0; a < 3; ++a) p->st.E[a] = p->E[a];
    for (int a = 0; a < p->nd; ++a) {
      Upload u;
      const int E = p->E[a];
      u.data.resize((size_t)E * (kSymR + 1) * sizeof(double2));
      double2 *t = (double2 *)u.data.data();
      for (int k = 0; k < E; ++k)
        for (int s = 0; s <= kSymR; ++s) {
          const long long q = ((long long)k * s) % E;
          const LD ang = -2.0L * kPi * (LD)q / (LD)E;
          t[(size_t)k * (kSymR + 1) + s] = make_double2((double)cosl(ang), (double)sinl(ang));
        }
      u.dst = ws.take(u.data.size());
      p->st.ph[a] = (const double2 *)u.dst;
      up.push_back(std::move(u));
    }
    if (p->nd == 2) {
      // line coefficients along y of every symbol at every x wavenumber k of
      // the half spectrum: R[sl] = sum_sx W[sl][sx] exp(-2 pi i k sx / E_x)
      // (uniform across a column's workgroup; tabulated once instead of per
      // column and pass)
      const int Ex = p->E[0], Hx = Ex / 2 + 1;
      Upload u;
      u.data.resize((size_t)4 * Hx * kSymW * sizeof(double2));
      double2 *t = (double2 *)u.data.data();
      for (int q = 0; q < 4; ++q)
        for (int k = 0; k < Hx; ++k)
          for (int sl = -kSymR; sl <= kSymR; ++sl) {
            LD re = 0.0L, im = 0.0L;
            for (int sx = -kSymR; sx <= kSymR; ++sx) {
              const LD w = (LD)W[q][(sl + kSymR) * kSymW + (sx + kSymR)];
              if (w == 0.0L) continue;
              const long long m = (((long long)k * sx) % Ex + Ex) % Ex;
              const LD ang = -2.0L * kPi * (LD)m / (LD)Ex;
              re += w * cosl(ang);
              im += w * sinl(ang);
            }
            t[((size_t)q * Hx + k) * kSymW + sl + kSymR] = make_double2((double)re, (double)im);
          }
      u.dst = ws.take(u.data.size());
      p->symR2 = (const double2 *)u.dst;
      up.push_back(std::move(u));
      if (is_gaussian(d->kernel)) {
        double s2 = 0.0;
        std::vector<double2> tab = gaussian_symbols_2d(d->kernel, d->dx, d->h_over_dx, p->E[0], p->E[1], s2);
        Upload g;
        g.data.assign((const char *)tab.data(), (const char *)(tab.data() + tab.size()));
        g.dst = ws.take(g.data.size());
        p->symF2 = (const double2 *)g.dst;
        up.push_back(std::move(g));
        p->sigma2_bound = s2;
      }
    }
    if (p->nd == 3) {
      // z lines: R[sl] = sum_{sy, sx} W[sl][sy][sx] exp(-2 pi i (k sx / E_x + o sy / E_y))
      // for k < E_x / 2 + 1 (x half spectrum) and o < E_y (y-extended rows)
      const int Ex = p->E[0], Ey = p->E[1], Hx = Ex / 2 + 1;
      auto phase = [](int k, int s, int E) {
        const long long m = (((long long)k * s) % E + E) % E;
        const LD ang = -2.0L * kPi * (LD)m / (LD)E;
        return std::make_pair(cosl(ang), sinl(ang));
      };
      std::vector<std::pair<LD, LD>> px((size_t)Hx * kSymW), py((size_t)Ey * kSymW);
      for (int k = 0; k < Hx; ++k)
        for (int sx = -kSymR; sx <= kSymR; ++sx) px[(size_t)k * kSymW + sx + kSymR] = phase(k, sx, Ex);
      for (int o = 0; o < Ey; ++o)
        for (int sy = -kSymR; sy <= kSymR; ++sy) py[(size_t)o * kSymW + sy + kSymR] = phase(o, sy, Ey);
      Upload u;
      u.data.resize((size_t)4 * Hx * Ey * kSymW * sizeof(double2));
      double2 *t = (double2 *)u.data.data();
      for (int q = 0; q < 4; ++q)
        for (int k = 0; k < Hx; ++k)
          for (int o = 0; o < Ey; ++o)
            for (int sl = -kSymR; sl <= kSymR; ++sl) {
              LD re = 0.0L, im = 0.0L;
              for (int sy = -kSymR; sy <= kSymR; ++sy)
                for (int sx = -kSymR; sx <= kSymR; ++sx) {
                  const LD w = (LD)W[q][((sl + kSymR) * kSymW + (sy + kSymR)) * kSymW + (sx + kSymR)];
                  if (w == 0.0L) continue;
                  const auto &a = px[(size_t)k * kSymW + sx + kSymR];
                  const auto &b = py[(size_t)o * kSymW + sy + kSymR];
                  re += w * (a.first * b.first - a.second * b.second);
                  im += w * (a.first * b.second + a.second * b.first);
                }
              t[(((size_t)q * Hx + k) * Ey + o) * kSymW + sl + kSymR] = make_double2((double)re, (double)im);
            }
      u.dst = ws.take(u.data.size());
      p->symR3 = (const double2 *)u.dst;
      up.push_back(std::move(u));
    }
  }
  // PPE plans and eigenvalues
  for (int a = 0; a < p->nd; ++a) {
    const int nn = p->n[a];
    int L, kind;
    if (!p->walled[a]) {
      kind = TRIG_DFT;
      L = nn;
    } else if (d->prs_bc[a][0] != d->prs_bc[a][1]) {
      kind = d->prs_bc[a][0] == FCSPH_BC_DIRICHLET ? TRIG_QWS : TRIG_QWC;
      L = 2 * (nn - 1);
    } else {
      kind = d->prs_bc[a][0] == FCSPH_BC_NEUMANN ? TRIG_DCT1 : TRIG_DST1;
      L = 2 * (nn - 1);
      // DCT-I / DST-I: one DFT of length N = n - 1 and a running sum (half
      // the transform length of the even / odd extension; at n = 1024 a
      // 2048-point instead of a 4096-point Bluestein FFT).  The PPE runs in
      // FP64 in both forms (in FP32 the running sum over N / 2 terms alone
      // would exceed the FP32 form's error target).
      if (nn >= 3) L = nn - 1;
    }
    p->trig_kind[a] = kind;
    const bool qw = kind == TRIG_QWS || kind == TRIG_QWC;
    p->ncoef[a] = kind == TRIG_DFT ? (a == 0 ? nn / 2 + 1 : nn) : (kind == TRIG_DCT1 ? nn : qw ? nn - 1 : nn - 2);
    const int minTL = 64;
    // Streamed large radices (instead of Bluestein) only while every line pair
    // of the axis fits on the chip at once (1024 SIMDs at the PPE kernels' two
    // waves each): there the pass is bound by one line's serial chain, which
    // they shorten; with more lines it is bound by throughput, and their
    // three waves per line (mostly idle for short lines) cost more than the
    // Bluestein transform's work (256^3 channel, N = 255: 617 against 291 us
    // per y pass).
    const long pairs = (long)((size_t)p->n[0] * p->n[1] * p->n[2] / nn + 1) / 2;
    // (batched plans: never; the grouped kernels carry no streamed stages)
    const bool stream = !d->batched && pairs * stream_threads(L, 0) <= 1024L * 2 * 64;
    // the narrow butterfly rule where the line fits (more waves per SIMD),
    // else the wide one (longer lines per workgroup)
    if (!make_line_plan(L, false, minTL, ws, up, p->trig[a], stream, false) &&
        !make_line_plan(L, false, minTL, ws, up, p->trig[a], stream, true)) {
      msg = "cannot plan a PPE transform of length " + std::to_string(L);
      return FCSPH_E_UNSUPPORTED;
    }
    if (p->trig[a].spare > 0) p->ppe_streamed = true;
    // eigenvalues indexed by storage position
    std::vector<double> mu(nn, 0.0);
    const LD dx = d->dx;
    for (int k = 0; k < nn; ++k) {
      LD th;   // mode angle per grid step
      if (kind == TRIG_DFT) {
        const int ks = (k <= nn / 2) ? k : k - nn;
        th = 2.0L * kPi * (LD)ks / (LD)nn;
      } else if (qw) {
        th = kPi * (LD)(2 * k + 1) / (LD)(2 * (nn - 1));   // quarter-wave mode k at position k
      } else if (kind == TRIG_DCT1 || a != 0) {
        th = kPi * (LD)k / (LD)(nn - 1);            // position = mode (lines, DCT rows)
      } else {
        th = kPi * (LD)(k + 1) / (LD)(nn - 1);      // DST-I rows: position p <-> mode p+1
      }
      LD m;
      if (d->eig == FCSPH_EIG_SPECTRAL) m = (th / dx) * (th / dx);
      else m = 4.0L / (dx * dx) * sinl(th / 2.0L) * sinl(th / 2.0L);
      mu[k] = (double)m;
    }
    Upload u;
    u.data.assign((const char *)mu.data(), (const char *)(mu.data() + mu.size()));
    u.dst = ws.take(u.data.size());
    p->mu[a] = (const double *)u.dst;
    up.push_back(std::move(u));
    if ((kind == TRIG_DCT1 || kind == TRIG_DST1) && L == nn - 1) {
      Upload q;
      const int N = nn - 1;
      std::vector<double2> t(N / 2 + 1);
      for (int j = 0; j <= N / 2; ++j) {
        const LD ang = kPi * (LD)j / (LD)N;
        t[j] = make_double2((double)cosl(ang), (double)sinl(ang));
      }
      q.data.assign((const char *)t.data(), (const char *)(t.data() + t.size()));
      q.dst = ws.take(q.data.size());
      p->dcs[a] = (const double2 *)q.dst;
      up.push_back(std::move(q));
    }
    if (qw) {
      // exp(-i pi j / 2N), j < 2N, N = n - 1
      Upload q;
      q.data.resize((size_t)L * sizeof(cpx<double>));
      for (int j = 0; j < L; ++j) {
        const LD ang = -kPi * (LD)j / (LD)L;
        put_cpx<double>(q.data, j, cosl(ang), sinl(ang));
      }
      q.dst = ws.take(q.data.size());
      p->qtw[a] = q.dst;
      up.push_back(std::move(q));
    }
  }
  // scratch
  const size_t P = (size_t)p->n[0] * p->n[1] * p->n[2];
  size_t rows = (size_t)p->n[1] * p->n[2];
  size_t rows_ext = (size_t)p->E[1] * p->n[2];     // 3D y-extended rows
  p->spec_elems = std::max(rows, rows_ext) * p->H;
  const size_t sb = p->spec_elems * ce;
  const size_t sb64 = p->spec_elems * sizeof(cpx<double>);   // also holds the FP64 divergence pass
  for (int i = 0; i < 3; ++i) p->S[i] = ws.take(sb64);
  const int nO = p->nd == 2 ? 6 : 12;
  for (int i = 0; i < nO; ++i) p->O[i] = ws.take(i < 3 ? sb64 : sb);
  if (p->nd == 3)
    for (int i = 0; i < 3; ++i) p->Y[i] = ws.take(sb64);
  for (int a = 0; a < p->nd; ++a) p->ustar[a] = (double *)ws.take(P * sizeof(double));
  p->rhs = ws.take(P * te);
  p->phi = (double *)ws.take(P * sizeof(double));
  p->counter = (unsigned long long *)ws.take(256);
  p->cpitch = p->trig_kind[0] == TRIG_DFT ? p->ncoef[0] : (std::max(p->ncoef[0], 1) + 1) / 2;
  p->coef = ws.take((size_t)p->cpitch * rows * sizeof(cpx<double>));   // PPE coefficients: FP64
  p->ext_scratch = (double *)ws.take((size_t)p->Efc[0] * p->Efc[1] * p->Efc[2] * sizeof(double));
  if (p->fp32 && p->walled[1])
    for (int i = 0; i < 3; ++i)
      p->edge[i] = ws.take((size_t)2 * p->n[2] * d->fc_d * p->H * sizeof(double2));
  for (int i = 0; i < 3; ++i) {
    p->ghx[i] = (double *)ws.take((size_t)p->n[1] * p->n[2] * 2 * kSymR * sizeof(double));
    p->ghy[i] = (double *)ws.take((size_t)2 * kSymR * (p->n[0] + 2 * kSymR) * p->n[2] * sizeof(double));
  }
  p->ws_bytes = ws.off + 256;
  return FCSPH_OK;
}

// ----------------------------------------------------------------- pipelines
// Runs the operator passes of its scope in FP64 on an FP32-mixed plan (the
// divergence of u* that forms the PPE right-hand side: the solenoidal part of
// u* cancels in it, so FP32 transforms would round relative to |G u| instead
// of |div u*|).  The plan's FP64 twin line plans and FP64-sized scratch
// spectra make this possible; outside the scope the plan is unchanged.
struct Fp64Passes {
  fcsph_plan *p;
  bool was;
  explicit Fp64Passes(fcsph_plan *pl) : p(pl), was(pl->fp32) {
    if (was) {
      for (int a = 0; a < 3; ++a) std::swap(p->op[a], p->op64[a]);
      p->fp32 = false;
    }
  }
  ~Fp64Passes() {
    if (was) {
      for (int a = 0; a < 3; ++a) std::swap(p->op[a], p->op64[a]);
      p->fp32 = true;
    }
  }
};

bool chk(fcsph_plan *p, hipError_t e, const char *where, fcsph_status &st) {
  if (e != hipSuccess) {
    st = hip_fail(p->ctx, e, where);
    return false;
  }
  return true;
}

// x-pass forward over the rows of a physical field f; rows (2l, 2l+1) packed.
hipError_t x_fwd_single(fcsph_plan *p, const double *f, int fc, void *S) {
  RowsFwdArgs a{};
  a.plan = p->op[0];
  const int rows = p->n[1] * p->n[2];
  a.nlines = (rows + 1) / 2;
  a.nx = p->n[0];
  a.E = p->E[0];
  a.H = p->H;
  a.fc = walls_for(p, 0, fc);
  a.inA = f;
  a.inB = f + p->n[0];
  a.strideA = a.strideB = 2L * p->n[0];
  a.nB = rows / 2;
  a.outA = S;
  a.outB = (char *)S + (size_t)p->H * (p->fp32 ? sizeof(cpx<float>) : sizeof(cpx<double>));
  a.ostrideA = a.ostrideB = 2L * p->H;
  a.B = pick_B(a.plan, p->fp32, p->want_B);
  a.ldsM = padded_len(a.plan.M, a.plan.pad);
  LaunchTimer t(p->ctx, "rows_fwd");
  return launch_rows_fwd(a, p->fp32, p->ctx->stream);
}

// x-pass forward of two fields with the same wall maps, packed row by row.
// edge0 / edge1 (FP32 2D plans): the FP64 boundary-row spectra of f0 / f1
// (the column pass's FC_y inputs) come out of the same launch.
hipError_t x_fwd_pair(fcsph_plan *p, const double *f0, const double *f1, int fc, void *S0, void *S1,
                      void *edge0 = nullptr, void *edge1 = nullptr) {
  RowsFwdArgs a{};
  a.plan = p->op[0];
  const int rows = p->n[1] * p->n[2];
  a.nlines = rows;
  a.nx = p->n[0];
  a.E = p->E[0];
  a.H = p->H;
  a.fc = walls_for(p, 0, fc);
  a.inA = f0;
  a.inB = f1;
  a.strideA = a.strideB = p->n[0];
  a.nB = rows;
  a.outA = S0;
  a.outB = S1;
  a.ostrideA = a.ostrideB = p->H;
  a.B = pick_B(a.plan, p->fp32, p->want_B);
  a.ldsM = padded_len(a.plan.M, a.plan.pad);
  if (edge0) {
    a.edge_rows = p->d.fc_d;
    a.ny = p->n[1];
    a.plan64 = p->op64[0];
    a.edgeA = edge0;
    a.edgeB = edge1;
  }
  LaunchTimer t(p->ctx, "rows_fwd_pair");
  return launch_rows_fwd(a, p->fp32, p->ctx->stream);
}

// 2D strided y pass with symbol multiplication.
ColsArgs cols_base(fcsph_plan *p, int mode, int fc) {
  ColsArgs c{};
  c.plan = p->op[1];
  c.mode = mode;
  c.ninner = p->H;
  c.nouter = 1;
  c.es = p->H;
  c.es_out = p->H;
  c.os_in = c.os_out = 0;
  c.nload = p->n[1];
  c.nstore = p->n[1];
  c.fc = walls_for(p, 1, fc);
  c.st = p->st;
  c.line_axis = 1;
  c.inner_axis = 0;
  c.outer_axis = -1;
  c.symR = p->symR2;
  c.symF = p->symF2;
  c.B = pick_B(c.plan, p->fp32, p->want_B, cols_lines_per_column(mode));
  c.ldsM = padded_len(c.plan.M, c.plan.pad);
  return c;
}

hipError_t cols_launch(fcsph_plan *p, const ColsArgs &c, int gy, const char *name) {
  LaunchTimer t(p->ctx, name);
  return launch_cols(c, gy, p->fp32, p->ctx->stream);
}

// FP32 plans: FP64 x spectra of the fc_d first and fc_d last rows of every
// z plane of a field (FC_x fused as in the x pass), the FP64 inputs of FC_y.
// 2D: the boundary rows of both walls of one field f (g null: packed in row
// pairs) or of two fields f, g (one row of each per line) in one launch;
// logical rows d .. 2d-1 map to the high wall's rows n_y - d .. n_y - 1 and
// land after the low wall's in the edge arrays.
hipError_t edge_fwd_2d(fcsph_plan *p, const double *f, const double *g, int fc, void *edge_f, void *edge_g) {
  const int d = p->d.fc_d;
  RowsFwdArgs a{};
  a.plan = p->op64[0];
  a.nlines = g ? 2 * d : d;
  a.nx = p->n[0];
  a.E = p->E[0];
  a.H = p->H;
  a.fc = walls_for(p, 0, fc);
  a.inA = f;
  a.inB = g;
  a.nB = a.nlines;
  a.map_per = d;
  a.map_plane = (long)(p->n[1] - d) * p->n[0];
  a.outA = edge_f;
  a.outB = g ? edge_g : (void *)((double2 *)edge_f + p->H);
  a.ostrideA = a.ostrideB = g ? (long)p->H : 2L * p->H;
  a.B = pick_B(a.plan, false, p->want_B);
  a.ldsM = padded_len(a.plan.M, a.plan.pad);
  LaunchTimer t(p->ctx, "rows_fwd_edge");
  return launch_rows_fwd(a, false, p->ctx->stream);
}

hipError_t edge_fwd(fcsph_plan *p, const double *f, int fc, void *edge) {
  const int d = p->d.fc_d, nz = p->n[2], rows = nz * d;
  if (nz == 1) return edge_fwd_2d(p, f, nullptr, fc, edge, nullptr);
  for (int h = 0; h < 2; ++h) {
    RowsFwdArgs a{};
    a.plan = p->op64[0];
    a.nlines = (rows + 1) / 2;
    a.nx = p->n[0];
    a.E = p->E[0];
    a.H = p->H;
    a.fc = walls_for(p, 0, fc);
    a.inA = f + (h ? (size_t)(p->n[1] - d) * p->n[0] : 0);
    a.nB = rows / 2;
    a.map_per = d;
    a.map_plane = (long)p->n[1] * p->n[0];
    a.outA = (double2 *)edge + (size_t)h * rows * p->H;
    a.outB = (double2 *)a.outA + p->H;
    a.ostrideA = a.ostrideB = 2L * p->H;
    a.B = pick_B(a.plan, false, p->want_B);
    a.ldsM = padded_len(a.plan.M, a.plan.pad);
    LaunchTimer t(p->ctx, "rows_fwd_edge");
    hipError_t e = launch_rows_fwd(a, false, p->ctx->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Attach FP64 boundary rows of nf fields to a strided pass that applies FC
// along y (FP32 plans only; FP64 plans read the line's own values).
hipError_t set_edges(fcsph_plan *p, ColsArgs &c, int nf, const double *const *fields, int fc) {
  for (int f = 0; f < 3; ++f) c.edge[f] = nullptr;
  if (!p->fp32 || !p->edge[0] || !c.fc.on || c.line_axis != 1) return hipSuccess;
  if (p->n[2] == 1 && nf == 2) {
    hipError_t e = edge_fwd_2d(p, fields[0], fields[1], fc, p->edge[0], p->edge[1]);
    if (e != hipSuccess) return e;
    c.edge[0] = (const double2 *)p->edge[0];
    c.edge[1] = (const double2 *)p->edge[1];
    return hipSuccess;
  }
  for (int f = 0; f < nf; ++f) {
    hipError_t e = edge_fwd(p, fields[f], fc, p->edge[f]);
    if (e != hipSuccess) return e;
    c.edge[f] = (const double2 *)p->edge[f];
  }
  return hipSuccess;
}

hipError_t x_inv_store(fcsph_plan *p, const void *spec0, const void *spec1, void *out0, void *out1,
                       bool out_double, double scale) {
  RowsInvArgs a{};
  a.plan = p->op[0];
  a.nrows = p->n[1] * p->n[2];
  a.nx = p->n[0];
  a.E = p->E[0];
  a.H = p->H;
  a.B = pick_B(a.plan, p->fp32, p->want_B);
  a.ldsM = padded_len(a.plan.M, a.plan.pad);
  a.spec[0] = spec0;
  a.spec[1] = spec1;
  a.spec_pitch = p->H;
  a.rpp = p->n[1];
  a.prow = p->nd == 3 ? p->E[1] : p->n[1];
  a.out[0] = out0;
  a.out[1] = out1;
  a.out_is_double = out_double ? 1 : 0;
  a.scale = scale;
  LaunchTimer t(p->ctx, "rows_inv_store");
  return launch_rows_inv(a, EPI_STORE, p->fp32, p->ctx->stream);
}

WallInfo wall_info(fcsph_plan *p) {
  WallInfo w{};
  w.ndim = p->nd;
  for (int a = 0; a < 3; ++a) {
    w.n[a] = p->n[a];
    w.walled[a] = p->walled[a];
    for (int s = 0; s < 2; ++s) w.dir[a][s] = p->walled[a] && p->d.vel_bc[a][s] == FCSPH_BC_DIRICHLET;
  }
  return w;
}

// ---- 3D (walls in y; x, z periodic): strided passes along y and z.
// Spectrum arrays: x half spectra [nz][rows][H] with rows = ny (compact) or
// E_y (y-extended, also used for the y-restricted results in place).
ColsArgs y_pass_args(fcsph_plan *p, int mode, int fc) {
  ColsArgs c{};
  c.plan = p->op[1];
  c.mode = mode;
  c.ninner = p->H;
  c.nouter = p->n[2];
  c.es = p->H;
  c.es_out = p->H;
  if (mode == COLS_FWD) {
    c.os_in = (long)p->n[1] * p->H;
    c.nload = p->n[1];
    c.nstore = p->E[1];
  } else {
    c.os_in = (long)p->E[1] * p->H;
    c.nload = p->E[1];
    c.nstore = p->n[1];
  }
  c.os_out = (long)p->E[1] * p->H;
  c.fc = walls_for(p, 1, fc);
  c.st = p->st;
  c.line_axis = 1;
  c.inner_axis = 0;
  c.outer_axis = 2;
  c.B = pick_B(c.plan, p->fp32, p->want_B, cols_lines_per_column(mode));
  c.ldsM = padded_len(c.plan.M, c.plan.pad);
  return c;
}

ColsArgs z_pass_args(fcsph_plan *p, int mode) {
  ColsArgs c{};
  c.plan = p->op[2];
  c.mode = mode;
  c.ninner = p->H;
  c.nouter = p->E[1];
  c.es = (long)p->E[1] * p->H;
  c.es_out = c.es;
  c.os_in = c.os_out = p->H;
  c.nload = c.nstore = p->n[2];
  c.fc = walls_for(p, 2, FCSPH_FIELD_VELOCITY);   // z is periodic: off
  c.st = p->st;
  c.line_axis = 2;
  c.inner_axis = 0;
  c.outer_axis = 1;
  c.symR = p->symR3;
  c.B = pick_B(c.plan, p->fp32, p->want_B, cols_lines_per_column(mode));
  c.ldsM = padded_len(c.plan.M, c.plan.pad);
  return c;
}

// y forward of nf spectra (FC along y with the field class's walls)
hipError_t y_fwd(fcsph_plan *p, int nf, void *const *in, void *const *out, int fc, const double *const *fields) {
  if (nf < 1 || nf > 3) return hipErrorInvalidValue;
  ColsArgs c = y_pass_args(p, COLS_FWD, fc);
  hipError_t e = set_edges(p, c, nf, fields, fc);
  if (e != hipSuccess) return e;
  for (int f = 0; f < nf; ++f) {
    c.in[f] = in[f];
    c.out[f][0] = out[f];
  }
  static const char *names[4] = {"cols_y_fwd", "cols_y_fwd1", "cols_y_fwd2", "cols_y_fwd3"};
  return cols_launch(p, c, nf, names[nf < 4 ? nf : 0]);
}

// y inverse of nf spectra in place (y-extended layout), restricted to ny rows
hipError_t y_inv(fcsph_plan *p, int nf, void *const *buf) {
  if (nf < 1 || nf > 3) return hipErrorInvalidValue;
  ColsArgs c = y_pass_args(p, COLS_INV, FCSPH_FIELD_VELOCITY);
  for (int f = 0; f < nf; ++f) {
    c.in[f] = buf[f];
    c.out[f][0] = buf[f];
  }
  static const char *names[4] = {"cols_y_inv", "cols_y_inv1", "cols_y_inv2", "cols_y_inv3"};
  return cols_launch(p, c, nf, names[nf < 4 ? nf : 0]);
}

DirectArgs direct_base(fcsph_plan *p, int fc) {
  DirectArgs a{};
  a.ndim = p->nd;
  for (int q = 0; q < 3; ++q) {
    a.n[q] = p->n[q];
    a.walled[q] = p->walled[q];
    a.fc[q] = walls_for(p, q, fc);
  }
  a.R = p->reach;
  a.taps = p->taps;
  a.ntaps = p->ntaps;
  for (int q = 0; q < 3; ++q)
    for (int i = 0; i < kSymW * kSymW; ++i) a.wd[q][i] = p->wd2[q][i];
  for (int q = 0; q < 3; ++q) {
    a.gx[q] = p->ghx[q];
    a.gy[q] = p->ghy[q];
  }
  a.out_is_double = p->fp32 ? 0 : 1;
  a.scale = 1.0;
  a.wi = wall_info(p);
  return a;
}

hipError_t direct_launch(fcsph_plan *p, const DirectArgs &a, int mode, const char *name) {
  const int nf = (mode == DIR_DIV || mode == DIR_STEP_A) ? 2 : 1;
  {
    LaunchTimer t(p->ctx, "direct_ghost");
    hipError_t e = launch_ghost2d(a, nf, p->ctx->stream);
    if (e != hipSuccess) return e;
  }
  LaunchTimer t(p->ctx, name);
  return launch_direct(a, mode, p->ctx->stream);
}

// 3D PPE (x, z periodic; y walled): DFT_x rows, then along y (forward),
// along z (forward, FP64 divide, inverse, all inverse scales), along y
// (inverse), and the inverse x DFT.
fcsph_status run_ppe3(fcsph_plan *p, const void *rhs, double *phi) {
  fcsph_status st = FCSPH_OK;
  // the PPE transforms run in FP64 in both forms; an FP32 plan's right-hand
  // side is read as float
  const bool f32 = false, rhs32 = p->fp32;
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
  PpeRowsArgs r{};
  r.plan = p->trig[0];
  r.kind = p->trig_kind[0];
  r.inverse = 0;
  r.nrows = ny * nz;
  r.nx = nx;
  r.ncoef = p->ncoef[0];
  r.cpitch = p->cpitch;
  r.in_real = rhs32 ? nullptr : (const double *)rhs;
  r.in_float = rhs32 ? (const float *)rhs : nullptr;
  r.coef = p->coef;
  r.qtw = p->qtw[0];
  r.dcs = p->dcs[0];
  r.B = pick_B(r.plan, f32, p->want_B, 1, ppe_line_len(p, 0));
  r.ldsM = padded_len(ppe_line_len(p, 0), r.plan.pad);
  {
    LaunchTimer t(p->ctx, "ppe_rows_fwd");
    if (!chk(p, launch_ppe_rows(r, f32, p->ctx->stream), "ppe rows", st)) return st;
  }
  PpeColsArgs cy{};
  cy.plan = p->trig[1];
  cy.kind = p->trig_kind[1];
  cy.ninner = p->cpitch;
  cy.nouter = nz;
  cy.es = p->cpitch;
  cy.os = (long)ny * p->cpitch;
  cy.nline = ny;
  cy.ncoef = p->ncoef[1];
  cy.data = p->coef;
  cy.qtw = p->qtw[1];
  cy.dcs = p->dcs[1];
  cy.B = pick_B(cy.plan, f32, p->want_B, 1, ppe_line_len(p, 1));
  cy.ldsM = padded_len(ppe_line_len(p, 1), cy.plan.pad);
  cy.solve = 0;
  {
    LaunchTimer t(p->ctx, "ppe_cols_y_fwd");
    if (!chk(p, launch_ppe_cols(cy, f32, p->ctx->stream), "ppe y", st)) return st;
  }
  PpeColsArgs cz{};
  cz.plan = p->trig[2];
  cz.kind = p->trig_kind[2];
  cz.ninner = p->cpitch;
  cz.nouter = ny;
  cz.es = (long)ny * p->cpitch;
  cz.os = p->cpitch;
  cz.nline = nz;
  cz.ncoef = p->ncoef[2];
  cz.solve = 1;
  cz.mu_line = p->mu[2];
  cz.mu_inner = p->mu[0];
  cz.inner_packed = 0;
  cz.inner_nmodes = p->ncoef[0];
  cz.mu_outer = p->mu[1];
  const double sy = p->trig_kind[1] == TRIG_DFT ? 1.0 / ny : 1.0 / (2.0 * (ny - 1));
  cz.scale = sy / nz;
  cz.data = p->coef;
  cz.qtw = p->qtw[2];
  cz.dcs = p->dcs[2];
  cz.B = pick_B(cz.plan, f32, p->want_B, 1, ppe_line_len(p, 2));
  cz.ldsM = padded_len(ppe_line_len(p, 2), cz.plan.pad);
  {
    LaunchTimer t(p->ctx, "ppe_cols_z_solve");
    if (!chk(p, launch_ppe_cols(cz, f32, p->ctx->stream), "ppe z", st)) return st;
  }
  cy.solve = 2;
  {
    LaunchTimer t(p->ctx, "ppe_cols_y_inv");
    if (!chk(p, launch_ppe_cols(cy, f32, p->ctx->stream), "ppe y inv", st)) return st;
  }
  r.inverse = 1;
  r.in_real = nullptr;
  r.in_float = nullptr;
  r.out = phi;
  r.scale = 1.0 / nx;
  {
    LaunchTimer t(p->ctx, "ppe_rows_inv");
    if (!chk(p, launch_ppe_rows(r, f32, p->ctx->stream), "ppe rows inverse", st)) return st;
  }
  return FCSPH_OK;
}

// spec non-null (2D): the right-hand side is not stored; the rows forward
// pass forms it from the divergence's x half spectrum spec (FP64), times
// spec_scale, rounded to FP32 when round32 (as the store of an FP32 plan).
// spec_out non-null (2D): the rows inverse pass also writes the x half spectra
// of phi (pressure maps, FP64) to spec_out, the first pass of the projection.
fcsph_status run_ppe(fcsph_plan *p, const void *rhs, double *phi, const void *spec = nullptr,
                     double spec_scale = 0.0, bool round32 = false, void *spec_out = nullptr) {
  fcsph_status st = FCSPH_OK;
  for (int a = 0; a < p->nd; ++a)
    if (p->trig_kind[a] < 0)
      return fail(p->ctx, FCSPH_E_UNSUPPORTED, "mixed Dirichlet/Neumann pressure walls on one axis are not built");
  if (p->nd == 3) return run_ppe3(p, rhs, phi);
  const bool f32 = false, rhs32 = p->fp32;   // FP64 transforms; FP32 plans pass a float rhs
  // P1: rows forward
  PpeRowsArgs r{};
  r.plan = p->trig[0];
  r.kind = p->trig_kind[0];
  r.inverse = 0;
  r.nrows = p->n[1];
  r.nx = p->n[0];
  r.ncoef = p->ncoef[0];
  r.cpitch = p->cpitch;
  r.in_real = rhs32 ? nullptr : (const double *)rhs;
  r.in_float = rhs32 ? (const float *)rhs : nullptr;
  r.coef = p->coef;
  r.qtw = p->qtw[0];
  r.dcs = p->dcs[0];
  r.B = pick_B(r.plan, f32, p->want_B, 1, ppe_line_len(p, 0));
  r.ldsM = padded_len(ppe_line_len(p, 0), r.plan.pad);
  PpeRowsArgs rf = r;
  if (spec) {
    // one line group runs both transforms: the larger thread count and line
    rf.spec = spec;
    rf.spec_pitch = p->H;
    rf.xplan = p->fp32 ? p->op64[0] : p->op[0];
    rf.xE = p->E[0];
    rf.xH = p->H;
    rf.in_scale = spec_scale;
    rf.round32 = round32 ? 1 : 0;
    rf.in_real = nullptr;
    rf.in_float = nullptr;
    rf.plan.TL = std::max(r.plan.TL, rf.xplan.TL);
    const int len = std::max(ppe_line_len(p, 0), rf.xplan.M);
    rf.B = pick_B(rf.plan, f32, p->want_B, 1, len);
    rf.ldsM = padded_len(len, r.plan.pad);
  }
  {
    LaunchTimer t(p->ctx, "ppe_rows_fwd");
    if (!chk(p, launch_ppe_rows(rf, f32, p->ctx->stream), "ppe rows", st)) return st;
  }
  // P2: columns forward, divide, inverse
  PpeColsArgs c{};
  c.plan = p->trig[1];
  c.kind = p->trig_kind[1];
  c.ninner = p->cpitch;
  c.nouter = 1;
  c.es = p->cpitch;
  c.os = 0;
  c.nline = p->n[1];
  c.ncoef = p->ncoef[1];
  c.solve = 1;
  c.mu_line = p->mu[1];
  c.mu_inner = p->mu[0];
  c.inner_packed = p->trig_kind[0] != TRIG_DFT;
  c.inner_nmodes = p->ncoef[0];
  c.mu_outer = nullptr;
  c.scale = p->trig_kind[1] == TRIG_DFT ? 1.0 / p->n[1] : 1.0 / (2.0 * (p->n[1] - 1));
  c.data = p->coef;
  c.qtw = p->qtw[1];
  c.dcs = p->dcs[1];
  c.B = pick_B(c.plan, f32, p->want_B, 1, ppe_line_len(p, 1));
  c.ldsM = padded_len(ppe_line_len(p, 1), c.plan.pad);
  if (p->d.eig == FCSPH_EIG_SPH) {
    // every axis periodic: the PPE's DFT wavenumbers are those of the symbol
    // tables (E = n), whose weights carry 1 / (E_x E_y)
    c.sph = 1;
    c.symR = p->symR2;
    c.sym_ninner = p->H;
    c.ph_line = p->st.ph[1];
    c.sph_norm = (double)p->E[0] * (double)p->E[1];
    c.mu_tol = 1e-14 * p->sigma2_bound;
  }
  {
    LaunchTimer t(p->ctx, "ppe_cols_solve");
    if (!chk(p, launch_ppe_cols(c, f32, p->ctx->stream), "ppe cols", st)) return st;
  }
  // P3: rows inverse
  r.inverse = 1;
  r.in_real = nullptr;
  r.in_float = nullptr;
  r.out = phi;
  r.scale = p->trig_kind[0] == TRIG_DFT ? 1.0 / p->n[0] : 1.0 / (2.0 * (p->n[0] - 1));
  if (spec_out) {
    r.spec_out = spec_out;
    r.spec_pitch = p->H;
    r.xplan = p->fp32 ? p->op64[0] : p->op[0];
    r.xE = p->E[0];
    r.xH = p->H;
    r.xfc = walls_for(p, 0, FCSPH_FIELD_PRESSURE);
    r.plan.TL = std::max(r.plan.TL, r.xplan.TL);
    const int len = std::max(ppe_line_len(p, 0), r.xplan.M);
    r.B = pick_B(r.plan, f32, p->want_B, 1, len);
    r.ldsM = padded_len(len, r.plan.pad);
  }
  {
    LaunchTimer t(p->ctx, "ppe_rows_inv");
    if (!chk(p, launch_ppe_rows(r, f32, p->ctx->stream), "ppe rows inverse", st)) return st;
  }
  return FCSPH_OK;
}

// Scratch of one Laplacian evaluation: x spectra (S), y-extended spectra (Y,
// 3D), output spectra (O), the FP64 boundary rows of FP32 plans (edge) and
// the ghost values of the direct tap sums (gx, gy).
struct LapBufs {
  void *S, *Y, *O, *edge;
  double *gx, *gy;
};

// Carve the buffers of one Laplacian evaluation out of a bump region (the
// static scratch of the no-allocation entry point); dry run with a null base.
void lap_scratch_layout(const fcsph_plan *p, Bump &ws, LapBufs &b) {
  const size_t sb64 = p->spec_elems * sizeof(cpx<double>);
  b.S = ws.take(sb64);
  b.O = ws.take(sb64);
  b.Y = p->nd == 3 ? ws.take(sb64) : nullptr;
  b.edge = (p->fp32 && p->walled[1] && p->nd == 2)
               ? ws.take((size_t)2 * p->n[2] * p->d.fc_d * p->H * sizeof(double2))
               : nullptr;
  if (p->direct) {
    b.gx = (double *)ws.take((size_t)p->n[1] * p->n[2] * 2 * kSymR * sizeof(double));
    b.gy = (double *)ws.take((size_t)2 * kSymR * (p->n[0] + 2 * kSymR) * p->n[2] * sizeof(double));
  } else {
    b.gx = b.gy = nullptr;
  }
}

size_t lap_scratch_bytes(const fcsph_plan *p) {
  Bump dry;
  LapBufs b{};
  lap_scratch_layout(p, dry, b);
  return dry.off;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char *fcsph_status_string(fcsph_status s) {
  switch (s) {
    case FCSPH_OK: return "ok";
    case FCSPH_E_INVALID: return "invalid argument";
    case FCSPH_E_UNSUPPORTED: return "unsupported";
    case FCSPH_E_WORKSPACE: return "workspace too small or misaligned";
    case FCSPH_E_HIP: return "HIP error";
    case FCSPH_E_NONFINITE: return "non-finite values";
  }
  return "unknown status";
}

fcsph_status fcsph_ctx_create(int device, void *hip_stream, fcsph_ctx **out) {
  if (!out) return FCSPH_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FCSPH_E_INVALID;
  fcsph_ctx *c = new (std::nothrow) fcsph_ctx;
  if (!c) return FCSPH_E_INVALID;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return FCSPH_E_HIP;
  }
  register_scratch(device);
  *out = c;
  return FCSPH_OK;
}

fcsph_status fcsph_ctx_destroy(fcsph_ctx *c) {
  if (!c) return FCSPH_OK;
  for (auto &l : c->launches) {
    hipEventDestroy(l.start);
    hipEventDestroy(l.stop);
  }
  for (auto e : c->event_pool) hipEventDestroy(e);
  delete c;
  return FCSPH_OK;
}

fcsph_status fcsph_ctx_sync(fcsph_ctx *c) {
  if (!c) return FCSPH_E_INVALID;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "device");
  return FCSPH_OK;
}

const char *fcsph_ctx_last_error(fcsph_ctx *c) { return c ? c->last_error.c_str() : "null context"; }

fcsph_status fcsph_ctx_set_timing(fcsph_ctx *c, int enable) {
  if (!c) return FCSPH_E_INVALID;
  c->timing = enable != 0;
  return FCSPH_OK;
}

fcsph_status fcsph_ctx_set_timing_only(fcsph_ctx *c, const char *name) {
  if (!c) return FCSPH_E_INVALID;
  if (name && std::strlen(name) > 31) return fail(c, FCSPH_E_INVALID, "timer name longer than 31 characters");
  c->timing_only = name ? name : "";
  return FCSPH_OK;
}

fcsph_status fcsph_ctx_read_timing(fcsph_ctx *c, int cap, char *names, int *counts, double *total_ms,
                                   int *n) {
  if (!c || !n || cap < 0 || (cap > 0 && (!names || !counts || !total_ms))) return FCSPH_E_INVALID;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
  std::vector<std::string> kinds;
  std::vector<int> cnt;
  std::vector<double> tot;
  for (auto &l : c->launches) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, l.start, l.stop);
    size_t k = 0;
    while (k < kinds.size() && kinds[k] != l.name) ++k;
    if (k == kinds.size()) {
      kinds.push_back(l.name);
      cnt.push_back(0);
      tot.push_back(0.0);
    }
    cnt[k] += 1;
    tot[k] += ms;
    c->event_pool.push_back(l.start);
    c->event_pool.push_back(l.stop);
  }
  c->launches.clear();
  int w = 0;
  for (size_t k = 0; k < kinds.size() && w < cap; ++k, ++w) {
    std::snprintf(names + 32 * w, 32, "%s", kinds[k].c_str());
    counts[w] = cnt[k];
    total_ms[w] = tot[k];
  }
  *n = w;
  return FCSPH_OK;
}

fcsph_status fcsph_plan_workspace_bytes(const fcsph_desc *d, size_t *bytes) {
  if (!bytes) return FCSPH_E_INVALID;
  std::string msg;
  fcsph_status s = validate(d, msg);
  if (s != FCSPH_OK) return s;
  fcsph_plan tmp;
  Bump ws;
  std::vector<Upload> up;
  s = layout(&tmp, d, ws, up, msg);
  if (s != FCSPH_OK) return s;
  *bytes = tmp.ws_bytes;
  return FCSPH_OK;
}

fcsph_status fcsph_plan_create(fcsph_ctx *c, const fcsph_desc *d, void *workspace, size_t bytes,
                               fcsph_plan **out) {
  if (!c || !out) return FCSPH_E_INVALID;
  *out = nullptr;
  std::string msg;
  fcsph_status s = validate(d, msg);
  if (s != FCSPH_OK) return fail(c, s, msg);
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(c, FCSPH_E_WORKSPACE, "workspace null or not 256-byte aligned");
  fcsph_plan *p = new (std::nothrow) fcsph_plan;
  if (!p) return fail(c, FCSPH_E_INVALID, "out of host memory");
  p->ctx = c;
  Bump ws;
  ws.base = (char *)workspace;
  std::vector<Upload> up;
  s = layout(p, d, ws, up, msg);
  if (s != FCSPH_OK) {
    delete p;
    return fail(c, s, msg);
  }
  if (p->ws_bytes > bytes) {
    delete p;
    return fail(c, FCSPH_E_WORKSPACE, "workspace too small: need " + std::to_string(ws.off + 256));
  }
  for (auto &u : up) {
    hipError_t e = hipMemcpyAsync(u.dst, u.data.data(), u.data.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(c, e, "table upload");
    }
  }
  // host staging buffers are pageable: finish the copies before they go away
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(c, e, "table upload sync");
  }
  *out = p;
  return FCSPH_OK;
}

fcsph_status fcsph_plan_destroy(fcsph_plan *p) {
  delete p;
  return FCSPH_OK;
}

fcsph_status fcsph_plan_transform_lengths(const fcsph_plan *p, int L[3]) {
  if (!p || !L) return FCSPH_E_INVALID;
  for (int a = 0; a < 3; ++a) L[a] = p->E[a];
  return FCSPH_OK;
}

fcsph_status fcsph_fc_extend(fcsph_plan *p, int fc, const double *f, double *f_ext) {
  if (!p || !f || !f_ext) return p ? fail(p->ctx, FCSPH_E_INVALID, "null pointer") : FCSPH_E_INVALID;
  if (fc != FCSPH_FIELD_VELOCITY && fc != FCSPH_FIELD_PRESSURE) return fail(p->ctx, FCSPH_E_INVALID, "bad field class");
  fcsph_status st = FCSPH_OK;
  int shape[3] = {p->n[0], p->n[1], p->n[2]};
  int nw = 0, last = -1;
  for (int a = 0; a < p->nd; ++a)
    if (p->walled[a]) { ++nw; last = a; }
  if (nw == 0) {
    size_t P = (size_t)shape[0] * shape[1] * shape[2];
    if (!chk(p, hipMemcpyAsync(f_ext, f, P * sizeof(double), hipMemcpyDeviceToDevice, p->ctx->stream), "copy", st)) return st;
    return FCSPH_OK;
  }
  // apply the walled axes in order x, y, z; with two walled axes the first
  // result goes to the plan's extension scratch
  if (nw > 2) return fail(p->ctx, FCSPH_E_UNSUPPORTED, "more than two walled axes");
  const double *src = f;
  for (int a = 0; a < p->nd; ++a) {
    if (!p->walled[a]) continue;
    double *dst = (a == last) ? f_ext : p->ext_scratch;
    FcWalls w = walls_for(p, a, fc);
    LaunchTimer t(p->ctx, "fc_extend");
    if (!chk(p, launch_fc_extend_axis(src, dst, p->nd, shape, a, w, p->ctx->stream), "fc_extend", st)) return st;
    shape[a] += p->d.fc_C;
    src = dst;
  }
  return FCSPH_OK;
}

fcsph_status fcsph_spectral_grad(fcsph_plan *p, int fc, const double *f, void *const *g) {
  if (!p) return FCSPH_E_INVALID;
  if (!f || !g) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  for (int a = 0; a < p->nd; ++a)
    if (!g[a]) return fail(p->ctx, FCSPH_E_INVALID, "null output");
  fcsph_status st = FCSPH_OK;
  if (p->nd == 3) {
    if (!chk(p, x_fwd_single(p, f, fc, p->S[0]), "grad x", st)) return st;
    if (!chk(p, y_fwd(p, 1, &p->S[0], &p->Y[0], fc, &f), "grad y", st)) return st;
    ColsArgs c = z_pass_args(p, COLS_OP);
    c.in[0] = p->Y[0];
    for (int q = 0; q < 3; ++q) {
      c.out[0][q] = p->O[q];
      c.sym[q] = q;
    }
    c.nout = 3;
    if (!chk(p, cols_launch(p, c, 1, "cols_z_op"), "grad z", st)) return st;
    if (!chk(p, y_inv(p, 3, &p->O[0]), "grad y inv", st)) return st;
    if (!chk(p, x_inv_store(p, p->O[0], p->O[1], g[0], g[1], !p->fp32, 1.0), "grad x inv", st)) return st;
    if (!chk(p, x_inv_store(p, p->O[2], nullptr, g[2], nullptr, !p->fp32, 1.0), "grad x inv", st)) return st;
    return FCSPH_OK;
  }
  if (p->direct) {
    DirectArgs a = direct_base(p, fc);
    a.in[0] = f;
    a.out[0] = g[0];
    a.out[1] = g[1];
    if (!chk(p, direct_launch(p, a, DIR_OPS, "direct_ops"), "grad", st)) return st;
    return FCSPH_OK;
  }
  if (!chk(p, x_fwd_single(p, f, fc, p->S[0]), "grad x", st)) return st;
  ColsArgs c = cols_base(p, COLS_OP, fc);
  if (!chk(p, set_edges(p, c, 1, &f, fc), "grad edges", st)) return st;
  c.in[0] = p->S[0];
  c.out[0][0] = p->O[0];
  c.out[0][1] = p->O[1];
  c.nout = 2;
  c.sym[0] = SYM_GX;
  c.sym[1] = SYM_GY;
  if (!chk(p, cols_launch(p, c, 1, "cols_op"), "grad y", st)) return st;
  if (!chk(p, x_inv_store(p, p->O[0], p->O[1], g[0], g[1], !p->fp32, 1.0), "grad x inv", st)) return st;
  return FCSPH_OK;
}

static fcsph_status lap_impl(fcsph_plan *p, int fc, const double *f, void *lap, const LapBufs &b) {
  fcsph_status st = FCSPH_OK;
  if (p->nd == 3) {
    if (!chk(p, x_fwd_single(p, f, fc, b.S), "lap x", st)) return st;
    void *Sv = b.S, *Yv = b.Y, *Ov = b.O;
    if (!chk(p, y_fwd(p, 1, &Sv, &Yv, fc, &f), "lap y", st)) return st;
    ColsArgs c = z_pass_args(p, COLS_OP);
    c.in[0] = b.Y;
    c.out[0][0] = b.O;
    c.sym[0] = SYM_LAP;
    c.nout = 1;
    if (!chk(p, cols_launch(p, c, 1, "cols_z_op"), "lap z", st)) return st;
    if (!chk(p, y_inv(p, 1, &Ov), "lap y inv", st)) return st;
    if (!chk(p, x_inv_store(p, b.O, nullptr, lap, nullptr, !p->fp32, 1.0), "lap x inv", st)) return st;
    return FCSPH_OK;
  }
  if (p->direct) {
    DirectArgs a = direct_base(p, fc);
    a.gx[0] = b.gx;
    a.gy[0] = b.gy;
    a.in[0] = f;
    a.out[3] = lap;
    if (!chk(p, direct_launch(p, a, DIR_OPS, "direct_ops"), "lap", st)) return st;
    return FCSPH_OK;
  }
  if (!chk(p, x_fwd_single(p, f, fc, b.S), "lap x", st)) return st;
  ColsArgs c = cols_base(p, COLS_OP, fc);
  if (p->fp32 && b.edge && c.fc.on) {
    if (!chk(p, edge_fwd(p, f, fc, b.edge), "lap edges", st)) return st;
    c.edge[0] = (const double2 *)b.edge;
  }
  c.in[0] = b.S;
  c.out[0][0] = b.O;
  c.nout = 1;
  c.sym[0] = SYM_LAP;
  if (!chk(p, cols_launch(p, c, 1, "cols_op"), "lap y", st)) return st;
  if (!chk(p, x_inv_store(p, b.O, nullptr, lap, nullptr, !p->fp32, 1.0), "lap x inv", st)) return st;
  return FCSPH_OK;
}

fcsph_status fcsph_spectral_lap(fcsph_plan *p, int fc, const double *f, void *lap) {
  if (!p) return FCSPH_E_INVALID;
  if (!f || !lap) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  if (fc != FCSPH_FIELD_VELOCITY && fc != FCSPH_FIELD_PRESSURE) return fail(p->ctx, FCSPH_E_INVALID, "bad field class");
  return lap_impl(p, fc, f, lap, LapBufs{p->S[0], p->Y[0], p->O[0], p->edge[0], p->ghx[0], p->ghy[0]});
}

fcsph_status fcsph_spectral_lap_noalloc(fcsph_plan *p, int fc, const double *f, void *lap) {
  if (!p) return FCSPH_E_INVALID;
  if (!f || !lap) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  if (fc != FCSPH_FIELD_VELOCITY && fc != FCSPH_FIELD_PRESSURE) return fail(p->ctx, FCSPH_E_INVALID, "bad field class");
  const size_t need = lap_scratch_bytes(p);
  if (need > kStaticScratchBytes)
    return fail(p->ctx, FCSPH_E_UNSUPPORTED,
                "lattice too large for the static scratch: needs " + std::to_string(need) + " bytes, the maximum is " +
                    std::to_string(kStaticScratchBytes));
  hipError_t e = hipSuccess;
  char *base = static_cast<char *>(scratch_of(p->ctx->device, &e));
  if (!base) return hip_fail(p->ctx, e, "static scratch address");
  Bump bb;
  bb.base = base;
  LapBufs b{};
  lap_scratch_layout(p, bb, b);
  return lap_impl(p, fc, f, lap, b);
}

static fcsph_status div3_impl(fcsph_plan *p, const double *const *u, void *out, bool out_double, double scale) {
  fcsph_status st = FCSPH_OK;
  if (!chk(p, x_fwd_pair(p, u[0], u[1], FCSPH_FIELD_VELOCITY, p->S[0], p->S[1]), "div x", st)) return st;
  if (!chk(p, x_fwd_single(p, u[2], FCSPH_FIELD_VELOCITY, p->S[2]), "div x", st)) return st;
  if (!chk(p, y_fwd(p, 3, &p->S[0], &p->Y[0], FCSPH_FIELD_VELOCITY, u), "div y", st)) return st;
  ColsArgs c = z_pass_args(p, COLS_DIV);
  for (int f = 0; f < 3; ++f) {
    c.in[f] = p->Y[f];
    c.sym[f] = f;
  }
  c.out[0][0] = p->O[0];
  c.nout = 1;
  if (!chk(p, cols_launch(p, c, 1, "cols_z_div"), "div z", st)) return st;
  if (!chk(p, y_inv(p, 1, &p->O[0]), "div y inv", st)) return st;
  if (!chk(p, x_inv_store(p, p->O[0], nullptr, out, nullptr, out_double, scale), "div x inv", st)) return st;
  return FCSPH_OK;
}

// spectra_ready: the x forward pass of (u0, u1) into S[0], S[1] was done by
// the pass that produced them (the fused u* epilogue of a step)
// store = false: stop before the last pass (the x inverse into out), whose
// input spectrum p->O[0] the caller hands to the PPE's fused row pass.
static fcsph_status div_impl(fcsph_plan *p, const double *u0, const double *u1, void *out, bool out_double,
                             double scale, bool spectra_ready = false, bool store = true) {
  fcsph_status st = FCSPH_OK;
  if (p->direct) {
    DirectArgs a = direct_base(p, FCSPH_FIELD_VELOCITY);
    a.in[0] = u0;
    a.in[1] = u1;
    a.out[0] = out;
    a.out_is_double = out_double ? 1 : 0;
    a.scale = scale;
    if (!chk(p, direct_launch(p, a, DIR_DIV, "direct_div"), "div", st)) return st;
    return FCSPH_OK;
  }
  if (!spectra_ready)
    if (!chk(p, x_fwd_pair(p, u0, u1, FCSPH_FIELD_VELOCITY, p->S[0], p->S[1]), "div x", st)) return st;
  ColsArgs c = cols_base(p, COLS_DIV, FCSPH_FIELD_VELOCITY);
  {
    const double *uu[2] = {u0, u1};
    if (!chk(p, set_edges(p, c, 2, uu, FCSPH_FIELD_VELOCITY), "div edges", st)) return st;
  }
  c.in[0] = p->S[0];
  c.in[1] = p->S[1];
  c.out[0][0] = p->O[0];
  c.nout = 1;
  c.sym[0] = SYM_GX;
  c.sym[1] = SYM_GY;
  if (!chk(p, cols_launch(p, c, 1, "cols_div"), "div y", st)) return st;
  if (!store) return FCSPH_OK;
  if (!chk(p, x_inv_store(p, p->O[0], nullptr, out, nullptr, out_double, scale), "div x inv", st)) return st;
  return FCSPH_OK;
}

fcsph_status fcsph_spectral_div(fcsph_plan *p, const double *const *u, void *div) {
  if (!p) return FCSPH_E_INVALID;
  if (!u || !div) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  for (int a = 0; a < p->nd; ++a)
    if (!u[a]) return fail(p->ctx, FCSPH_E_INVALID, "null input");
  if (p->nd == 3) return div3_impl(p, u, div, !p->fp32, 1.0);
  return div_impl(p, u[0], u[1], div, !p->fp32, 1.0);
}

fcsph_status fcsph_check_finite(fcsph_plan *p, const double *x, size_t n, unsigned long long *count) {
  if (!p) return FCSPH_E_INVALID;
  if ((!x && n) || !count) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  fcsph_status st = FCSPH_OK;
  if (!chk(p, launch_count_nonfinite(x, n, p->counter, p->ctx->stream), "finiteness count", st)) return st;
  unsigned long long c = 0;
  if (!chk(p, hipMemcpyAsync(&c, p->counter, sizeof(c), hipMemcpyDeviceToHost, p->ctx->stream), "copy count", st))
    return st;
  if (!chk(p, hipStreamSynchronize(p->ctx->stream), "finiteness sync", st)) return st;
  *count = c;
  if (c) return fail(p->ctx, FCSPH_E_NONFINITE, std::to_string(c) + " non-finite values");
  return FCSPH_OK;
}

fcsph_status fcsph_ppe_solve(fcsph_plan *p, const void *rhs, double *phi) {
  if (!p) return FCSPH_E_INVALID;
  if (!rhs || !phi) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  return run_ppe(p, rhs, phi);
}

// EXTENDED PPE domain: the projection of u* on the extended periodic lattice
// (its alternative to the physical-domain PPE in the section integrating FC
// into the spectral ISPH solver): e_a = DFT(FC(u*_a)), phi_hat =
// (rho/dt) sum_a S_a e_a / sum_a S_a^2 (zero where the sum vanishes),
// u_a <- restriction of IDFT(e_a - (dt/rho) S_a phi_hat), Dirichlet walls
// reset; p_out <- restriction of IDFT(phi_hat).
static fcsph_status project_extended(fcsph_plan *p, double *const *u, double *p_out,
                                     const double *const *wall_vel, double dt_proj, bool spectra_ready = false) {
  fcsph_status st = FCSPH_OK;
  hipStream_t s = p->ctx->stream;
  double *phi = p_out ? p_out : p->phi;
  double norm = 1.0;
  for (int a = 0; a < p->nd; ++a) norm *= (double)p->E[a];
  ColsArgs c = p->nd == 2 ? cols_base(p, COLS_PROJ, FCSPH_FIELD_VELOCITY) : z_pass_args(p, COLS_PROJ);
  c.B = 1;
  c.proj_dtr = dt_proj / p->d.rho;
  c.proj_tol = 1e-14 * p->sigma2_bound / (norm * norm);
  c.proj_inv_norm = 1.0 / norm;
  c.nout = p->nd + 1;
  for (int q = 0; q < p->nd; ++q) c.sym[q] = q;     // SYM_GX, SYM_GY, SYM_GZ
  RowsInvArgs r{};
  r.plan = p->op[0];
  r.nrows = p->n[1] * p->n[2];
  r.nx = p->n[0];
  r.E = p->E[0];
  r.H = p->H;
  r.B = 1;
  r.ldsM = padded_len(r.plan.M, r.plan.pad);
  r.spec_pitch = p->H;
  r.rpp = p->n[1];
  r.prow = p->nd == 3 ? p->E[1] : p->n[1];
  for (int q = 0; q < p->nd; ++q) {
    r.wall[q] = wall_vel ? wall_vel[q] : nullptr;
    r.unew[q] = u[q];
  }
  r.assign = 1;
  r.wi = wall_info(p);
  if (p->nd == 2) {
    if (!spectra_ready &&
        !chk(p, x_fwd_pair(p, p->ustar[0], p->ustar[1], FCSPH_FIELD_VELOCITY, p->S[0], p->S[1]), "proj x", st))
      return st;
    c.in[0] = p->S[0];
    c.in[1] = p->S[1];
    for (int q = 0; q < 3; ++q) c.out[0][q] = p->O[q];
    if (!chk(p, cols_launch(p, c, 1, "cols_proj"), "proj y", st)) return st;
    r.spec[0] = p->O[0];
    r.spec[1] = p->O[1];
    {
      LaunchTimer t(p->ctx, "rows_inv_proj");
      if (!chk(p, launch_rows_inv(r, EPI_STEP_D2, false, s), "proj x inv", st)) return st;
    }
    if (!chk(p, x_inv_store(p, p->O[2], nullptr, phi, nullptr, true, 1.0), "proj phi x inv", st)) return st;
    return FCSPH_OK;
  }
  if (!chk(p, x_fwd_pair(p, p->ustar[0], p->ustar[1], FCSPH_FIELD_VELOCITY, p->S[0], p->S[1]), "proj3 x", st))
    return st;
  if (!chk(p, x_fwd_single(p, p->ustar[2], FCSPH_FIELD_VELOCITY, p->S[2]), "proj3 x", st)) return st;
  {
    const double *us[3] = {p->ustar[0], p->ustar[1], p->ustar[2]};
    if (!chk(p, y_fwd(p, 3, &p->S[0], &p->Y[0], FCSPH_FIELD_VELOCITY, us), "proj3 y", st)) return st;
  }
  for (int q = 0; q < 3; ++q) c.in[q] = p->Y[q];
  for (int q = 0; q < 4; ++q) c.out[0][q] = p->O[q];
  if (!chk(p, cols_launch(p, c, 1, "cols_z_proj"), "proj3 z", st)) return st;
  // y inverse of the four outputs (a strided pass takes at most three fields)
  if (!chk(p, y_inv(p, 3, &p->O[0]), "proj3 y inv", st)) return st;
  if (!chk(p, y_inv(p, 1, &p->O[3]), "proj3 y inv", st)) return st;
  r.spec[0] = p->O[0];
  r.spec[1] = p->O[1];
  r.spec[2] = p->O[2];
  {
    LaunchTimer t(p->ctx, "rows_inv_proj3");
    if (!chk(p, launch_rows_inv(r, EPI_STEP_D3, false, s), "proj3 x inv", st)) return st;
  }
  if (!chk(p, x_inv_store(p, p->O[3], nullptr, phi, nullptr, true, 1.0), "proj3 phi x inv", st)) return st;
  return FCSPH_OK;
}

// One projection step or RK3 sub-step.  u* uses dt and the RK terms; the
// PPE right-hand side is (rho / dt_proj) div u* and the correction
// u* - (dt_proj / rho) grad phi (eqs. PPE and u^n+1 with dt_proj = a_k dt;
// the first-order form has dt_proj = dt).
static fcsph_status step_impl(fcsph_plan *p, double *const *u, double *p_out, const double *const *force,
                              const double *const *wall_vel, double dt, double nu, double dt_proj,
                              const RkTerms &rk) {
  if (!p) return FCSPH_E_INVALID;
  if (!u) return fail(p->ctx, FCSPH_E_INVALID, "null velocity");
  for (int a = 0; a < p->nd; ++a)
    if (!u[a]) return fail(p->ctx, FCSPH_E_INVALID, "null velocity component");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(nu >= 0.0) || !std::isfinite(nu))
    return fail(p->ctx, FCSPH_E_INVALID, "dt must be positive and nu non-negative");
  if (rk.on && p->d.ppe_domain == FCSPH_PPE_EXTENDED)
    return fail(p->ctx, FCSPH_E_UNSUPPORTED, "RK3 sub-steps are built for the physical-domain PPE");
  fcsph_status st = FCSPH_OK;
  hipStream_t s = p->ctx->stream;
  const bool f32 = p->fp32;
  if (p->nd == 3) {
    // A: 12 derivatives of (u, v, w), fused u*
    if (!chk(p, x_fwd_pair(p, u[0], u[1], FCSPH_FIELD_VELOCITY, p->S[0], p->S[1]), "step3 A x", st)) return st;
    if (!chk(p, x_fwd_single(p, u[2], FCSPH_FIELD_VELOCITY, p->S[2]), "step3 A x", st)) return st;
    if (!chk(p, y_fwd(p, 3, &p->S[0], &p->Y[0], FCSPH_FIELD_VELOCITY, u), "step3 A y", st)) return st;
    ColsArgs c = z_pass_args(p, COLS_OP);
    for (int f = 0; f < 3; ++f) {
      c.in[f] = p->Y[f];
      for (int q = 0; q < 4; ++q) c.out[f][q] = p->O[4 * f + q];
    }
    c.nout = 4;
    c.sym[0] = SYM_GX;
    c.sym[1] = SYM_GY;
    c.sym[2] = SYM_GZ;
    c.sym[3] = SYM_LAP;
    if (!chk(p, cols_launch(p, c, 3, "cols_z_op_step_a"), "step3 A z", st)) return st;
    for (int g = 0; g < 4; ++g)
      if (!chk(p, y_inv(p, 3, &p->O[3 * g]), "step3 A y inv", st)) return st;
    RowsInvArgs r{};
    r.plan = p->op[0];
    r.nrows = p->n[1] * p->n[2];
    r.nx = p->n[0];
    r.E = p->E[0];
    r.H = p->H;
    r.B = 1;
    r.ldsM = padded_len(r.plan.M, r.plan.pad);
    // rows of at most 4 line-group widths: one line group takes the six lines
    // in turn, paired (Gx, Gy), (Gz, L) per component; otherwise the lines
    // are spread over the workgroup's line groups
    const bool seq = r.nx <= 4 * r.plan.TL;
    const int order_seq[12] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
    const int order_par[12] = {0, 1, 2, 4, 5, 6, 8, 9, 10, 3, 7, 11};
    for (int k = 0; k < 12; ++k) r.spec[k] = p->O[seq ? order_seq[k] : order_par[k]];
    r.spec_pitch = p->H;
    r.rpp = p->n[1];
    r.prow = p->E[1];
    for (int q = 0; q < 3; ++q) {
      r.u[q] = u[q];
      r.f[q] = force ? force[q] : nullptr;
      r.wall[q] = wall_vel ? wall_vel[q] : nullptr;
      r.ustar[q] = p->ustar[q];
      r.unew[q] = u[q];
    }
    r.dt = dt;
    r.rk = rk;
    r.nu = nu;
    r.dt_over_rho = dt_proj / p->d.rho;
    r.wi = wall_info(p);
    {
      LaunchTimer t(p->ctx, "rows_inv_step_a3");
      if (!chk(p, launch_rows_inv(r, seq ? EPI_STEP_A3S : EPI_STEP_A3, f32, s), "step3 A x inv", st)) return st;
    }
    if (p->d.ppe_domain == FCSPH_PPE_EXTENDED) return project_extended(p, u, p_out, wall_vel, dt_proj);
    // B (FP64 transforms in both forms), C
    {
      Fp64Passes g64(p);
      st = div3_impl(p, p->ustar, p->rhs, !f32, p->d.rho / dt_proj);
    }
    if (st != FCSPH_OK) return st;
    double *phi = p_out ? p_out : p->phi;
    st = run_ppe(p, p->rhs, phi);
    if (st != FCSPH_OK) return st;
    // D (FP64 transforms in both forms, as in 2D)
    Fp64Passes g64(p);
    const bool fd = p->fp32;
    if (!chk(p, x_fwd_single(p, phi, FCSPH_FIELD_PRESSURE, p->S[0]), "step3 D x", st)) return st;
    if (!chk(p, y_fwd(p, 1, &p->S[0], &p->Y[0], FCSPH_FIELD_PRESSURE, &phi), "step3 D y", st)) return st;
    ColsArgs cd = z_pass_args(p, COLS_OP);
    cd.in[0] = p->Y[0];
    for (int q = 0; q < 3; ++q) {
      cd.out[0][q] = p->O[q];
      cd.sym[q] = q;
    }
    cd.nout = 3;
    if (!chk(p, cols_launch(p, cd, 1, "cols_z_op_step_d"), "step3 D z", st)) return st;
    if (!chk(p, y_inv(p, 3, &p->O[0]), "step3 D y inv", st)) return st;
    RowsInvArgs rd = r;
    rd.plan = p->op[0];
    rd.ldsM = padded_len(rd.plan.M, rd.plan.pad);
    rd.spec[0] = p->O[0];
    rd.spec[1] = p->O[1];
    rd.spec[2] = p->O[2];
    {
      LaunchTimer t(p->ctx, "rows_inv_step_d3");
      if (!chk(p, launch_rows_inv(rd, EPI_STEP_D3, fd, s), "step3 D x inv", st)) return st;
    }
    return FCSPH_OK;
  }
  if (p->direct) {
    DirectArgs a = direct_base(p, FCSPH_FIELD_VELOCITY);
    a.in[0] = u[0];
    a.in[1] = u[1];
    for (int q = 0; q < 2; ++q) {
      a.f[q] = force ? force[q] : nullptr;
      a.wall[q] = wall_vel ? wall_vel[q] : nullptr;
      a.ustar[q] = p->ustar[q];
    }
    a.dt = dt;
    a.rk = rk;
    a.nu = nu;
    a.dt_over_rho = dt_proj / p->d.rho;
    if (!chk(p, direct_launch(p, a, DIR_STEP_A, "direct_step_a"), "step A", st)) return st;
    st = div_impl(p, p->ustar[0], p->ustar[1], p->rhs, !f32, p->d.rho / dt_proj);
    if (st != FCSPH_OK) return st;
    double *phi = p_out ? p_out : p->phi;
    st = run_ppe(p, p->rhs, phi);
    if (st != FCSPH_OK) return st;
    DirectArgs b = direct_base(p, FCSPH_FIELD_PRESSURE);
    b.in[0] = phi;
    for (int q = 0; q < 2; ++q) {
      b.wall[q] = wall_vel ? wall_vel[q] : nullptr;
      b.ustar_in[q] = p->ustar[q];
      b.unew[q] = u[q];
    }
    b.dt_over_rho = dt_proj / p->d.rho;
    if (!chk(p, direct_launch(p, b, DIR_STEP_D, "direct_step_d"), "step D", st)) return st;
    return FCSPH_OK;
  }
  // A: u* = u - dt [(u.grad)u - nu lap u - f], Dirichlet walls <- wall data
  ColsArgs c = cols_base(p, COLS_OP, FCSPH_FIELD_VELOCITY);
  // FP32 plans: the FP64 boundary-row spectra (FC_y inputs) come out of the
  // x pass itself
  const bool edges_fused = p->fp32 && p->edge[0] && c.fc.on && c.line_axis == 1 && p->n[2] == 1;
  if (!chk(p, x_fwd_pair(p, u[0], u[1], FCSPH_FIELD_VELOCITY, p->S[0], p->S[1],
                         edges_fused ? p->edge[0] : nullptr, edges_fused ? p->edge[1] : nullptr),
           "step A x", st))
    return st;
  if (edges_fused) {
    c.edge[0] = (const double2 *)p->edge[0];
    c.edge[1] = (const double2 *)p->edge[1];
    c.edge[2] = nullptr;
  } else if (!chk(p, set_edges(p, c, 2, u, FCSPH_FIELD_VELOCITY), "step A edges", st)) {
    return st;
  }
  c.in[0] = p->S[0];
  c.in[1] = p->S[1];
  c.out[0][0] = p->O[0];
  c.out[0][1] = p->O[1];
  c.out[0][2] = p->O[2];
  c.out[1][0] = p->O[3];
  c.out[1][1] = p->O[4];
  c.out[1][2] = p->O[5];
  c.nout = 3;
  c.sym[0] = SYM_GX;
  c.sym[1] = SYM_GY;
  c.sym[2] = SYM_LAP;
  if (!chk(p, cols_launch(p, c, 2, "cols_op_step_a"), "step A y", st)) return st;
  RowsInvArgs r{};
  r.plan = p->op[0];
  r.nrows = p->n[1];
  r.nx = p->n[0];
  r.E = p->E[0];
  r.H = p->H;
  r.B = 1;
  r.ldsM = padded_len(r.plan.M, r.plan.pad);
  r.spec[0] = p->O[0];
  r.spec[1] = p->O[1];
  r.spec[2] = p->O[3];
  r.spec[3] = p->O[4];
  r.spec[4] = p->O[2];
  r.spec[5] = p->O[5];
  r.spec_pitch = p->H;
  r.rpp = p->n[1];
  r.prow = p->n[1];
  r.u[0] = u[0];
  r.u[1] = u[1];
  r.f[0] = force ? force[0] : nullptr;
  r.f[1] = force ? force[1] : nullptr;
  r.wall[0] = wall_vel ? wall_vel[0] : nullptr;
  r.wall[1] = wall_vel ? wall_vel[1] : nullptr;
  r.ustar[0] = p->ustar[0];
  r.ustar[1] = p->ustar[1];
  r.dt = dt;
  r.rk = rk;
  r.nu = nu;
  r.dt_over_rho = dt_proj / p->d.rho;
  r.wi = wall_info(p);
  if ((size_t)r.ldsM * 16 + 16ull * r.nx > (size_t)kMaxLds)
    return fail(p->ctx, FCSPH_E_UNSUPPORTED, "x line too long for the fused step kernel");
  // the epilogue also runs the FP64 x forward pass of (u*, v*) that the
  // divergence (or the EXTENDED projection) starts with (FP32 plans: with
  // the FP64 plan of the same length)
  const bool fused = true;
  r.fwd_fused = 1;
  r.fwd_fc = walls_for(p, 0, FCSPH_FIELD_VELOCITY);
  r.fwd_out[0] = p->S[0];
  r.fwd_out[1] = p->S[1];
  r.plan64 = f32 ? p->op64[0] : p->op[0];
  {
    LaunchTimer t(p->ctx, "rows_inv_step_a");
    if (!chk(p, launch_rows_inv(r, EPI_STEP_A2, f32, s), "step A x inv", st)) return st;
  }
  if (p->d.ppe_domain == FCSPH_PPE_EXTENDED) return project_extended(p, u, p_out, wall_vel, dt_proj, fused);
  // B: b = (rho/dt) div u*, FP64 transforms in both forms
  // (2D: the divergence stops at its x spectrum, which the PPE's row pass
  // transforms back itself; b is never stored)
  const bool fuse_rhs = p->nd == 2;
  {
    Fp64Passes g64(p);
    st = div_impl(p, p->ustar[0], p->ustar[1], p->rhs, !f32, p->d.rho / dt_proj, fused, !fuse_rhs);
  }
  if (st != FCSPH_OK) return st;
  // C: PPE
  double *phi = p_out ? p_out : p->phi;
  // (2D, likewise: the rows inverse pass also writes phi's x spectra for D)
  st = fuse_rhs ? run_ppe(p, nullptr, phi, p->O[0], p->d.rho / dt_proj, f32, p->S[0]) : run_ppe(p, p->rhs, phi);
  if (st != FCSPH_OK) return st;
  // D: u = u* - dt/rho grad phi, walls reset; FP64 transforms in both forms
  // (the projection cancels the irrotational part of u*, so FP32 rounding
  // relative to |grad phi| would dominate the result)
  Fp64Passes g64(p);
  const bool fd = p->fp32;
  if (!fuse_rhs)
    if (!chk(p, x_fwd_single(p, phi, FCSPH_FIELD_PRESSURE, p->S[0]), "step D x", st)) return st;
  ColsArgs cd = cols_base(p, COLS_OP, FCSPH_FIELD_PRESSURE);
  {
    const double *ph = phi;
    if (!chk(p, set_edges(p, cd, 1, &ph, FCSPH_FIELD_PRESSURE), "step D edges", st)) return st;
  }
  cd.in[0] = p->S[0];
  cd.out[0][0] = p->O[0];
  cd.out[0][1] = p->O[1];
  cd.nout = 2;
  cd.sym[0] = SYM_GX;
  cd.sym[1] = SYM_GY;
  if (!chk(p, cols_launch(p, cd, 1, "cols_op_step_d"), "step D y", st)) return st;
  RowsInvArgs rd = r;
  rd.plan = p->op[0];
  rd.ldsM = padded_len(rd.plan.M, rd.plan.pad);
  rd.spec[0] = p->O[0];
  rd.spec[1] = p->O[1];
  rd.B = pick_B(rd.plan, fd, p->want_B);
  rd.unew[0] = u[0];
  rd.unew[1] = u[1];
  {
    LaunchTimer t(p->ctx, "rows_inv_step_d");
    if (!chk(p, launch_rows_inv(rd, EPI_STEP_D2, fd, s), "step D x inv", st)) return st;
  }
  return FCSPH_OK;
}

fcsph_status fcsph_project_step(fcsph_plan *p, double *const *u, double *p_out, const double *const *force,
                                const double *const *wall_vel, double dt, double nu) {
  RkTerms rk{};
  return step_impl(p, u, p_out, force, wall_vel, dt, nu, dt, rk);
}

fcsph_status fcsph_advect_rk3_substep(fcsph_plan *p, int k, double *u, double *F_store, const double *c, double dt,
                                      const double *inflow) {
  if (!p) return FCSPH_E_INVALID;
  if (!u || !F_store || !c) return fail(p->ctx, FCSPH_E_INVALID, "null pointer");
  if (k < 0 || k > 2) return fail(p->ctx, FCSPH_E_INVALID, "RK3 sub-step index must be 0, 1 or 2");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p->ctx, FCSPH_E_INVALID, "dt must be positive");
  if (p->nd != 2 || p->direct || p->fp32)
    return fail(p->ctx, FCSPH_E_UNSUPPORTED, "linear advection is built for FP64 2D plans on the FFT routes");
  static const double kg[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
  static const double kz[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
  fcsph_status st = FCSPH_OK;
  if (!chk(p, x_fwd_single(p, u, kFieldScalar, p->S[0]), "advect x", st)) return st;
  ColsArgs cc = cols_base(p, COLS_OP, kFieldScalar);
  if (!chk(p, set_edges(p, cc, 1, (const double *const *)&u, kFieldScalar), "advect edges", st)) return st;
  cc.in[0] = p->S[0];
  cc.out[0][0] = p->O[0];
  cc.out[0][1] = p->O[1];
  cc.nout = 2;
  cc.sym[0] = SYM_GX;
  cc.sym[1] = SYM_GY;
  if (!chk(p, cols_launch(p, cc, 1, "cols_op_advect"), "advect y", st)) return st;
  RowsInvArgs r{};
  r.plan = p->op[0];
  r.nrows = p->n[1];
  r.nx = p->n[0];
  r.E = p->E[0];
  r.H = p->H;
  r.B = pick_B(r.plan, p->fp32, p->want_B);
  r.ldsM = padded_len(r.plan.M, r.plan.pad);
  r.spec[0] = p->O[0];
  r.spec[1] = p->O[1];
  r.spec_pitch = p->H;
  r.rpp = p->n[1];
  r.prow = p->n[1];
  r.u[0] = u;
  r.unew[0] = u;
  r.wall[0] = inflow;
  r.dt = dt;
  r.rk.on = 1;
  r.rk.g = kg[k];
  r.rk.z = kz[k];
  r.rk.F[0] = F_store;
  r.adv_c[0] = c[0];
  r.adv_c[1] = c[1];
  // inflow walls (C . n < 0) take the caller's data; outflow walls are free
  r.wi = wall_info(p);
  for (int a = 0; a < 2; ++a) {
    r.wi.dir[a][0] = p->walled[a] && c[a] > 0.0;
    r.wi.dir[a][1] = p->walled[a] && c[a] < 0.0;
  }
  LaunchTimer t(p->ctx, "rows_inv_advect");
  if (!chk(p, launch_rows_inv(r, EPI_ADVECT2, p->fp32, p->ctx->stream), "advect x inv", st)) return st;
  return FCSPH_OK;
}

fcsph_status fcsph_rk3_substep(fcsph_plan *p, int k, double *const *u, double *p_out, const double *const *force,
                               const double *const *wall_vel, double *const *F_store, double dt, double nu) {
  if (!p) return FCSPH_E_INVALID;
  if (k < 0 || k > 2) return fail(p->ctx, FCSPH_E_INVALID, "RK3 sub-step index must be 0, 1 or 2");
  if (!F_store) return fail(p->ctx, FCSPH_E_INVALID, "null RK3 F store");
  for (int c = 0; c < p->nd; ++c)
    if (!F_store[c]) return fail(p->ctx, FCSPH_E_INVALID, "null RK3 F store component");
  // low-storage RK3 coefficients (temporal discretisation section)
  static const double ka[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  static const double kg[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
  static const double kz[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
  RkTerms rk{};
  rk.on = 1;
  rk.g = kg[k];
  rk.z = kz[k];
  rk.a = ka[k];
  for (int c = 0; c < p->nd; ++c) rk.F[c] = F_store[c];
  return step_impl(p, u, p_out, force, wall_vel, dt, nu, ka[k] * dt, rk);
}

}  // extern "C"

// ===================================================================== batches
// A batch runs the projection steps / PPE solves of many plans with grouped
// launches: each item's launch sequence is recorded (not issued), items whose
// sequences have the same kernels and launch shapes form a group, and every
// launch of a group is issued once with gridDim.z = group size, each
// workgroup reading its item's argument struct from the batch workspace.
// Groups run on their own streams (fork / join around the batch stream) so
// groups of different shapes overlap on the device.
namespace {
constexpr int kBatchStreams = 8;
enum { BATCH_STEP = 0, BATCH_PPE = 1 };
}  // namespace

struct fcsph_batch {
  fcsph_ctx *ctx = nullptr;
  int max_items = 0;
  unsigned char *dev = nullptr;      // workspace (argument arrays)
  size_t dev_bytes = 0;
  unsigned char *host = nullptr;     // pinned staging of the argument arrays
  size_t host_bytes = 0;
  hipEvent_t upload_done = nullptr;
  hipStream_t stream = nullptr;      // the batch's own stream (capturable)
  hipStream_t gs[kBatchStreams] = {};
  hipEvent_t fork = nullptr, join[kBatchStreams] = {}, done = nullptr;
  struct Item {
    fcsph_plan *p;
    int kind;
    Recorder rec;
  };
  std::vector<Item> items;
  struct Issue {
    const void *gfunc;
    dim3 grid, block;
    size_t lds;
    const void *args;                // device pointer of the group's argument array
    int stream;                      // group stream index
  };
  std::vector<Issue> issues;         // launch list of the last batch_launch
  int nstreams_used = 0;
  int ngroups = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
fcsph_status batch_fail(fcsph_batch *b, fcsph_status s, const std::string &m) { return fail(b->ctx, s, m); }

hipError_t batch_issue_all(fcsph_batch *b, hipStream_t s) {
  // fork: every used group stream waits for the batch stream
  hipError_t e = hipEventRecord(b->fork, s);
  if (e != hipSuccess) return e;
  for (int k = 0; k < b->nstreams_used; ++k)
    if ((e = hipStreamWaitEvent(b->gs[k], b->fork, 0)) != hipSuccess) return e;
  for (const fcsph_batch::Issue &is : b->issues) {
    void *arg = const_cast<void *>(is.args);
    void *params[1] = {&arg};
    e = hipLaunchKernel(is.gfunc, is.grid, is.block, params, is.lds, b->gs[is.stream]);
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < b->nstreams_used; ++k) {
    if ((e = hipEventRecord(b->join[k], b->gs[k])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, b->join[k], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

void batch_drop_graph(fcsph_batch *b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}
}  // namespace

extern "C" {

// Per item: at most kBatchMaxLaunches launches of at most kBatchMaxArgs bytes,
// plus the 256-byte alignment of each group's array.
constexpr int kBatchMaxLaunches = 64;
constexpr size_t kBatchMaxArgs = 2048;
static_assert(sizeof(RowsFwdArgs) <= kBatchMaxArgs && sizeof(RowsInvArgs) <= kBatchMaxArgs &&
                  sizeof(ColsArgs) <= kBatchMaxArgs && sizeof(PpeRowsArgs) <= kBatchMaxArgs &&
                  sizeof(PpeColsArgs) <= kBatchMaxArgs && sizeof(DirectArgs) <= kBatchMaxArgs,
              "kernel argument struct larger than the batch slot");

fcsph_status fcsph_batch_workspace_bytes(int max_items, size_t *bytes) {
  if (max_items < 1 || !bytes) return FCSPH_E_INVALID;
  *bytes = (size_t)max_items * kBatchMaxLaunches * (kBatchMaxArgs + 256);
  return FCSPH_OK;
}

fcsph_status fcsph_batch_create(fcsph_ctx *c, int max_items, void *workspace, size_t bytes, fcsph_batch **out) {
  if (!c || !out || max_items < 1 || !workspace) return c ? fail(c, FCSPH_E_INVALID, "bad batch arguments") : FCSPH_E_INVALID;
  *out = nullptr;
  size_t need = 0;
  fcsph_batch_workspace_bytes(max_items, &need);
  if (bytes < need || ((uintptr_t)workspace & 255)) return fail(c, FCSPH_E_WORKSPACE, "batch workspace too small or misaligned");
  fcsph_batch *b = new (std::nothrow) fcsph_batch;
  if (!b) return FCSPH_E_INVALID;
  b->ctx = c;
  b->max_items = max_items;
  b->dev = (unsigned char *)workspace;
  b->dev_bytes = bytes;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  for (int k = 0; k < kBatchStreams && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&b->gs[k], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming);
  for (int k = 0; k < kBatchStreams && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
  if (e == hipSuccess) {
    b->host_bytes = bytes;
    e = hipHostMalloc((void **)&b->host, bytes, hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    fcsph_batch_destroy(b);
    return hip_fail(c, e, "batch create");
  }
  *out = b;
  return FCSPH_OK;
}

fcsph_status fcsph_batch_destroy(fcsph_batch *b) {
  if (!b) return FCSPH_OK;
  if (b->stream) hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  for (int k = 0; k < kBatchStreams; ++k) {
    if (b->gs[k]) hipStreamDestroy(b->gs[k]);
    if (b->join[k]) hipEventDestroy(b->join[k]);
  }
  if (b->fork) hipEventDestroy(b->fork);
  if (b->done) hipEventDestroy(b->done);
  if (b->upload_done) {
    hipEventSynchronize(b->upload_done);
    hipEventDestroy(b->upload_done);
  }
  if (b->stream) hipStreamDestroy(b->stream);
  if (b->host) hipHostFree(b->host);
  delete b;
  return FCSPH_OK;
}

fcsph_status fcsph_batch_clear(fcsph_batch *b) {
  if (!b) return FCSPH_E_INVALID;
  b->items.clear();
  return FCSPH_OK;
}

static fcsph_status batch_add(fcsph_batch *b, fcsph_plan *p, int kind) {
  if ((int)b->items.size() >= b->max_items) return batch_fail(b, FCSPH_E_INVALID, "batch is full");
  if (p->ppe_streamed)
    return batch_fail(b, FCSPH_E_UNSUPPORTED,
                      "the plan's PPE uses streamed radix stages (single launches only): create it with batched = 1");
  for (const fcsph_batch::Item &it : b->items)
    if (it.p == p) return batch_fail(b, FCSPH_E_INVALID, "a plan may appear once per batch (its scratch is shared)");
  b->items.push_back({p, kind, Recorder{}});
  return FCSPH_OK;
}

fcsph_status fcsph_batch_add_step(fcsph_batch *b, fcsph_plan *p, double *const *u, double *p_out,
                                  const double *const *force, const double *const *wall_vel, double dt,
                                  double nu) {
  if (!b || !p) return b ? batch_fail(b, FCSPH_E_INVALID, "null plan") : FCSPH_E_INVALID;
  fcsph_status st = batch_add(b, p, BATCH_STEP);
  if (st != FCSPH_OK) return st;
  Recorder *&r = active_recorder();
  r = &b->items.back().rec;
  st = fcsph_project_step(p, u, p_out, force, wall_vel, dt, nu);
  r = nullptr;
  if (st == FCSPH_OK && b->items.back().rec.recs.size() > (size_t)kBatchMaxLaunches)
    st = fail(p->ctx, FCSPH_E_UNSUPPORTED, "too many launches for a batch item");
  if (st != FCSPH_OK) {
    b->items.pop_back();
    return fail(b->ctx, st, std::string("batch step: ") + fcsph_ctx_last_error(p->ctx));
  }
  return FCSPH_OK;
}

fcsph_status fcsph_batch_add_rk3_substep(fcsph_batch *b, fcsph_plan *p, int k, double *const *u, double *p_out,
                                         const double *const *force, const double *const *wall_vel,
                                         double *const *F_store, double dt, double nu) {
  if (!b || !p) return b ? batch_fail(b, FCSPH_E_INVALID, "null plan") : FCSPH_E_INVALID;
  fcsph_status st = batch_add(b, p, BATCH_STEP);
  if (st != FCSPH_OK) return st;
  Recorder *&r = active_recorder();
  r = &b->items.back().rec;
  st = fcsph_rk3_substep(p, k, u, p_out, force, wall_vel, F_store, dt, nu);
  r = nullptr;
  if (st == FCSPH_OK && b->items.back().rec.recs.size() > (size_t)kBatchMaxLaunches)
    st = fail(p->ctx, FCSPH_E_UNSUPPORTED, "too many launches for a batch item");
  if (st != FCSPH_OK) {
    b->items.pop_back();
    return fail(b->ctx, st, std::string("batch RK3 sub-step: ") + fcsph_ctx_last_error(p->ctx));
  }
  return FCSPH_OK;
}

fcsph_status fcsph_batch_add_ppe(fcsph_batch *b, fcsph_plan *p, const void *rhs, double *phi) {
  if (!b || !p) return b ? batch_fail(b, FCSPH_E_INVALID, "null plan") : FCSPH_E_INVALID;
  fcsph_status st = batch_add(b, p, BATCH_PPE);
  if (st != FCSPH_OK) return st;
  Recorder *&r = active_recorder();
  r = &b->items.back().rec;
  st = fcsph_ppe_solve(p, rhs, phi);
  r = nullptr;
  if (st == FCSPH_OK && b->items.back().rec.recs.size() > (size_t)kBatchMaxLaunches)
    st = fail(p->ctx, FCSPH_E_UNSUPPORTED, "too many launches for a batch item");
  if (st != FCSPH_OK) {
    b->items.pop_back();
    return fail(b->ctx, st, std::string("batch ppe: ") + fcsph_ctx_last_error(p->ctx));
  }
  return FCSPH_OK;
}

fcsph_status fcsph_batch_launch(fcsph_batch *b) {
  if (!b) return FCSPH_E_INVALID;
  fcsph_ctx *c = b->ctx;
  batch_drop_graph(b);
  b->issues.clear();
  if (b->items.empty()) return FCSPH_OK;
  // group items by launch signature
  std::vector<std::string> sig(b->items.size());
  for (size_t i = 0; i < b->items.size(); ++i) {
    std::string &k = sig[i];
    for (const LaunchRecord &r : b->items[i].rec.recs) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "%p/%u.%u.%u/%u/%zu/%zu;", r.gfunc, r.grid.x, r.grid.y, r.grid.z, r.block.x,
                    r.lds, r.args.size());
      k += buf;
    }
  }
  std::vector<std::vector<int>> groups;
  std::vector<std::string> gsig;
  for (size_t i = 0; i < sig.size(); ++i) {
    size_t g = 0;
    while (g < gsig.size() && gsig[g] != sig[i]) ++g;
    if (g == gsig.size()) {
      gsig.push_back(sig[i]);
      groups.emplace_back();
    }
    groups[g].push_back((int)i);
  }
  // lay out the argument arrays: group by group, launch by launch
  if (hipEventSynchronize(b->upload_done) != hipSuccess) return hip_fail(c, hipGetLastError(), "batch upload wait");
  size_t off = 0;
  b->nstreams_used = std::min<int>((int)groups.size(), kBatchStreams);
  b->ngroups = (int)groups.size();
  for (size_t g = 0; g < groups.size(); ++g) {
    const std::vector<int> &m = groups[g];
    const Recorder &r0 = b->items[m[0]].rec;
    for (size_t k = 0; k < r0.recs.size(); ++k) {
      const size_t asz = r0.recs[k].args.size();
      off = (off + 255) & ~size_t(255);
      if (off + asz * m.size() > b->dev_bytes) return fail(c, FCSPH_E_WORKSPACE, "batch argument arrays exceed the workspace");
      for (size_t q = 0; q < m.size(); ++q)
        std::memcpy(b->host + off + q * asz, b->items[m[q]].rec.recs[k].args.data(), asz);
      fcsph_batch::Issue is;
      is.gfunc = r0.recs[k].gfunc;
      is.grid = dim3(r0.recs[k].grid.x, r0.recs[k].grid.y, (unsigned)m.size());
      is.block = r0.recs[k].block;
      is.lds = r0.recs[k].lds;
      is.args = b->dev + off;
      is.stream = (int)(g % kBatchStreams);
      b->issues.push_back(is);
      off += asz * m.size();
    }
  }
  hipError_t e = hipSetDevice(c->device);
  // the batch stream follows the context stream, uploads, runs the groups
  if (e == hipSuccess) e = hipEventRecord(b->done, c->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->done, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(b->dev, b->host, off, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->upload_done, b->stream);
  if (e == hipSuccess) e = batch_issue_all(b, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->done, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, b->done, 0);
  if (e != hipSuccess) return hip_fail(c, e, "batch launch");
  return FCSPH_OK;
}

fcsph_status fcsph_batch_capture(fcsph_batch *b) {
  if (!b) return FCSPH_E_INVALID;
  fcsph_ctx *c = b->ctx;
  if (b->issues.empty()) return fail(c, FCSPH_E_INVALID, "nothing launched to capture");
  batch_drop_graph(b);
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(c, e, "batch capture begin");
  hipError_t e2 = batch_issue_all(b, b->stream);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (e2 != hipSuccess || e != hipSuccess) {
    batch_drop_graph(b);
    return hip_fail(c, e2 != hipSuccess ? e2 : e, "batch capture");
  }
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    batch_drop_graph(b);
    return hip_fail(c, e, "batch graph instantiate");
  }
  return FCSPH_OK;
}

fcsph_status fcsph_batch_replay(fcsph_batch *b) {
  if (!b) return FCSPH_E_INVALID;
  fcsph_ctx *c = b->ctx;
  if (!b->exec) return fail(c, FCSPH_E_INVALID, "no captured graph");
  hipError_t e = hipEventRecord(b->done, c->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->done, 0);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->done, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, b->done, 0);
  if (e != hipSuccess) return hip_fail(c, e, "batch replay");
  return FCSPH_OK;
}

fcsph_status fcsph_batch_info(const fcsph_batch *b, int *items, int *groups, int *launches) {
  if (!b) return FCSPH_E_INVALID;
  if (items) *items = (int)b->items.size();
  if (groups) *groups = b->ngroups;
  if (launches) *launches = (int)b->issues.size();
  return FCSPH_OK;
}

}  // extern "C"
