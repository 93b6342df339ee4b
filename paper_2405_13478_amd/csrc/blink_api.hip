// Host side of libblink.so: argument validation, workspace layout and the
// launch sequences behind the C ABI declared in include/blink.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "blink.h"
#include "blink_kernels.hpp"

using namespace blink;

// Workspace of blink_image_batch_noalloc: a fixed array in the code object,
// one copy on every GPU the library runs on, held until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host the name
// is only a stand-in): it takes the device address from hipGetSymbolAddress
// once per device and uses that.
static __device__ __align__(256) unsigned char scratch[BLINK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SORT_RUN_SMALL = 1024;
constexpr int SORT_RUN = 8192;
constexpr int MAX_GRID_Y = 65535;
constexpr size_t CHUNK_TARGET_BYTES = size_t(1) << 30;    // half-spectrum bytes per chunk

bool n_supported(int n) {
  switch (n) {
    case 8: case 12: case 16: case 32: case 64: case 128: case 180:
    case 256: case 512: case 1024: case 2048: case 4096:
      return true;
    default:
      return false;
  }
}

inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int KB_MAX_SUPPORT = 16;
// sharpest accepted shape: I0(beta) stays within FP32 range where the weights
// come from cyl_bessel_i0f
constexpr double KB_MAX_BETA = 80.0;
// supports up to this take the kernel-gridding form with fewer row-weight registers
constexpr int KB_SMALL_SUPPORT = 8;

// A phase centre other than zenith asks for the geometric rotation.
inline bool rotates(const blink_problem* p) { return p->phase_l != 0.0 || p->phase_m != 0.0; }
// a delay per visibility: geometric rotation or cable lengths
inline bool delays(const blink_problem* p, const blink_inputs* in) { return rotates(p) || in->cable_m != nullptr; }

// pi sqrt(0.5625 W^2 - 0.8): the Kaiser-Bessel shape for a grid twice the
// kept image (Beatty, Nishimura and Pauly 2005); negative when W is too small.
double kb_default_beta(int w) {
  const double q = 0.5625 * w * w - 0.8;
  return q > 0 ? M_PI * sqrt(q) : -1.0;
}

// I0(x) by its power series sum_k ((x/2)^2)^k / (k!)^2 (all terms positive;
// run to double rounding), for the kernel's normalisation 1 / I0(beta).
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500 && term > 1e-17 * sum; ++k) {
    term *= q / ((double)k * k);
    sum += term;
  }
  return sum;
}

// Polynomial of the Kaiser-Bessel weight in s = 2w - 1, w = 1 - (2d/W)^2
// (see kb_weight): C interpolated at KB_CHEB_NODES Chebyshev points of s, the
// Chebyshev series truncated after the first degree D whose dropped terms sum
// below 2e-8 in magnitude, then rewritten in powers of s (double) and rounded
// once to float (kpoly[k] of s^k, zeros above D). Switched off when no D below
// KB_POLY_TERMS suffices or the interpolant's last terms have not decayed.
constexpr int KB_CHEB_NODES = 40;

void kb_poly(double beta, ImgArgs* a) {
  const int n = KB_CHEB_NODES;
  const double pi = 3.14159265358979323846;
  const double inv = 1.0 / bessel_i0(beta);
  double g[KB_CHEB_NODES], c[KB_CHEB_NODES];
  for (int i = 0; i < n; ++i) {
    const double s = cos(pi * (i + 0.5) / n);
    g[i] = bessel_i0(beta * sqrt(0.5 * (1.0 + s))) * inv;
  }
  for (int j = 0; j < n; ++j) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += g[i] * cos(pi * j * (i + 0.5) / n);
    c[j] = acc * (j == 0 ? 1.0 : 2.0) / n;
  }
  a->kpoly_on = 0;
  if (fabs(c[n - 1]) + fabs(c[n - 2]) > 1e-12) return;       // not resolved by n nodes
  int deg = -1;
  double tail = 0.0;
  for (int j = n - 1; j >= 0; --j) {                         // smallest D with sum_{j > D} |c_j| < 2e-8
    if (tail + fabs(c[j]) >= 2e-8) { deg = j; break; }
    tail += fabs(c[j]);
  }
  if (deg < 0) deg = 0;
  if (deg > KB_POLY_TERMS - 1) return;
  // sum_j c_j T_j(s) in powers of s: T_0 = 1, T_1 = s, T_{j+1} = 2 s T_j - T_{j-1}
  double m[KB_POLY_TERMS] = {0.0}, t0[KB_POLY_TERMS] = {0.0}, t1[KB_POLY_TERMS] = {0.0};
  t0[0] = 1.0;
  t1[1] = 1.0;
  m[0] = c[0];
  if (deg >= 1) m[1] += c[1];
  for (int j = 2; j <= deg; ++j) {
    double t2[KB_POLY_TERMS] = {0.0};
    for (int k = 0; k <= j; ++k) t2[k] = (k > 0 ? 2.0 * t1[k - 1] : 0.0) - t0[k];
    for (int k = 0; k <= j; ++k) m[k] += c[j] * t2[k];
    for (int k = 0; k < KB_POLY_TERMS; ++k) { t0[k] = t1[k]; t1[k] = t2[k]; }
  }
  for (int k = 0; k < KB_POLY_TERMS; ++k) a->kpoly[k] = k <= deg ? (float)m[k] : 0.0f;
  a->kpoly_deg = deg;
  a->kpoly_on = 1;
}

struct Work {
  unsigned long long* key[2];
  int* idx[2];
  int* counters;      // [2T]: n_unflagged then n_valid
  double* su;
  double* sv;
  int* perm;
  double* sd;         // sorted geometric delays, only with a phase rotation
  double* vmax;       // [T] largest |v| of the usable baselines (image call)
  int* bnd;
  int* ncz;
  int* wpart;
  int* kpart;
  int wstride;
  float2* half;
  float2* gamma;
  float2* pacc;
  int* kdens;         // kernel gridding with uniform weighting: [chunk][B]
  float2* gfull;      // adjoint with a gridding kernel: [chunk][N/2][N]
};

int default_chunk(const blink_problem* p, int call, long long n_img) {
  if (p->chunk_images > 0) return (int)std::min<long long>(p->chunk_images, std::max<long long>(n_img, 1));
  long long per = 1;
  if (call != BLINK_CALL_GRID) per = (long long)(p->grid_n / 2) * p->out_n * 8;
  // the adjoint with a gridding kernel also keeps every transformed column
  if (call == BLINK_CALL_ADJOINT && p->kernel_support > 0) per += (long long)(p->grid_n / 2) * p->grid_n * 8;
  long long c = std::max<long long>(1, (long long)CHUNK_TARGET_BYTES / per);
  c = std::min<long long>(c, std::max<long long>(n_img, 1));
  return (int)std::min<long long>(c, MAX_GRID_Y);
}

// Lays out the workspace (base may be null to only size it).
size_t carve(const blink_problem* p, int call, int chunk, char* base, Work* w) {
  const size_t T = (size_t)p->n_time, B = (size_t)p->n_bl, N = (size_t)p->grid_n;
  const size_t M = (size_t)p->out_n;
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* r = base ? base + o : nullptr;
    o += al(bytes);
    return r;
  };
  Work x{};
  x.key[0] = (unsigned long long*)take(T * B * 8);
  x.key[1] = (unsigned long long*)take(T * B * 8);
  x.idx[0] = (int*)take(T * B * 4);
  x.idx[1] = (int*)take(T * B * 4);
  x.counters = (int*)take(2 * T * 4);
  x.su = (double*)take(T * B * 8);
  x.sv = (double*)take(T * B * 8);
  x.perm = (int*)take(T * B * 4);
  // delay table of the phase rotation or cable correction (whether one is
  // applied depends on the inputs, which the size query does not see)
  x.sd = (double*)take(T * B * 8);
  if (call == BLINK_CALL_IMAGE) x.vmax = (double*)take(T * 8);
  const size_t n_img = (size_t)p->n_time * (size_t)p->n_chan;
  x.bnd = (int*)take(n_img * (N + 2) * 4);
  x.ncz = (int*)take(n_img * 4);
  x.wstride = (int)((N + 1) / 2);      // column tiles per image for any tile width >= 2
  x.wpart = (int*)take(n_img * x.wstride * 4);
  x.kpart = (int*)take(n_img * x.wstride * 4);
  if (call == BLINK_CALL_IMAGE || call == BLINK_CALL_ADJOINT)
    x.half = (float2*)take((size_t)chunk * (N / 2) * M * 8);
  if (call == BLINK_CALL_ADJOINT) {
    x.gamma = (float2*)take((size_t)chunk * B * 8);
    x.pacc = (float2*)take(B * 8);
  }
  if (p->kernel_support > 0 && p->weighting == BLINK_UNIFORM)
    x.kdens = (int*)take((size_t)chunk * B * 4);
  if (call == BLINK_CALL_ADJOINT && p->kernel_support > 0)
    x.gfull = (float2*)take((size_t)chunk * (N / 2) * N * 8);
  if (w) *w = x;
  return o;
}

blink_status validate_problem(const blink_problem* p, int call) {
  if (!p) return BLINK_E_ARG;
  if (p->n_time < 0 || p->n_chan < 0 || p->n_bl < 0 || p->n_ant < 0) return BLINK_E_SIZE;
  if (!(p->pixscale > 0.0) || !isfinite(p->pixscale)) return BLINK_E_ARG;
  if (p->weighting != BLINK_NATURAL && p->weighting != BLINK_UNIFORM) return BLINK_E_ARG;
  if (p->norm != BLINK_NORM_NONE && p->norm != BLINK_NORM_WEIGHTS) return BLINK_E_ARG;
  if (p->vis_type < BLINK_VIS_C64 || p->vis_type > BLINK_VIS_BF16) return BLINK_E_ARG;
  if (p->chunk_images < 0) return BLINK_E_ARG;
  if (p->cols_per_wg != 0 && p->cols_per_wg != 2 && p->cols_per_wg != 4 && p->cols_per_wg != 8)
    return BLINK_E_ARG;
  if (p->rows_wg < 0) return BLINK_E_ARG;
  if (p->kernel_support < 0 || p->kernel_support > KB_MAX_SUPPORT) return BLINK_E_ARG;
  if (p->reproject != 0 && p->reproject != 1) return BLINK_E_ARG;
  if (!isfinite(p->phase_l) || !isfinite(p->phase_m) ||
      !(p->phase_l * p->phase_l + p->phase_m * p->phase_m < 1.0))
    return BLINK_E_ARG;
  if (p->kernel_support > 0) {
    if (!isfinite(p->kernel_beta) || p->kernel_beta > KB_MAX_BETA) return BLINK_E_ARG;
    if (p->kernel_beta < 0 && kb_default_beta(p->kernel_support) < 0) return BLINK_E_ARG;
  }
  if (call < BLINK_CALL_GRID || call > BLINK_CALL_ADJOINT) return BLINK_E_ARG;
  if (p->grid_n < 2 || (p->grid_n & 1)) return BLINK_E_SIZE;
  if (call != BLINK_CALL_GRID) {
    if (p->out_n < 2 || (p->out_n & 1) || p->out_n > p->grid_n) return BLINK_E_SIZE;
  }
  const long long T = p->n_time, C = p->n_chan, B = p->n_bl, N = p->grid_n;
  if (T * C > INT32_MAX || T * B > INT32_MAX) return BLINK_E_SIZE;
  if ((double)T * C * B > 9.0e18 || (double)T * C * N * N > 9.0e18) return BLINK_E_SIZE;
  if (!n_supported(p->grid_n)) return BLINK_E_UNSUPPORTED;
  return BLINK_OK;
}

blink_status validate_inputs(const blink_problem* p, const blink_inputs* in) {
  if (!in) return BLINK_E_ARG;
  const long long n_img = (long long)p->n_time * p->n_chan;
  if (n_img == 0 || p->n_bl == 0) return BLINK_OK;
  if (!in->vis || !in->uvw_m || !in->freq_hz) return BLINK_E_ARG;
  if (p->vis_type != BLINK_VIS_C64 && !in->vis_scale) return BLINK_E_ARG;
  if (in->gains && (!in->ant1 || !in->ant2 || p->n_ant < 1)) return BLINK_E_ARG;
  if (in->cable_m && (!in->ant1 || !in->ant2 || p->n_ant < 1)) return BLINK_E_ARG;
  return BLINK_OK;
}

blink_status check_ws(const blink_problem* p, int call, void* ws, size_t ws_bytes, int* chunk) {
  const long long n_img = (long long)p->n_time * p->n_chan;
  *chunk = default_chunk(p, call, n_img);
  const size_t need = carve(p, call, *chunk, nullptr, nullptr);
  if (need == 0) return BLINK_OK;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return BLINK_E_WORKSPACE;
  return BLINK_OK;
}

blink_status launched() {
  return hipGetLastError() == hipSuccess ? BLINK_OK : BLINK_E_HIP;
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Records a start/end HIP event pair around launches when active (timed
// entry point); a no-op otherwise.
struct Timer {
  hipStream_t st = nullptr;
  bool on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  int cls = -1;
  bool bad = false;                      // an event record failed: timings are not trustworthy
  hipEvent_t cur = nullptr;
  void begin(int c) {
    if (!on) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
    if (hipEventRecord(e, st) != hipSuccess) bad = true;
    cls = c;
    cur = e;
  }
  void end() {
    if (!on || !cur) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
    if (hipEventRecord(e, st) != hipSuccess) bad = true;
    ev.push_back({cls, {cur, e}});
    cur = nullptr;
  }
  blink_status collect(blink_kernel_times* out) {
    for (int k = 0; k < BLINK_KCLASS_COUNT; ++k) { out->ms[k] = 0.0; out->launches[k] = 0; }
    blink_status r = bad ? BLINK_E_HIP : BLINK_OK;
    if (r == BLINK_OK && !ev.empty() && hipEventSynchronize(ev.back().second.second) != hipSuccess)
      r = BLINK_E_HIP;
    for (auto& x : ev) {
      float ms = 0.f;
      if (r == BLINK_OK && hipEventElapsedTime(&ms, x.second.first, x.second.second) == hipSuccess) {
        out->ms[x.first] += ms;
        out->launches[x.first] += 1;
      }
      (void)hipEventDestroy(x.second.first);
      (void)hipEventDestroy(x.second.second);
    }
    ev.clear();
    return r;
  }
};

// What run_sort produced beside the sorted lists.
constexpr int SORTED_VMAX = 1;     // the per-timestep largest |v|
constexpr int SORTED_BOUNDS = 2;   // the cell bounds of every image (one channel per timestep)

// per-timestep order of the usable baselines by u (metres). With `img` (the
// image call), the small-list sort also writes the per-timestep largest |v|
// and, when there is one channel per timestep, the images' cell bounds.
int run_sort(const blink_problem* p, const blink_inputs* in, const Work& w, hipStream_t st,
             Timer* tm = nullptr, bool img = false) {
  Timer none;
  Timer& T_ = tm ? *tm : none;
  const int T = p->n_time, B = p->n_bl;
  SortArgs s{};
  s.T = T; s.B = B;
  s.uvw = in->uvw_m; s.flags = in->flags;
  s.key[0] = w.key[0]; s.key[1] = w.key[1];
  s.idx[0] = w.idx[0]; s.idx[1] = w.idx[1];
  s.n_unflagged = w.counters; s.n_valid = w.counters + T;
  s.su = w.su; s.sv = w.sv; s.perm = w.perm;
  s.sd = delays(p, in) ? w.sd : nullptr;
  if (s.sd != nullptr) {
    s.pl = p->phase_l;
    s.pm = p->phase_m;
    s.pn1 = sqrt(1.0 - p->phase_l * p->phase_l - p->phase_m * p->phase_m) - 1.0;
    s.cable = in->cable_m;
    s.ant1 = in->ant1;
    s.ant2 = in->ant2;
    s.n_ant = p->n_ant;
  }
  if (p->reproject && rotates(p)) {
    // axes of the tangent plane at s0 (the zenith frame's east and north
    // axes carried by the smallest rotation that takes zenith to s0)
    const double l0 = p->phase_l, m0 = p->phase_m;
    const double n0 = sqrt(1.0 - l0 * l0 - m0 * m0);
    const double k = 1.0 / (1.0 + n0);
    s.proj = 1;
    s.eu[0] = n0 + m0 * m0 * k; s.eu[1] = -l0 * m0 * k; s.eu[2] = -l0;
    s.ev[0] = -l0 * m0 * k; s.ev[1] = n0 + l0 * l0 * k; s.ev[2] = -m0;
  }
  const bool small = B > 0 && B <= SORT_RUN;
  const bool bounds = img && small && p->n_chan == 1;
  if (img && small) s.vmax = w.vmax;
  if (bounds) {
    s.N = p->grid_n;
    s.kw = p->kernel_support;
    s.ndx = (double)p->grid_n * p->pixscale;
    s.freq = in->freq_hz;
    s.bnd = w.bnd;
    s.ncz = w.ncz;
  }
  if (B == 0 || B > SORT_RUN) {
    T_.begin(0);
    hipLaunchKernelGGL(k_sort_init, dim3(cdiv(2LL * T, 256)), dim3(256), 0, st, w.counters, 2 * T);
    T_.end();
  }
  if (B == 0 || T == 0) return 0;
  for (int t0 = 0; t0 < T; t0 += MAX_GRID_Y) {
    const int nt = std::min(MAX_GRID_Y, T - t0);
    s.t0 = t0;
    T_.begin(0);
    if (B <= SORT_RUN_SMALL) {
      if (bounds) hipLaunchKernelGGL((k_sort_small<SORT_RUN_SMALL, true>), dim3(1, nt), dim3(1024), 0, st, s);
      else hipLaunchKernelGGL((k_sort_small<SORT_RUN_SMALL>), dim3(1, nt), dim3(1024), 0, st, s);
      T_.end();
      continue;
    }
    if (B <= SORT_RUN) {
      if (bounds) hipLaunchKernelGGL((k_sort_small<SORT_RUN, true>), dim3(1, nt), dim3(1024), 0, st, s);
      else hipLaunchKernelGGL((k_sort_small<SORT_RUN>), dim3(1, nt), dim3(1024), 0, st, s);
      T_.end();
      continue;
    }
    hipLaunchKernelGGL((k_sort_run<SORT_RUN>), dim3(cdiv(B, SORT_RUN), nt), dim3(1024), 0, st, s);
    T_.end();
    int src = 0;
    for (long long wdt = SORT_RUN; wdt < B; wdt *= 2) {
      T_.begin(0);
      hipLaunchKernelGGL(k_merge, dim3(cdiv(B, 256), nt), dim3(256), 0, st, s, (int)wdt, src);
      T_.end();
      src ^= 1;
    }
    T_.begin(0);
    hipLaunchKernelGGL(k_sort_finish, dim3(cdiv(B, 256), nt), dim3(256), 0, st, s, src);
    T_.end();
  }
  return small && img ? (SORTED_VMAX | (bounds ? SORTED_BOUNDS : 0)) : 0;
}

ImgArgs make_args(const blink_problem* p, const blink_inputs* in, const Work& w) {
  ImgArgs a{};
  a.T = p->n_time; a.C = p->n_chan; a.B = p->n_bl; a.N = p->grid_n; a.M = p->out_n;
  a.weighting = p->weighting; a.norm = p->norm; a.vis_type = p->vis_type;
  a.ndx = (double)p->grid_n * p->pixscale;
  a.vis = in->vis; a.vis_scale = in->vis_scale; a.freq = in->freq_hz;
  a.ant1 = in->ant1; a.ant2 = in->ant2;
  a.gains = reinterpret_cast<const float2*>(in->gains);
  a.n_ant = p->n_ant;
  a.su = w.su; a.sv = w.sv; a.perm = w.perm; a.sd = delays(p, in) ? w.sd : nullptr;
  a.n_unflagged = w.counters; a.n_valid = w.counters + p->n_time;
  a.vmax = w.vmax;
  a.bnd = w.bnd; a.ncz = w.ncz; a.wpart = w.wpart; a.kpart = w.kpart; a.wstride = w.wstride;
  a.half = w.half; a.gamma = w.gamma; a.pacc = w.pacc;
  a.kdens = w.kdens;
  a.gfull = w.gfull;
  a.kw = p->kernel_support;
  if (a.kw > 0) {
    const double beta = p->kernel_beta < 0 ? kb_default_beta(a.kw) : p->kernel_beta;
    a.kbeta = (float)beta;
    a.kinv = (float)(1.0 / bessel_i0(beta));
    a.kbeta_d = beta;
    a.ktaper0_d = beta > 0 ? sinh(beta) / beta : 1.0;
    a.k2w = (float)(2.0 / a.kw);
    kb_poly(beta, &a);
  }
  return a;
}

// per-entry cell occupancy for kernel gridding with uniform weighting
template <int N>
void launch_kb_density(const ImgArgs& a, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_kb_density<N>, dim3((unsigned)n), dim3(DENS_WAVES * WAVE),
                     (size_t)DENS_WAVES * N * sizeof(int), st, a);
}

template <int N, bool UNI, int CPW>
void launch_cols_image(ImgArgs& a, int n, hipStream_t st) {
  using C_ = Cols<N, CPW>;
  a.wtiles = a.ntiles = (int)cdiv(N / 2, CPW);
  const dim3 g1((unsigned)(cdiv(n, 8) * 8LL * a.ntiles));
  hipLaunchKernelGGL((k_grid_cols<N, MODE_IMAGE, UNI, CPW>), g1, dim3(C_::THREADS), C_::grid_lds_bytes(UNI), st, a);
}

// the cutout M = N/2 (half of the grid's field) gets the form with the
// cutout fixed at compile time
template <int N>
constexpr bool half_cutout_form() { return N >= 512; }

template <int N, int CPW, bool UNI>
void launch_cols_half(ImgArgs& a, int n, hipStream_t st) {
  using C_ = ColsHalf<N, CPW, UNI>;
  a.ntiles = (int)cdiv(N / 2, CPW);
  a.wtiles = N / 2;                       // one partial per column
  const dim3 g1((unsigned)(cdiv(n, 8) * 8LL * a.ntiles));
  if constexpr (half_cutout_form<N>()) {
    if (a.M == N / 2) {
      hipLaunchKernelGGL((k_grid_cols_half<N, CPW, UNI, N / 4>), g1, dim3(C_::THREADS), C_::LDS, st, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_grid_cols_half<N, CPW, UNI>), g1, dim3(C_::THREADS), C_::LDS, st, a);
}

// Power-of-two sizes up to 2048 take the column kernel whose exchanges go
// through half-length LDS buffers (measured at N = 1024, natural weighting:
// 4.52 ms per 7,680 images against 5.20 ms with full-length buffers); other
// sizes and kernel gridding take the full-length one.
template <int N>
constexpr bool cols_half() { return plan_even(N) && N <= 2048; }

template <int N, bool UNI>
void launch_cols_image(ImgArgs& a, int n, int cpw, hipStream_t st) {
  if constexpr (cols_half<N>()) {
    if (cpw == 2) launch_cols_half<N, 2, UNI>(a, n, st);
    else if (cpw == 4) launch_cols_half<N, 4, UNI>(a, n, st);
    else launch_cols_half<N, 8, UNI>(a, n, st);
  } else {
    if (cpw == 2) launch_cols_image<N, UNI, 2>(a, n, st);
    else if (cpw == 4) launch_cols_image<N, UNI, 4>(a, n, st);
    else launch_cols_image<N, UNI, 8>(a, n, st);
  }
}

// LDS one workgroup of the column kernel needs at a tile width (checked
// against the 160 KiB of a gfx950 CU before any launch).
template <int N>
size_t cols_lds(int cpw, bool uni, bool kb) {
  if (cols_half<N>() && !kb) {
    if (uni) return cpw == 2 ? ColsHalf<N, 2, true>::LDS : cpw == 4 ? ColsHalf<N, 4, true>::LDS
                                                            : ColsHalf<N, 8, true>::LDS;
    return cpw == 2 ? ColsHalf<N, 2, false>::LDS : cpw == 4 ? ColsHalf<N, 4, false>::LDS
                                                            : ColsHalf<N, 8, false>::LDS;
  }
  return cpw == 2 ? Cols<N, 2>::grid_lds_bytes(uni) : cpw == 4 ? Cols<N, 4>::grid_lds_bytes(uni)
                                                          : Cols<N, 8>::grid_lds_bytes(uni);
}
constexpr size_t LDS_PER_CU = size_t(160) << 10;

// Row pass: the block-store variant when the cutout half-width is a
// multiple of the wavefront width (and the plan's last stage allows it).
// Measured on MI355X: faster at N = 1024, slower than per-lane stores at
// N = 2048 (4.85 against 4.1 ms per 384 images), so larger N keep those.
constexpr int ROWS_BLOCK_STORE_MAX_N = 1024;
// Row pass through half-length LDS buffers at power-of-two sizes up to 2048.
template <int N>
constexpr bool rows_half() { return plan_even(N) && N <= 2048; }
template <int N>
constexpr size_t rows_lds_base() { return rows_half<N>() ? RowsHalf<N>::LDS : Rows<N>::LDS; }

template <int N, bool KB>
void launch_rows(const blink_problem* p, ImgArgs& a, long long nwg, size_t lds, hipStream_t st) {
  if constexpr (rows_half<N>()) {
    if constexpr (blocks_aligned(N) && N <= ROWS_BLOCK_STORE_MAX_N) {
      if ((p->out_n / 2) % WAVE == 0) {
        if constexpr (half_cutout_form<N>()) {
          if (p->out_n == N / 2) {
            hipLaunchKernelGGL((k_rows_half<N, true, KB, N / 4>), dim3((unsigned)nwg), dim3(RowsHalf<N>::THREADS),
                               lds, st, a);
            return;
          }
        }
        hipLaunchKernelGGL((k_rows_half<N, true, KB>), dim3((unsigned)nwg), dim3(RowsHalf<N>::THREADS), lds, st, a);
        return;
      }
    }
    hipLaunchKernelGGL((k_rows_half<N, false, KB>), dim3((unsigned)nwg), dim3(RowsHalf<N>::THREADS), lds, st, a);
  } else {
    if constexpr (blocks_aligned(N) && N <= ROWS_BLOCK_STORE_MAX_N) {
      if ((p->out_n / 2) % WAVE == 0) {
        hipLaunchKernelGGL((k_rows<N, true, KB>), dim3((unsigned)nwg), dim3(Rows<N>::THREADS), lds, st, a);
        return;
      }
    }
    hipLaunchKernelGGL((k_rows<N, false, KB>), dim3((unsigned)nwg), dim3(Rows<N>::THREADS), lds, st, a);
  }
}

template <int N>
blink_status image_n(const blink_problem* p, ImgArgs a, int chunk, hipStream_t st, Timer* tm, int sorted) {
  Timer& T_ = *tm;
  const long long n_img = (long long)p->n_time * p->n_chan;
  const bool uni = p->weighting == BLINK_UNIFORM;
  const bool kb = p->kernel_support > 0;
  // kernel gridding runs at the default tile width only
  const int cpw = kb ? cols_per_wg(N) : (p->cols_per_wg ? p->cols_per_wg : cols_per_wg(N));
  if (cols_lds<N>(cpw, uni, kb) > LDS_PER_CU) return BLINK_E_UNSUPPORTED;
  const size_t rows_lds = rows_lds_base<N>() + (kb ? (size_t)p->out_n * sizeof(float) : 0);
  if (rows_lds > LDS_PER_CU) return BLINK_E_UNSUPPORTED;
  // partials per image: one per column (half-length column kernel) or per tile
  a.wtiles = cols_half<N>() && !kb ? N / 2 : (int)cdiv(N / 2, cpw);
  if (!(sorted & SORTED_BOUNDS)) {
    T_.begin(1);
    hipLaunchKernelGGL(k_bounds, dim3((unsigned)n_img), dim3(256), 0, st, a);
    T_.end();
  }
  for (long long i0 = 0; i0 < n_img; i0 += chunk) {
    const int n = (int)std::min<long long>(chunk, n_img - i0);
    a.img0 = (int)i0; a.nimg = n;
    if (a.kdens != nullptr) {
      T_.begin(2);
      launch_kb_density<N>(a, n, st);
      T_.end();
    }
    T_.begin(2);
    if (kb) {
      constexpr int CPW = cols_per_wg(N);
      using C_ = Cols<N, CPW>;
      a.ntiles = (int)cdiv(N / 2, CPW);
      const dim3 g1((unsigned)(cdiv(n, 8) * 8LL * a.ntiles));
      if (p->kernel_support <= KB_SMALL_SUPPORT)
        hipLaunchKernelGGL((k_grid_cols<N, MODE_IMAGE, false, CPW, true, KB_SMALL_SUPPORT>), g1, dim3(C_::THREADS),
                           C_::grid_lds_bytes(false), st, a);
      else
        hipLaunchKernelGGL((k_grid_cols<N, MODE_IMAGE, false, CPW, true, KB_MAX_SUPPORT>), g1, dim3(C_::THREADS),
                           C_::grid_lds_bytes(false), st, a);
    } else if (uni) {
      launch_cols_image<N, true>(a, n, cpw, st);
    } else {
      launch_cols_image<N, false>(a, n, cpw, st);
    }
    T_.end();
    // row pass: one workgroup per row tile, or a persistent grid of rows_wg workgroups
    const long long row_tiles = (long long)n * cdiv(p->out_n / 2, Rows<N>::PPW);
    const long long nwg = p->rows_wg > 0 ? std::min<long long>(row_tiles, p->rows_wg) : row_tiles;
    T_.begin(3);
    if (kb) launch_rows<N, true>(p, a, nwg, rows_lds, st);
    else launch_rows<N, false>(p, a, nwg, rows_lds, st);
    T_.end();
  }
  return launched();
}

template <int N>
blink_status grid_n(const blink_problem* p, ImgArgs a, int chunk, hipStream_t st) {
  const long long n_img = (long long)p->n_time * p->n_chan;
  const bool uni = p->weighting == BLINK_UNIFORM;
  const size_t lds1 = Cols<N>::grid_lds_bytes(true);
  a.wtiles = (int)cdiv(N, Cols<N>::CPW);
  hipLaunchKernelGGL(k_bounds, dim3((unsigned)n_img), dim3(256), 0, st, a);
  for (long long i0 = 0; i0 < n_img; i0 += chunk) {
    const int n = (int)std::min<long long>(chunk, n_img - i0);
    a.img0 = (int)i0; a.nimg = n;
    a.ntiles = (int)cdiv(N, Cols<N>::CPW);
    const dim3 g1((unsigned)(cdiv(n, 8) * 8LL * a.ntiles));
    if (a.kdens != nullptr) launch_kb_density<N>(a, n, st);
    if (p->kernel_support > KB_SMALL_SUPPORT)
      hipLaunchKernelGGL((k_grid_cols<N, MODE_GRID, false, Cols<N>::CPW, true, KB_MAX_SUPPORT>), g1,
                         dim3(Cols<N>::THREADS), lds1, st, a);
    else if (p->kernel_support > 0)
      hipLaunchKernelGGL((k_grid_cols<N, MODE_GRID, false, Cols<N>::CPW, true, KB_SMALL_SUPPORT>), g1,
                         dim3(Cols<N>::THREADS), lds1, st, a);
    else if (uni)
      hipLaunchKernelGGL((k_grid_cols<N, MODE_GRID, true>), g1, dim3(Cols<N>::THREADS), lds1, st, a);
    else
      hipLaunchKernelGGL((k_grid_cols<N, MODE_GRID, false>), g1, dim3(Cols<N>::THREADS), lds1, st, a);
  }
  if (a.weight_sum || a.n_dropped)
    hipLaunchKernelGGL(k_grid_finish, dim3(cdiv(n_img, 256)), dim3(256), 0, st, a, (int)n_img);
  return launched();
}

template <int N>
blink_status adjoint_n(const blink_problem* p, ImgArgs a, int chunk, hipStream_t st) {
  const long long n_img = (long long)p->n_time * p->n_chan;
  const bool uni = p->weighting == BLINK_UNIFORM;
  const bool kb = p->kernel_support > 0;
  if (a.gains)
    hipLaunchKernelGGL(k_fill2, dim3(cdiv(a.B, 256)), dim3(256), 0, st, a.pacc, (size_t)a.B);
  a.wtiles = (int)cdiv(N / 2, Cols<N>::CPW);
  hipLaunchKernelGGL(k_bounds, dim3((unsigned)n_img), dim3(256), 0, st, a);
  for (long long i0 = 0; i0 < n_img; i0 += chunk) {
    const int n = (int)std::min<long long>(chunk, n_img - i0);
    a.img0 = (int)i0; a.nimg = n;
    if (a.kdens != nullptr) launch_kb_density<N>(a, n, st);
    // W from the forward call's weight sums when the caller passes them, else
    // counted again from the sorted lists (with a gridding kernel: by the
    // forward column pass itself, whose transformed columns the row pass
    // below then overwrites)
    if (a.wsum_in == nullptr && kb) {
      constexpr int CPW = Cols<N>::CPW;
      a.ntiles = (int)cdiv(N / 2, CPW);
      const dim3 g1((unsigned)(cdiv(n, 8) * 8LL * a.ntiles));
      const size_t lds = Cols<N, CPW>::grid_lds_bytes(false);
      if (p->kernel_support <= KB_SMALL_SUPPORT)
        hipLaunchKernelGGL((k_grid_cols<N, MODE_IMAGE, false, CPW, true, KB_SMALL_SUPPORT>), g1,
                           dim3(Cols<N, CPW>::THREADS), lds, st, a);
      else
        hipLaunchKernelGGL((k_grid_cols<N, MODE_IMAGE, false, CPW, true, KB_MAX_SUPPORT>), g1,
                           dim3(Cols<N, CPW>::THREADS), lds, st, a);
    } else if (a.wsum_in == nullptr) {
      const dim3 gw(cdiv(N / 2, Cols<N>::CPW), n);
      const size_t ldsw = uni ? (size_t)Cols<N>::CPW * N * sizeof(int) : 0;
      if (uni)
        hipLaunchKernelGGL((k_weights<N, true>), gw, dim3(Cols<N>::THREADS), ldsw, st, a);
      else
        hipLaunchKernelGGL((k_weights<N, false>), gw, dim3(Cols<N>::THREADS), ldsw, st, a);
    }
    const dim3 g2(cdiv(p->out_n / 2, Rows<N>::PPW), n);
    hipLaunchKernelGGL((k_rows_adj<N>), g2, dim3(Rows<N>::THREADS), Rows<N>::LDS, st, a);
    // flagged and dropped baselines are never visited: their gradients are zero
    const size_t ng = (size_t)n * a.B;
    hipLaunchKernelGGL(k_fill2, dim3(cdiv((long long)ng, 256)), dim3(256), 0, st,
                       a.vis_grad + (size_t)i0 * a.B, ng);
    if (a.gains)
      hipLaunchKernelGGL(k_fill2, dim3(cdiv((long long)ng, 256)), dim3(256), 0, st, a.gamma, ng);
    a.ntiles = (int)cdiv(N / 2, Cols<N>::CPW);
    const dim3 g1((unsigned)(cdiv(n, 8) * 8LL * a.ntiles));
    const size_t lds1 = Cols<N>::lds_bytes(uni && !kb);
    if (kb) {
      hipLaunchKernelGGL((k_cols_adj<N, false, true>), g1, dim3(Cols<N>::THREADS), lds1, st, a);
      const dim3 gd(cdiv(a.B, 256), n);
      if (p->kernel_support <= KB_SMALL_SUPPORT)
        hipLaunchKernelGGL((k_degrid_kb<N, KB_SMALL_SUPPORT>), gd, dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL((k_degrid_kb<N, KB_MAX_SUPPORT>), gd, dim3(256), 0, st, a);
    } else if (uni) {
      hipLaunchKernelGGL((k_cols_adj<N, true>), g1, dim3(Cols<N>::THREADS), lds1, st, a);
    } else {
      hipLaunchKernelGGL((k_cols_adj<N, false>), g1, dim3(Cols<N>::THREADS), lds1, st, a);
    }
    if (a.gains)
      hipLaunchKernelGGL(k_gq_reduce, dim3(cdiv(a.B, 64)), dim3(256), 0, st, a);
  }
  if (a.gains && a.gain_grad)
    hipLaunchKernelGGL(k_gain_grad, dim3(p->n_ant), dim3(256), 0, st, a);
  return launched();
}

template <int N>
blink_status fft2d_n(const float2* in, float2* out, int batch, int sign, hipStream_t st) {
  const long long rows = (long long)batch * N;
  constexpr long long ROWS_PER_LAUNCH = 1LL << 30;
  for (long long r0 = 0; r0 < rows; r0 += ROWS_PER_LAUNCH) {
    const long long nr = std::min<long long>(rows - r0, ROWS_PER_LAUNCH);
    const dim3 g(cdiv(nr, Fft2<N>::VPW));
    if (sign > 0)
      hipLaunchKernelGGL((k_fft_rows<N, +1>), g, dim3(Fft2<N>::THREADS), Fft2<N>::LDS, st, in + r0 * N, out + r0 * N, (int)nr);
    else
      hipLaunchKernelGGL((k_fft_rows<N, -1>), g, dim3(Fft2<N>::THREADS), Fft2<N>::LDS, st, in + r0 * N, out + r0 * N, (int)nr);
  }
  for (long long b0 = 0; b0 < batch; b0 += MAX_GRID_Y) {
    const int nb = (int)std::min<long long>(MAX_GRID_Y, batch - b0);
    const dim3 g(cdiv(N, Fft2<N>::VPW), nb);
    float2* d = out + (size_t)b0 * N * N;
    if (sign > 0)
      hipLaunchKernelGGL((k_fft_cols<N, +1>), g, dim3(Fft2<N>::THREADS), Fft2<N>::LDS, st, d);
    else
      hipLaunchKernelGGL((k_fft_cols<N, -1>), g, dim3(Fft2<N>::THREADS), Fft2<N>::LDS, st, d);
  }
  return launched();
}

#define BLINK_DISPATCH_N(n, CALL)                                    \
  switch (n) {                                                       \
    case 8: return CALL(8);                                          \
    case 12: return CALL(12);                                        \
    case 16: return CALL(16);                                        \
    case 32: return CALL(32);                                        \
    case 64: return CALL(64);                                        \
    case 128: return CALL(128);                                      \
    case 180: return CALL(180);                                      \
    case 256: return CALL(256);                                      \
    case 512: return CALL(512);                                      \
    case 1024: return CALL(1024);                                    \
    case 2048: return CALL(2048);                                    \
    case 4096: return CALL(4096);                                    \
    default: return BLINK_E_UNSUPPORTED;                             \
  }

}  // namespace

extern "C" {

const char* blink_status_string(blink_status s) {
  switch (s) {
    case BLINK_OK: return "ok";
    case BLINK_E_ARG: return "invalid argument";
    case BLINK_E_SIZE: return "invalid size";
    case BLINK_E_UNSUPPORTED: return "unsupported configuration";
    case BLINK_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case BLINK_E_HIP: return "HIP launch failed";
    default: return "unknown status";
  }
}

int32_t blink_supported_n(int32_t n) { return n_supported(n) ? 1 : 0; }

size_t blink_workspace_size(const blink_problem* p, int32_t call) {
  if (validate_problem(p, call) != BLINK_OK) return 0;
  const long long n_img = (long long)p->n_time * p->n_chan;
  return carve(p, call, default_chunk(p, call, n_img), nullptr, nullptr);
}

blink_status blink_grid(const blink_problem* p, const blink_inputs* in, blink_c32* grid,
                        int32_t* counts, float* weight_sum, int32_t* n_dropped, void* workspace,
                        size_t ws_bytes, blink_stream_t stream) {
  blink_status e = validate_problem(p, BLINK_CALL_GRID);
  if (e != BLINK_OK) return e;
  if ((e = validate_inputs(p, in)) != BLINK_OK) return e;
  const long long n_img = (long long)p->n_time * p->n_chan;
  if (n_img > 0 && !grid) return BLINK_E_ARG;
  if (n_img == 0) return BLINK_OK;
  int chunk = 0;
  if ((e = check_ws(p, BLINK_CALL_GRID, workspace, ws_bytes, &chunk)) != BLINK_OK) return e;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Work w{};
  carve(p, BLINK_CALL_GRID, chunk, static_cast<char*>(workspace), &w);
  run_sort(p, in, w, st);
  ImgArgs a = make_args(p, in, w);
  a.grid = reinterpret_cast<float2*>(grid);
  a.counts = counts;
  a.weight_sum = weight_sum;
  a.n_dropped = n_dropped;
#define BLINK_GRID_CALL(n) grid_n<n>(p, a, chunk, st)
  BLINK_DISPATCH_N(p->grid_n, BLINK_GRID_CALL)
#undef BLINK_GRID_CALL
}

blink_status blink_fft2d(const blink_c32* in, blink_c32* out, int32_t batch, int32_t n,
                         int32_t sign, blink_stream_t stream) {
  if (!in || !out) return BLINK_E_ARG;
  if (sign != 1 && sign != -1) return BLINK_E_ARG;
  if (batch < 0 || n < 1) return BLINK_E_SIZE;
  if (!n_supported(n)) return BLINK_E_UNSUPPORTED;
  if (batch == 0) return BLINK_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const float2* i = reinterpret_cast<const float2*>(in);
  float2* o = reinterpret_cast<float2*>(out);
#define BLINK_FFT_CALL(N_) fft2d_n<N_>(i, o, batch, sign, st)
  BLINK_DISPATCH_N(n, BLINK_FFT_CALL)
#undef BLINK_FFT_CALL
}

static blink_status image_batch_impl(const blink_problem* p, const blink_inputs* in, float* images,
                                     float* weight_sum, void* workspace, size_t ws_bytes,
                                     blink_stream_t stream, Timer* tm) {
  blink_status e = validate_problem(p, BLINK_CALL_IMAGE);
  if (e != BLINK_OK) return e;
  if ((e = validate_inputs(p, in)) != BLINK_OK) return e;
  const long long n_img = (long long)p->n_time * p->n_chan;
  if (n_img > 0 && !images) return BLINK_E_ARG;
  if (n_img == 0) return BLINK_OK;
  int chunk = 0;
  if ((e = check_ws(p, BLINK_CALL_IMAGE, workspace, ws_bytes, &chunk)) != BLINK_OK) return e;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  tm->st = st;
  Work w{};
  carve(p, BLINK_CALL_IMAGE, chunk, static_cast<char*>(workspace), &w);
  const int sorted = run_sort(p, in, w, st, tm, true);
  if (p->n_bl > 0 && !(sorted & SORTED_VMAX)) {
    tm->begin(0);
    hipLaunchKernelGGL(k_vmax, dim3((unsigned)p->n_time), dim3(256), 0, st, w.sv, w.counters + p->n_time,
                       p->n_bl, w.vmax);
    tm->end();
  }
  ImgArgs a = make_args(p, in, w);
  if (p->n_bl == 0) a.vmax = nullptr;
  a.images = images;
  a.weight_sum = weight_sum;
#define BLINK_IMAGE_CALL(n) image_n<n>(p, a, chunk, st, tm, sorted)
  BLINK_DISPATCH_N(p->grid_n, BLINK_IMAGE_CALL)
#undef BLINK_IMAGE_CALL
}

blink_status blink_image_batch(const blink_problem* p, const blink_inputs* in, float* images,
                               float* weight_sum, void* workspace, size_t ws_bytes,
                               blink_stream_t stream) {
  Timer off;
  return image_batch_impl(p, in, images, weight_sum, workspace, ws_bytes, stream, &off);
}

blink_status blink_image_batch_timed(const blink_problem* p, const blink_inputs* in,
                                     float* images, float* weight_sum, void* workspace,
                                     size_t ws_bytes, blink_stream_t stream,
                                     blink_kernel_times* times) {
  if (!times) return BLINK_E_ARG;
  Timer tm;
  tm.on = true;
  blink_status e = image_batch_impl(p, in, images, weight_sum, workspace, ws_bytes, stream, &tm);
  const blink_status c = tm.collect(times);
  return e != BLINK_OK ? e : c;
}

}  // extern "C"

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
blink_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return BLINK_E_HIP;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return BLINK_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (noalloc_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return BLINK_E_HIP;
    noalloc_ptr[dev] = ptr;
  }
  *out = noalloc_ptr[dev];
  return BLINK_OK;
}

// Workspace bytes of an image call on tb timesteps of p with `chunk` images
// per internal chunk.
size_t block_need(const blink_problem* p, int tb, int chunk) {
  blink_problem q = *p;
  q.n_time = tb;
  return carve(&q, BLINK_CALL_IMAGE, chunk, nullptr, nullptr);
}

// Splits the cube into blocks of whole timesteps whose workspace fits the
// scratch array and picks the largest chunk that fits with them. Returns
// false when one timestep with a chunk of one image does not fit.
bool plan_noalloc(const blink_problem* p, int* tb, int* chunk) {
  const size_t cap = BLINK_NOALLOC_SCRATCH_BYTES;
  const size_t per_img = (size_t)(p->grid_n / 2) * (size_t)p->out_n * 8;   // half spectrum of one image
  int t = p->n_time;
  while (t > 1 && block_need(p, t, 1) > cap) t = (t + 1) / 2;
  if (block_need(p, t, 1) > cap) return false;
  const size_t fixed = block_need(p, t, 0);
  long long ch = (long long)((cap - fixed) / (per_img + 255));   // al() adds at most 255 bytes
  ch = std::min<long long>(ch, (long long)t * p->n_chan);
  ch = std::min<long long>(ch, MAX_GRID_Y);
  if (p->chunk_images > 0) ch = std::min<long long>(ch, p->chunk_images);
  ch = std::max<long long>(ch, 1);
  while (ch > 1 && block_need(p, t, (int)ch) > cap) --ch;
  *tb = t;
  *chunk = (int)ch;
  return true;
}

}  // namespace

extern "C" {

blink_status blink_image_batch_noalloc(const blink_problem* p, const blink_inputs* in, float* images,
                                       float* weight_sum, blink_stream_t stream) {
  blink_status e = validate_problem(p, BLINK_CALL_IMAGE);
  if (e != BLINK_OK) return e;
  if ((e = validate_inputs(p, in)) != BLINK_OK) return e;
  const long long n_img = (long long)p->n_time * p->n_chan;
  if (n_img > 0 && !images) return BLINK_E_ARG;
  if (n_img == 0) return BLINK_OK;
  int tb = 0, chunk = 0;
  if (!plan_noalloc(p, &tb, &chunk)) return BLINK_E_WORKSPACE;
  void* ws = nullptr;
  if ((e = scratch_address(&ws)) != BLINK_OK) return e;
  const size_t B = (size_t)p->n_bl, C = (size_t)p->n_chan, MM = (size_t)p->out_n * p->out_n;
  const size_t vsz = p->vis_type == BLINK_VIS_C64 ? 8 : 4;
  blink_problem q = *p;
  q.chunk_images = chunk;
  for (int t0 = 0; t0 < p->n_time; t0 += tb) {
    q.n_time = std::min(tb, p->n_time - t0);
    const size_t i0 = (size_t)t0 * C;                      // first image of the block
    blink_inputs s = *in;
    s.vis = static_cast<const char*>(in->vis) + i0 * B * vsz;
    s.uvw_m = in->uvw_m + (size_t)t0 * B * 3;
    if (in->flags) s.flags = in->flags + (size_t)t0 * B;
    Timer off;
    e = image_batch_impl(&q, &s, images + i0 * MM, weight_sum ? weight_sum + i0 : nullptr, ws,
                         BLINK_NOALLOC_SCRATCH_BYTES, stream, &off);
    if (e != BLINK_OK) return e;
  }
  return BLINK_OK;
}

blink_status blink_degrid_adjoint(const blink_problem* p, const blink_inputs* in,
                                  const float* image_grad, const float* weight_sum,
                                  blink_c32* vis_grad, blink_c32* gain_grad, void* workspace,
                                  size_t ws_bytes, blink_stream_t stream) {
  blink_status e = validate_problem(p, BLINK_CALL_ADJOINT);
  if (e != BLINK_OK) return e;
  if ((e = validate_inputs(p, in)) != BLINK_OK) return e;
  const long long n_img = (long long)p->n_time * p->n_chan;
  if (gain_grad && (!in->gains || !in->ant1 || !in->ant2 || p->n_ant < 1)) return BLINK_E_ARG;
  if (n_img > 0 && p->n_bl > 0 && (!image_grad || !vis_grad)) return BLINK_E_ARG;
  int chunk = 0;
  if (n_img > 0 && p->n_bl > 0 &&
      (e = check_ws(p, BLINK_CALL_ADJOINT, workspace, ws_bytes, &chunk)) != BLINK_OK)
    return e;
  if (n_img == 0 || p->n_bl == 0) {
    if (gain_grad && p->n_ant > 0) {
      hipLaunchKernelGGL(k_fill2, dim3(cdiv(p->n_ant, 256)), dim3(256), 0,
                         reinterpret_cast<hipStream_t>(stream),
                         reinterpret_cast<float2*>(gain_grad), (size_t)p->n_ant);
      return launched();
    }
    return BLINK_OK;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Work w{};
  carve(p, BLINK_CALL_ADJOINT, chunk, static_cast<char*>(workspace), &w);
  run_sort(p, in, w, st);
  ImgArgs a = make_args(p, in, w);
  a.image_grad = image_grad;
  a.wsum_in = weight_sum;
  a.vis_grad = reinterpret_cast<float2*>(vis_grad);
  a.gain_grad = reinterpret_cast<float2*>(gain_grad);
#define BLINK_ADJ_CALL(n) adjoint_n<n>(p, a, chunk, st)
  BLINK_DISPATCH_N(p->grid_n, BLINK_ADJ_CALL)
#undef BLINK_ADJ_CALL
}

blink_status blink_dynamic_spectra(const float* images, int32_t n_time, int32_t n_chan, int32_t n_pix,
                                   int32_t ref_mode, int32_t ref_len, const float* ref_image,
                                   float* spectra, blink_stream_t stream) {
  if (n_time < 0 || n_chan < 0 || n_pix < 0 || n_chan > MAX_GRID_Y) return BLINK_E_SIZE;
  if ((double)n_time * n_chan * n_pix > 4.0e18) return BLINK_E_SIZE;
  if (ref_mode < BLINK_REF_NONE || ref_mode > BLINK_REF_MODEL) return BLINK_E_ARG;
  static_assert(BLINK_REF_MAX_LEN <= DS_KMAX, "window beyond the kernel's halo");
  if (ref_mode == BLINK_REF_MEAN && (ref_len < 1 || ref_len > BLINK_REF_MAX_LEN)) return BLINK_E_ARG;
  const long long n = (long long)n_time * n_chan * n_pix;
  if (n == 0) return BLINK_OK;
  if (!images || !spectra) return BLINK_E_ARG;
  if (ref_mode == BLINK_REF_MODEL && !ref_image) return BLINK_E_ARG;
  const int k = ref_mode == BLINK_REF_MEAN ? ref_len : 0;
  const long long npt8 = ((n_pix + DS_PP - 1) / DS_PP + 7) / 8 * 8;   // pixel tiles, padded to 8
  const long long ntt = (n_time + DS_TT - 1) / DS_TT;
  const long long wgs = npt8 * ntt * n_chan;
  if (wgs > INT32_MAX) return BLINK_E_SIZE;
  const dim3 g((unsigned)wgs);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool vec = n_pix % 4 == 0 && n_time % 4 == 0 && ((uintptr_t)images % 16) == 0 &&
                   ((uintptr_t)spectra % 16) == 0;
  if (vec)
    hipLaunchKernelGGL((k_dynspec<true>), g, dim3(DS_THREADS), dynspec_lds(k, n_time), st, images, (int)n_time,
                       (int)n_chan, (long long)n_pix, (int)ref_mode, k, ref_image, spectra, (int)npt8);
  else
    hipLaunchKernelGGL((k_dynspec<false>), g, dim3(DS_THREADS), dynspec_lds(k, n_time), st, images, (int)n_time,
                       (int)n_chan, (long long)n_pix, (int)ref_mode, k, ref_image, spectra, (int)npt8);
  return launched();
}

blink_status blink_correlate(const int8_t* volt, int32_t n_time, int32_t n_chan, int32_t n_ant,
                             int32_t n_samp, blink_c32* vis, float* autos, blink_stream_t stream) {
  if (n_time < 0 || n_chan < 0 || n_ant < 0 || n_samp < 0) return BLINK_E_SIZE;
  const long long nimg = (long long)n_time * n_chan;
  if (nimg == 0) return BLINK_OK;
  if (n_ant < 2 || n_samp % 16 != 0 || n_samp > XE_MAX_SAMPLES) return BLINK_E_SIZE;
  if ((double)nimg * n_ant * n_samp * 2 > 4.0e18) return BLINK_E_SIZE;
  if (!vis || (n_samp > 0 && !volt)) return BLINK_E_ARG;
  if ((uintptr_t)volt % 16 != 0) return BLINK_E_ARG;
  XeArgs a{};
  a.volt = volt;
  a.vis = reinterpret_cast<float2*>(vis);
  a.autos = autos;
  a.T = n_time; a.C = n_chan; a.A = n_ant; a.S = n_samp;
  a.nt = (n_ant + XE_TILE - 1) / XE_TILE;
  a.npairs = a.nt * (a.nt + 1) / 2;
  a.nimg = nimg;
  const long long wgs = (nimg + 7) / 8 * 8 * a.npairs;
  if (wgs > INT32_MAX) return BLINK_E_SIZE;
  // (n_samp = 0 runs no step and writes zeros)
  hipLaunchKernelGGL(k_xengine, dim3((unsigned)wgs), dim3(WAVE), 0, reinterpret_cast<hipStream_t>(stream), a);
  return launched();
}

}  // extern "C"
