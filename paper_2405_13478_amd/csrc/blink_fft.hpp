// Device-side FFT building blocks for gfx950: small DFT codelets in registers
// and a self-sorting (Stockham) mixed-radix transform of one length-N vector
// held in LDS and processed by a single 64-lane wavefront.
//
// The 2D inverse transform of the dirty image (Sec. 4.3 Eq. 6, Sec. 5.2.2) is
// evaluated as column transforms followed by row transforms built from these.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace blink {

constexpr int WAVE = 64;

template <int V>
using ic = std::integral_constant<int, V>;

// f(ic<B>{}), f(ic<B + 1>{}), ..., f(ic<E - 1>{}): a loop whose index is a
// compile-time constant in the body.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * (SIGN * i)
template <int SIGN>
__device__ __forceinline__ float2 mul_si(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// a * (c + SIGN * i * s)
template <int SIGN>
__device__ __forceinline__ float2 mul_cs(float2 a, float c, float s) {
  const float ss = SIGN > 0 ? s : -s;
  return make_float2(a.x * c - a.y * ss, a.x * ss + a.y * c);
}

// LDS index padding: one spare element every 16 keeps the strided accesses
// of the Stockham stages off a single bank group.
__device__ __forceinline__ constexpr int pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4) + 4; }

// Orders this wavefront's LDS reads before its later LDS writes (and vice
// versa). LDS executes one wavefront's DS instructions in issue order, so a
// compiler-level fence at wavefront scope is all that is needed.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- codelets
// X[k] = sum_n x[n] exp(SIGN 2 pi i n k / R), in place on v[0..R).
namespace kc {
constexpr float R2 = 0.70710678118654752440f;   // cos(pi/4)
constexpr float C8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float S8 = 0.38268343236508977173f;   // sin(pi/8)
constexpr float S3 = 0.86602540378443864676f;   // sin(2 pi/3)
constexpr float C51 = 0.30901699437494742410f;  // cos(2 pi/5)
constexpr float S51 = 0.95105651629515357212f;  // sin(2 pi/5)
constexpr float C52 = -0.80901699437494742410f; // cos(4 pi/5)
constexpr float S52 = 0.58778525229247312917f;  // sin(4 pi/5)
}  // namespace kc

template <int SIGN>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int SIGN>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const float2 s13 = cadd(a1, a3), d13 = mul_si<SIGN>(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

template <int SIGN>
__device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
  const float2 s = cadd(a1, a2);
  const float2 d = mul_si<SIGN>(csub(a1, a2));
  const float2 m = make_float2(a0.x - 0.5f * s.x, a0.y - 0.5f * s.y);
  a0 = cadd(a0, s);
  a1 = make_float2(m.x + kc::S3 * d.x, m.y + kc::S3 * d.y);
  a2 = make_float2(m.x - kc::S3 * d.x, m.y - kc::S3 * d.y);
}

template <int SIGN>
__device__ __forceinline__ void dft5(float2* a) {
  const float2 s14 = cadd(a[1], a[4]), d14 = mul_si<SIGN>(csub(a[1], a[4]));
  const float2 s23 = cadd(a[2], a[3]), d23 = mul_si<SIGN>(csub(a[2], a[3]));
  const float2 x0 = a[0];
  const float2 p1 = make_float2(x0.x + kc::C51 * s14.x + kc::C52 * s23.x, x0.y + kc::C51 * s14.y + kc::C52 * s23.y);
  const float2 p2 = make_float2(x0.x + kc::C52 * s14.x + kc::C51 * s23.x, x0.y + kc::C52 * s14.y + kc::C51 * s23.y);
  const float2 q1 = make_float2(kc::S51 * d14.x + kc::S52 * d23.x, kc::S51 * d14.y + kc::S52 * d23.y);
  const float2 q2 = make_float2(kc::S52 * d14.x - kc::S51 * d23.x, kc::S52 * d14.y - kc::S51 * d23.y);
  a[0] = make_float2(x0.x + s14.x + s23.x, x0.y + s14.y + s23.y);
  a[1] = cadd(p1, q1);
  a[4] = csub(p1, q1);
  a[2] = cadd(p2, q2);
  a[3] = csub(p2, q2);
}

// radix 8 as 4 x 2: x[2 n1 + n2] -> DFT4 over n1, twiddle w8^(n2 k1), DFT2 over n2
template <int SIGN>
__device__ __forceinline__ void dft8(float2* a) {
  dft4<SIGN>(a[0], a[2], a[4], a[6]);
  dft4<SIGN>(a[1], a[3], a[5], a[7]);
  a[3] = mul_cs<SIGN>(a[3], kc::R2, kc::R2);
  a[5] = mul_si<SIGN>(a[5]);
  a[7] = mul_cs<SIGN>(a[7], -kc::R2, kc::R2);
  float2 b[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    b[k1] = cadd(a[2 * k1], a[2 * k1 + 1]);
    b[k1 + 4] = csub(a[2 * k1], a[2 * k1 + 1]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = b[i];
}

// Complex add / subtract of operands that may be known zero at compile time
// (ZA: a is zero, ZB: b is zero): the known-zero terms cost nothing.
template <bool ZA, bool ZB>
__device__ __forceinline__ float2 zadd(float2 a, float2 b) {
  if constexpr (ZA && ZB) return make_float2(0.f, 0.f);
  else if constexpr (ZA) return b;
  else if constexpr (ZB) return a;
  else return cadd(a, b);
}
template <bool ZA, bool ZB>
__device__ __forceinline__ float2 zsub(float2 a, float2 b) {
  if constexpr (ZA && ZB) return make_float2(0.f, 0.f);
  else if constexpr (ZA) return make_float2(-b.x, -b.y);
  else if constexpr (ZB) return a;
  else return csub(a, b);
}

// dft4 with inputs Z0..Z3 known to be zero
template <int SIGN, bool Z0, bool Z1, bool Z2, bool Z3>
__device__ __forceinline__ void dft4z(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = zadd<Z0, Z2>(a0, a2), d02 = zsub<Z0, Z2>(a0, a2);
  const float2 s13 = zadd<Z1, Z3>(a1, a3), d13 = mul_si<SIGN>(zsub<Z1, Z3>(a1, a3));
  constexpr bool ZS = Z0 && Z2, ZD = Z1 && Z3;
  a0 = zadd<ZS, ZD>(s02, s13);
  a2 = zsub<ZS, ZD>(s02, s13);
  a1 = zadd<ZS, ZD>(d02, d13);
  a3 = zsub<ZS, ZD>(d02, d13);
}

// radix 16 as 4 x 4: x[4 n1 + n2] -> DFT4 over n1, twiddle w16^(n2 k1), DFT4 over n2.
// ZB: the inputs x[8 - ZB/2 .. 8 + ZB/2) are known to be zero (a transform's
// first stage whose middle input rows are empty); they are neither read nor
// added. Every other term is added exactly as in the full codelet, so the
// outputs are the same numbers.
template <int SIGN, int ZB = 0>
__device__ __forceinline__ void dft16(float2* a) {
  static_assert(ZB % 2 == 0 && ZB >= 0 && ZB <= 8, "zero band of the radix-16 codelet");
  constexpr int zlo = 8 - ZB / 2, zhi = 8 + ZB / 2;
  static_for<0, 4>([&](auto nc) {
    constexpr int n2 = decltype(nc)::value;
    dft4z<SIGN, (n2 >= zlo && n2 < zhi), (n2 + 4 >= zlo && n2 + 4 < zhi), (n2 + 8 >= zlo && n2 + 8 < zhi),
          (n2 + 12 >= zlo && n2 + 12 < zhi)>(a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]);
  });
  // a[n2 + 4 k1] now holds DFT4 output k1 of column n2; twiddle by w16^(n2 k1)
  a[5] = mul_cs<SIGN>(a[5], kc::C8, kc::S8);      // n2=1 k1=1 : w^1
  a[9] = mul_cs<SIGN>(a[9], kc::R2, kc::R2);      // n2=1 k1=2 : w^2
  a[13] = mul_cs<SIGN>(a[13], kc::S8, kc::C8);    // n2=1 k1=3 : w^3
  a[6] = mul_cs<SIGN>(a[6], kc::R2, kc::R2);      // n2=2 k1=1 : w^2
  a[10] = mul_si<SIGN>(a[10]);                    // n2=2 k1=2 : w^4
  a[14] = mul_cs<SIGN>(a[14], -kc::R2, kc::R2);   // n2=2 k1=3 : w^6
  a[7] = mul_cs<SIGN>(a[7], kc::S8, kc::C8);      // n2=3 k1=1 : w^3
  a[11] = mul_cs<SIGN>(a[11], -kc::R2, kc::R2);   // n2=3 k1=2 : w^6
  a[15] = mul_cs<SIGN>(a[15], -kc::C8, -kc::S8);  // n2=3 k1=3 : w^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<SIGN>(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
  // a[4 k1 + k2] holds X[k1 + 4 k2]: transpose into natural order
  float2 b[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) b[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = b[i];
}

template <int R, int SIGN, int ZB = 0>
__device__ __forceinline__ void dft(float2* a) {
  static_assert(ZB == 0 || R == 16, "zero band only in the radix-16 codelet");
  if constexpr (R == 2) dft2<SIGN>(a[0], a[1]);
  else if constexpr (R == 3) dft3<SIGN>(a[0], a[1], a[2]);
  else if constexpr (R == 4) dft4<SIGN>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 5) dft5<SIGN>(a);
  else if constexpr (R == 8) dft8<SIGN>(a);
  else if constexpr (R == 16) dft16<SIGN, ZB>(a);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------- plans
__host__ __device__ constexpr int pick_radix(int rem) {
  return rem % 16 == 0 ? 16 : rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 2 == 0 ? 2
       : rem % 5 == 0 ? 5 : rem % 3 == 0 ? 3 : 0;
}
__host__ __device__ constexpr bool plan_ok(int n) {
  if (n < 2) return false;
  while (n > 1) {
    const int r = pick_radix(n);
    if (r == 0) return false;
    n /= r;
  }
  return true;
}

// Twiddles of the stages: one table per stage after the first, laid out
// [(r - 1) * NS + k] = w_{NS R}^(k r), concatenated in stage order, so that for
// a fixed r the lanes of a wavefront read consecutive entries.
__host__ __device__ constexpr int tw_entries_before(int n, int ns) {
  int total = 0, cur = 1;
  while (cur < ns) {
    const int r = pick_radix(n / cur);
    if (cur > 1) total += (r - 1) * cur;
    cur *= r;
  }
  return total;
}
__host__ __device__ constexpr int tw_entries(int n) { return tw_entries_before(n, n); }

// One Stockham stage of radix R after NS points have been combined:
// butterfly j reads x[j + r N/R], twiddles by w_{NS R}^(SIGN (j mod NS) r),
// applies the length-R DFT and writes y[(j / NS) NS R + (j mod NS) + r NS].
// (Self-sorting radix-R formulation of the Stockham FFT; output in natural
// order after the last stage.) In place on buf; one wavefront per vector.
//
// Padded LDS addresses: when a stride is a multiple of 16 the padded index of
// base + r * stride is pad(base) + r * (stride + stride / 16), and for NS = 1
// with R dividing 16 it is pad(j R) + r, so every access is a per-lane base
// plus a compile-time offset that folds into the LDS instruction.
// Second half of a stage: twiddle, DFT and write of the butterflies whose
// inputs v[p][r] = x[j + r N/R] (j = lane + 64 p) are already in registers.
template <int N, int R, int NS, int SIGN>
__device__ __forceinline__ void stockham_stage_regs(float2* buf, int lane, const float2* __restrict__ tw,
                                                    float2 (&v)[(N / R + WAVE - 1) / WAVE][R]) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + WAVE - 1) / WAVE;
  constexpr bool WR_LIN = NS % 16 == 0 || (NS == 1 && 16 % R == 0);   // write offsets fold
  constexpr int WR_STEP = NS == 1 ? 1 : NS + NS / 16;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = lane + p * WAVE;
    if (NB % WAVE == 0 || j < NB) {
      const int k = j % NS;
      if constexpr (NS > 1) {
        constexpr int TW0 = tw_entries_before(N, NS);             // folded at compile time
        const float2* t1 = tw + TW0 + k;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = t1[(r - 1) * NS];
          if (SIGN < 0) w.y = -w.y;
          v[p][r] = cmul(v[p][r], w);
        }
      }
      dft<R, SIGN>(v[p]);
      const int base = (j / NS) * NS * R + k;
      if constexpr (WR_LIN) {
        const int b = pad(base);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[b + r * WR_STEP] = v[p][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pad(base + r * NS)] = v[p][r];
      }
    }
  }
  wave_sync();
}

template <int N, int R, int NS, int SIGN>
__device__ __forceinline__ void stockham_stage(float2* buf, int lane, const float2* __restrict__ tw) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + WAVE - 1) / WAVE;
  constexpr bool RD_LIN = NB % 16 == 0;                       // read offsets fold
  constexpr int RD_STEP = NB + NB / 16;
  float2 v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = lane + p * WAVE;
    if (NB % WAVE == 0 || j < NB) {
      if constexpr (RD_LIN) {
        const int b = pad(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[b + r * RD_STEP];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[pad(j + r * NB)];
      }
    }
  }
  wave_sync();
  stockham_stage_regs<N, R, NS, SIGN>(buf, lane, tw, v);
}

// Last stage of the transform with the outputs handed to emit(ic<QB>, X)
// from registers instead of being written back to LDS. Each call covers the
// wavefront's block of consecutive frequencies q = QB + lane, QB a
// compile-time constant (lanes beyond the stage's butterflies are inactive),
// so global stores stay coalesced and the caller can decide per block with
// wave-uniform tests.
template <int N, int R, int NS, int SIGN, class Emit>
__device__ __forceinline__ void stockham_last_emit(float2* buf, int lane, const float2* __restrict__ tw,
                                                   Emit&& emit) {
  static_assert(NS * R == N, "last stage");
  constexpr int NB = N / R;
  constexpr int PER = (NB + WAVE - 1) / WAVE;
  constexpr bool RD_LIN = NB % 16 == 0;
  constexpr int RD_STEP = NB + NB / 16;
  float2 v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = lane + p * WAVE;
    if (NB % WAVE == 0 || j < NB) {
      if constexpr (RD_LIN) {
        const int b = pad(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[b + r * RD_STEP];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[pad(j + r * NB)];
      }
    }
  }
  static_for<0, PER>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    const int j = lane + p * WAVE;
    if (NB % WAVE == 0 || j < NB) {
      if constexpr (NS > 1) {
        constexpr int TW0 = tw_entries_before(N, NS);
        const float2* t1 = tw + TW0 + j;                          // k = j in the last stage
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = t1[(r - 1) * NS];
          if (SIGN < 0) w.y = -w.y;
          v[p][r] = cmul(v[p][r], w);
        }
      }
      dft<R, SIGN>(v[p]);
      static_for<0, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        emit(ic<p * WAVE + r * NS>{}, v[p][r]);
      });
    }
  });
}

// base[i] = v with the byte offset formed in 32 bits, so that the store can
// take a scalar base address and a 32-bit per-lane offset (i * sizeof(T) must
// stay below 4 GiB).
template <class T>
__device__ __forceinline__ void store_at(T* base, unsigned i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)) = v;
}

// Centred cutout of a length-N spectrum: frequency q goes to position q + hm
// if q < hm, to q - (N - hm) if q >= N - hm, and is dropped otherwise (2 hm
// kept points; output position hm holds frequency 0). For the block
// q = QB + lane the tests are wave-uniform unless the block straddles a
// boundary; st(pos) performs the store. Positions are unsigned so that the
// store can address a scalar base plus a 32-bit lane offset.
template <int N, int QB, class Store>
__device__ __forceinline__ void cutout_block(unsigned lane, int hm, Store&& st) {
  if (QB + WAVE <= hm) {
    st((unsigned)(QB + hm) + lane);
  } else if (QB >= N - hm) {
    st((unsigned)(QB - (N - hm)) + lane);
  } else if (QB < hm || QB + WAVE > N - hm) {
    const int q = QB + (int)lane;
    if (q < hm) st((unsigned)(q + hm));
    else if (q >= N - hm) st((unsigned)(q - (N - hm)));
    // keeps the compiler from merging these per-lane stores with the block
    // stores above, which would turn their scalar offsets into per-lane ones
    asm volatile("" ::: "memory");
  }
}

// Per-lane form of the same cutout (no block tests): fewest registers.
template <int N, int QB, class Store>
__device__ __forceinline__ void cutout_lane(unsigned lane, int hm, Store&& st) {
  const int q = QB + (int)lane;
  if (q < hm || q >= N - hm) st((unsigned)(q < hm ? q + hm : q - (N - hm)));
}

// Stride of the last stage of the length-n plan (the NS it is entered with).
__host__ __device__ constexpr int last_stage_ns(int n) {
  int cur = 1;
  while (n / cur / pick_radix(n / cur) > 1) cur *= pick_radix(n / cur);
  return cur;
}
// Compact last stage: when the plan ends in a radix-4 stage after NS > 1
// points, only its r = 1 twiddles w^k are kept (a prefix of the table) and
// w^2k, w^3k are formed from them in registers. Saves 2 NS table entries.
__host__ __device__ constexpr bool compact_last(int n) {
  return last_stage_ns(n) > 1 && pick_radix(n / last_stage_ns(n)) == 4;
}
__host__ __device__ constexpr int tw_entries_compact(int n) {
  return compact_last(n) ? tw_entries_before(n, last_stage_ns(n)) + last_stage_ns(n) : tw_entries(n);
}
// True when every emitted block q = QB + lane of the last stage starts at a
// multiple of the wavefront width and has all lanes active.
__host__ __device__ constexpr bool blocks_aligned(int n) {
  return plan_ok(n) && last_stage_ns(n) % WAVE == 0 && (n / pick_radix(n / last_stage_ns(n))) % WAVE == 0;
}

// Cutout store for blocks aligned to the wavefront width with hm a multiple
// of it as well: each block is wholly kept or wholly dropped.
template <int N, int QB, class Store>
__device__ __forceinline__ void cutout_block_aligned(unsigned lane, int hm, Store&& st) {
  static_assert(QB % WAVE == 0, "block not aligned");
  if (QB < hm) st((unsigned)(QB + hm) + lane);
  else if (QB >= N - hm) st((unsigned)(QB - (N - hm)) + lane);
}

// Whole transform with the last stage emitting (see stockham_last_emit). The
// buffer is left holding the input of the last stage.
template <int N, int SIGN, int NS = 1, class Emit>
__device__ __forceinline__ void wave_fft_emit(float2* buf, int lane, const float2* __restrict__ tw,
                                              Emit&& emit) {
  constexpr int R = pick_radix(N / NS);
  static_assert(R != 0, "length not supported by the radix set");
  if constexpr (NS * R == N) {
    stockham_last_emit<N, R, NS, SIGN>(buf, lane, tw, emit);
  } else {
    stockham_stage<N, R, NS, SIGN>(buf, lane, tw);
    wave_fft_emit<N, SIGN, NS * R>(buf, lane, tw, emit);
  }
}

// ------------------------------------------------- half-length exchange
// The same transform with every stage-to-stage exchange passing through a
// buffer of N/2 points (padded) instead of N, in two rounds: the outputs of
// index below N/2 first, then the rest. A Stockham stage's output
// y[(j / NS) NS R + (j mod NS) + r NS] lies below N/2 exactly when its
// butterfly j is below NB / 2 (NS R divides N/2 for every stage but the last),
// and the next stage's input x[j + r N/R] lies below N/2 exactly when r < R/2.
// So each round writes the outputs of one half of the butterflies and reads
// one half of every next butterfly's inputs; the lower-half writes and the
// upper-half reads are at padded index minus pad(N/2), which is a
// compile-time offset on the read side. Halving the LDS of a transform lets
// twice as many wavefronts share a CU; the arithmetic and its order are those
// of the full-buffer stages.
__host__ __device__ constexpr bool plan_even(int n) {
  if (n < 2 || n % 32 != 0) return false;
  while (n > 1) {
    const int r = pick_radix(n);
    if (r == 0 || r % 2 != 0) return false;
    n /= r;
  }
  return true;
}

// Twiddle and DFT of the butterflies held in registers (no LDS traffic).
template <int N, int R, int NS, int SIGN, int ZB = 0, bool CL = false>
__device__ __forceinline__ void stage_compute(int lane, const float2* __restrict__ tw,
                                              float2 (&v)[(N / R + WAVE - 1) / WAVE][R]) {
  static_assert(ZB == 0 || NS == 1, "a zero band only on the first stage's inputs");
  constexpr int NB = N / R;
  constexpr int PER = (NB + WAVE - 1) / WAVE;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = lane + p * WAVE;
    if (NB % WAVE == 0 || j < NB) {
      if constexpr (NS > 1) {
        constexpr int TW0 = tw_entries_before(N, NS);
        const float2* t1 = tw + TW0 + j % NS;
        if constexpr (CL && NS * R == N && R == 4) {      // compact last stage
          float2 w1 = t1[0];
          if (SIGN < 0) w1.y = -w1.y;
          const float2 w2 = cmul(w1, w1);
          v[p][1] = cmul(v[p][1], w1);
          v[p][2] = cmul(v[p][2], w2);
          v[p][3] = cmul(v[p][3], cmul(w1, w2));
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = t1[(r - 1) * NS];
            if (SIGN < 0) w.y = -w.y;
            v[p][r] = cmul(v[p][r], w);
          }
        }
      }
      dft<R, SIGN, ZB>(v[p]);
    }
  }
}

// Round HF of a stage's writes: outputs of the butterflies j in
// [HF NB/2, (HF + 1) NB/2) to hbuf at padded index - HF pad(N/2).
template <int N, int R, int NS, int HF>
__device__ __forceinline__ void half_write(float2* hbuf, int lane, const float2 (&v)[(N / R + WAVE - 1) / WAVE][R]) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + WAVE - 1) / WAVE;
  constexpr int HB = NB / 2;
  constexpr int PH = pad(N / 2);
  constexpr bool WR_LIN = NS % 16 == 0 || (NS == 1 && 16 % R == 0);
  constexpr int WR_STEP = NS == 1 ? 1 : NS + NS / 16;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = lane + p * WAVE;
    bool in;
    if constexpr (HB % WAVE == 0) in = HF == 0 ? p * WAVE < HB : p * WAVE >= HB;   // whole registers
    else in = HF == 0 ? j < HB : (j >= HB && j < NB);
    if (in) {
      const int base = (j / NS) * NS * R + j % NS;
      if constexpr (WR_LIN) {
        const int b = pad(base) - HF * PH;
#pragma unroll
        for (int r = 0; r < R; ++r) hbuf[b + r * WR_STEP] = v[p][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) hbuf[pad(base + r * NS) - HF * PH] = v[p][r];
      }
    }
  }
}

// Round HF of a stage's reads: inputs r in [HF R/2, (HF + 1) R/2), except
// those in the zero band [R/2 - ZB/2, R/2 + ZB/2) (first stage only), which
// the codelet treats as zero and which are not read.
template <int N, int R, int HF, int ZB = 0>
__device__ __forceinline__ void half_read(const float2* hbuf, int lane, float2 (&v)[(N / R + WAVE - 1) / WAVE][R]) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + WAVE - 1) / WAVE;
  constexpr bool RD_LIN = NB % 16 == 0;
  constexpr int RD_STEP = NB + NB / 16;
  constexpr int PH = pad(N / 2);
  constexpr int zlo = R / 2 - ZB / 2, zhi = R / 2 + ZB / 2;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = lane + p * WAVE;
    if (NB % WAVE == 0 || j < NB) {
      if constexpr (RD_LIN) {
        const int b = pad(j);
#pragma unroll
        for (int r = HF * R / 2; r < (HF + 1) * R / 2; ++r)
          if (r < zlo || r >= zhi) v[p][r] = hbuf[b + (r * RD_STEP - HF * PH)];
      } else {
#pragma unroll
        for (int r = HF * R / 2; r < (HF + 1) * R / 2; ++r)
          if (r < zlo || r >= zhi) v[p][r] = hbuf[pad(j + r * NB) - HF * PH];
      }
    }
  }
}

// Zero bands of the first stage that the transforms are compiled for: the
// inputs of a radix-16 first stage at rows [N/2 - ZB N/32, N/2 + ZB N/32)
// are empty when every nonzero row i satisfies min(i, N - i) < N/2 - ZB N/32.
// Given that bound (the largest min(i, N - i) + 1 of a nonzero row), the
// widest band that applies; 0 when none does or the first radix is not 16.
__host__ __device__ constexpr int zero_band(int n, int bound) {
  if (pick_radix(n) != 16) return 0;
  for (int zb = 6; zb > 0; zb -= 2)
    if (zb != 2 && bound <= n / 2 - zb * (n / 32)) return zb;
  return 0;
}



// The stages from NS on, given the stage's inputs in v; the last stage hands
// its outputs to emit(ic<QB>, X) as stockham_last_emit does.
// ZB: zero band of the first stage's inputs (NS = 1 only; see zero_band).
// CL: the table is compact in its last stage (tw_entries_compact).
template <int N, int SIGN, int NS, int ZB = 0, bool CL = false, class Emit>
__device__ __forceinline__ void half_chain(float2* hbuf, int lane, const float2* __restrict__ tw,
                                           float2 (&v)[(N / pick_radix(N / NS) + WAVE - 1) / WAVE][pick_radix(N / NS)],
                                           Emit&& emit) {
  constexpr int R = pick_radix(N / NS);
  constexpr int PER = (N / R + WAVE - 1) / WAVE;
  stage_compute<N, R, NS, SIGN, ZB, CL>(lane, tw, v);
  if constexpr (NS * R == N) {
    static_for<0, PER>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      if ((N / R) % WAVE == 0 || lane + p * WAVE < N / R) {
        static_for<0, R>([&](auto rc) {
          constexpr int r = decltype(rc)::value;
          emit(ic<p * WAVE + r * NS>{}, v[p][r]);
        });
      }
    });
  } else {
    constexpr int R2 = pick_radix(N / (NS * R));
    float2 v2[(N / R2 + WAVE - 1) / WAVE][R2];
    half_write<N, R, NS, 0>(hbuf, lane, v);
    wave_sync();
    half_read<N, R2, 0>(hbuf, lane, v2);
    wave_sync();
    half_write<N, R, NS, 1>(hbuf, lane, v);
    wave_sync();
    half_read<N, R2, 1>(hbuf, lane, v2);
    wave_sync();
    half_chain<N, SIGN, NS * R, 0, CL>(hbuf, lane, tw, v2, emit);
  }
}

// Registers of the first stage's inputs: v[p][r] = x[lane + 64 p + r N/R0].
template <int N>
struct HalfIn {
  static constexpr int R = pick_radix(N);
  static constexpr int PER = (N / R + WAVE - 1) / WAVE;
  float2 v[PER][R];
};

// ZB: the zero band of the first stage's inputs (see zero_band; the inputs in
// it need not have been read into `in`), 0 for none.
template <int N, int SIGN, int ZB = 0, bool CL = false, class Emit>
__device__ __forceinline__ void wave_fft_half_emit(float2* hbuf, int lane, const float2* __restrict__ tw,
                                                   HalfIn<N>& in, Emit&& emit) {
  static_assert(plan_even(N), "half-length exchange needs even radices");
  half_chain<N, SIGN, 1, ZB, CL>(hbuf, lane, tw, in.v, emit);
}

template <int N, int SIGN, int NS = 1>
__device__ __forceinline__ void wave_fft(float2* buf, int lane, const float2* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS);
    static_assert(R != 0, "length not supported by the radix set");
    stockham_stage<N, R, NS, SIGN>(buf, lane, tw);
    wave_fft<N, SIGN, NS * R>(buf, lane, tw);
  }
}

}  // namespace blink
