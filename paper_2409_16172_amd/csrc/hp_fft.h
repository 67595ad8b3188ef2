// Device-side FFT engine for gfx950: register-resident Stockham transforms.
//
// A transform of length N (power of two) is computed by T = N/E threads, each
// holding E elements in registers.  On entry and on exit thread j holds the
// elements j + T*s, s = 0..E-1, of its line, so that loads and stores of a
// wavefront touch consecutive addresses (or consecutive row segments of a
// column tile).  Each radix-R stage performs E/R butterflies per thread; the
// data is exchanged through LDS between stages (autosort, no bit reversal),
// and the last stage writes its outputs straight back into the same registers.
//
// Sign convention: forward uses exp(-2 pi i jk/N), inverse exp(+2 pi i jk/N),
// both unnormalised; the Fourier transform of the paper (Eqn. FT) fixes the
// forward sign.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hp {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.re * s, a.im * s}; }

// exp(2 pi i m / 16) for m = 0..15 (real and imaginary parts).
__host__ __device__ constexpr double cos16(int m) {
  constexpr double c1 = 0.92387953251128675613;   // cos(pi/8)
  constexpr double c2 = 0.70710678118654752440;   // cos(pi/4)
  constexpr double c3 = 0.38268343236508977173;   // cos(3pi/8)
  constexpr double t[16] = {1.0, c1, c2, c3, 0.0, -c3, -c2, -c1, -1.0, -c1, -c2, -c3, 0.0, c3, c2, c1};
  return t[m & 15];
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m - 4); }

// Multiply by the constant w = exp(DIR * 2 pi i k / N), N <= 16, with the trivial
// cases folded at compile time.
template <typename R, int N, int K, int DIR>
__device__ __forceinline__ cpx<R> twc(cpx<R> a) {
  constexpr int m = ((K * (16 / N)) % 16 + 16) % 16;      // angle index on the 16-grid
  constexpr int md = DIR > 0 ? m : (16 - m) % 16;
  if constexpr (md == 0) return a;
  else if constexpr (md == 4) return {-a.im, a.re};        // * i
  else if constexpr (md == 8) return {-a.re, -a.im};
  else if constexpr (md == 12) return {a.im, -a.re};       // * -i
  else if constexpr (md == 2 || md == 6 || md == 10 || md == 14) {
    constexpr R h = (R)0.70710678118654752440;
    constexpr R cr = (md == 2 || md == 14) ? h : -h;
    constexpr R ci = (md == 2 || md == 6) ? h : -h;
    // (a.re + i a.im)(cr + i ci) with |cr| = |ci| = h
    return {h * ((cr > 0 ? a.re : -a.re) - (ci > 0 ? a.im : -a.im)),
            h * ((ci > 0 ? a.re : -a.re) + (cr > 0 ? a.im : -a.im))};
  } else {
    constexpr R cr = (R)cos16(md), ci = (R)sin16(md);
    return {a.re * cr - a.im * ci, a.re * ci + a.im * cr};
  }
}

// In-register DFT of size N <= 16 by radix-2 decimation in time.
// in[i] -> out[k] = sum_i in[i] exp(DIR 2 pi i ik / N).
template <typename R, int N, int DIR>
struct Dft {
  __device__ __forceinline__ static void run(const cpx<R>* in, cpx<R>* out) {
    if constexpr (N == 1) {
      out[0] = in[0];
    } else if constexpr (N == 2) {
      out[0] = cadd(in[0], in[1]);
      out[1] = csub(in[0], in[1]);
    } else {
      constexpr int H = N / 2;
      cpx<R> ev[H], od[H], E[H], O[H];
#pragma unroll
      for (int i = 0; i < H; ++i) { ev[i] = in[2 * i]; od[i] = in[2 * i + 1]; }
      Dft<R, H, DIR>::run(ev, E);
      Dft<R, H, DIR>::run(od, O);
      combine<0>(E, O, out);
    }
  }
  template <int K>
  __device__ __forceinline__ static void combine(const cpx<R>* E, const cpx<R>* O, cpx<R>* out) {
    if constexpr (K < N / 2) {
      cpx<R> o = twc<R, N, K, DIR>(O[K]);
      out[K] = cadd(E[K], o);
      out[K + N / 2] = csub(E[K], o);
      combine<K + 1>(E, O, out);
    }
  }
};

// LDS index of element p of a line between two stages (a stage writes runs of
// elements NS apart, the next reads elements T apart).  Chosen with the gfx950
// bank-conflict counters over every exchange of the transforms below:
//  * 16-byte elements (FP64 complex): p xor ((p >> 3) & 7), a permutation inside
//    aligned groups of eight; no conflicts at any line length or interleave,
//    where one pad element every E left a two-way conflict on each read of an
//    exchange (1024^2 FP64 symbol pass 85.6 -> 80.3 us, combine 64.8 -> 62.7 us);
//  * 8-byte elements (FP32 complex): one pad element every E elements.  It is
//    conflict free in the column passes; the xor map inside groups of sixteen
//    would also clear the row passes, but its address arithmetic pushes the FP32
//    symbol and combine passes past 256 registers (1024^2 mixed apply 108 ->
//    167 us).
// Both maps send [0, n) into [0, lds_elems_e(n)) one to one.
template <int ES, int E>
__device__ __forceinline__ int lidx(int p) {
  if constexpr (ES == 16) return p ^ ((p >> 3) & 7);
  else return p + p / E;
}
template <int E>
__host__ __device__ constexpr int lds_elems_e(int n) { return n + n / E; }

// Elements per thread (fewer for tiny transforms).
#ifndef HP_E64
#define HP_E64 8
#endif
#ifndef HP_E32
#define HP_E32 16
#endif
template <typename R>
__host__ __device__ constexpr int elems_per_thread(int n) {
  return n < (sizeof(R) == 8 ? HP_E64 : HP_E32) ? n : (sizeof(R) == 8 ? HP_E64 : HP_E32);
}

// Synchronisation between the LDS write and read of an exchange.  When every
// transform lives inside one wavefront (its T threads are consecutive and T
// divides 64) the wavefront's own ordering of LDS operations suffices, with
// fences that keep the compiler from moving LDS accesses across.
template <bool WAVE>
__device__ __forceinline__ void xsync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    // workgroup barrier ordering LDS only: global loads issued before it (e.g. the
    // next node's data or twiddles) stay in flight
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
}

// Returns p unchanged, but hides its value from the optimiser (an empty asm
// statement with side effects).  Twiddle loads addressed through it can be
// neither hoisted out of a loop nor scheduled ahead of an earlier stage, so only
// one stage's twiddles are live at a time.
// The pointer must address global memory; it goes through the asm as a
// global-address-space pointer so that the loads stay global (not flat) loads.
template <typename T>
__device__ __forceinline__ const T* reload_each_time(const T* p) {
  using GP = const __attribute__((address_space(1))) T*;
  GP g = (GP)p;
  asm volatile("" : "+s"(g));
  return (const T*)g;
}

// Exchange between lanes l and l ^ 32 of a wavefront (v_permlane32_swap): lanes
// 0-31 keep a and receive into b the a of lanes 32-63; lanes 32-63 keep b and
// receive into a the b of lanes 0-31.  All 64 lanes must be active.
__device__ __forceinline__ void lane_swap32(double& a, double& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
  b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}
// An FP32 complex value goes through as one 64-bit word (its re and im as the two
// halves), the same instruction pattern as an FP64 value: with each float bit-cast
// on its own, this compiler kept the first result for both outputs.
__device__ __forceinline__ void lane_swap32(cpx<float>& a, cpx<float>& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(cpx<float>, ((unsigned long long)hi[0] << 32) | lo[0]);
  b = __builtin_bit_cast(cpx<float>, ((unsigned long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void lane_swap32(cpx<double>& a, cpx<double>& b) {
  lane_swap32(a.re, b.re);
  lane_swap32(a.im, b.im);
}
// The same between lanes l and l ^ 16 (v_permlane16_swap): lanes with bit 4 clear
// keep a and receive into b the a of lane l + 16; the others keep b and receive
// into a the b of lane l - 16.
__device__ __forceinline__ void lane_swap16(double& a, double& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
  b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void lane_swap16(cpx<float>& a, cpx<float>& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(cpx<float>, ((unsigned long long)hi[0] << 32) | lo[0]);
  b = __builtin_bit_cast(cpx<float>, ((unsigned long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void lane_swap16(cpx<double>& a, cpx<double>& b) {
  lane_swap16(a.re, b.re);
  lane_swap16(a.im, b.im);
}
template <int D, typename R>
__device__ __forceinline__ void lane_swap(cpx<R>& a, cpx<R>& b) {
  static_assert(D == 16 || D == 32, "lane distance");
  if constexpr (D == 32) lane_swap32(a, b);
  else lane_swap16(a, b);
}

// Which exchange before the last stage of a length-N transform with E elements
// per thread can go through lanes: 2 when the last stage has radix 2 and the one
// before it radix E (thread j trades half its elements with thread j ^ T/2), 4
// when the last has radix 4 after one of radix E (threads j, j ^ T/4, j ^ T/2,
// j ^ 3T/4 trade a quarter with each other), else 0.
template <int N, int E>
__host__ __device__ constexpr int lane_exchange_kind() {
  int ns = 1, prev = 0, r = 0;
  while (ns < N) {
    prev = r;
    r = (N / ns) < E ? (N / ns) : E;
    ns *= r;
  }
  if (prev != E) return 0;
  return (r == 2 || r == 4) ? r : 0;
}

template <int N, int NS, int E>
__host__ __device__ constexpr int stage_radix() {
  return (N / NS) < E ? (N / NS) : E;
}

// One Stockham stage of radix R at sub-transform size NS, then the next stage.
// tw: table of exp(-2 pi i m / N), m < N.
// ILV: several transforms share one LDS array with their elements interleaved
// (element p of transform g at lidx(p) * ILV + g; the caller passes lds + g),
// so that lanes of neighbouring transforms touch neighbouring banks.
// SWP (0, 16 or 32): the exchange before the last stage goes through lanes
// instead of LDS when lane_exchange_kind says it can.  With thread j = h (T/K) + L,
// K the last radix, L < T/K, after the stage before the last thread j holds the
// positions h N/K + L + (T/K) t, t < E, and needs L + (T/K)(h + K s), s < E.
//  * K = 2: it keeps the t of its own parity (h) and trades the rest with thread
//    j ^ T/2, which the caller places at lane ^ SWP of the same wavefront, with
//    h = 0 on the lanes whose bit log2(SWP) is clear.
//  * K = 4 (SWP = 32): threads h = 0..3 of one L sit at lanes differing in bits 5
//    (h bit 1) and 4 (h bit 0); a trade over lane bit 5 of the t with t mod 4 in
//    {2, 3} (or {0, 1}) and then one over lane bit 4 of the odd (even) t leave each
//    thread the E/4 elements t = h + 4c of every h', which belong at s = (E/4) h' + c.
// In both cases the element a lane keeps sits in the register it keeps, so the
// trades need no per-lane selects, and the final order is a fixed renaming.
template <typename R, int N, int E, int DIR, int NS, bool WAVE, int ILV, bool RELOAD = false, int SWP = 0>
struct Stage {
  __device__ __forceinline__ static void run(cpx<R> (&x)[E], cpx<R>* lds, int j, const cpx<R>* __restrict__ tw) {
    if constexpr (RELOAD && NS > 1) tw = reload_each_time(tw);
    constexpr int RS = stage_radix<N, NS, E>();
    constexpr int B = E / RS;
    constexpr int T = N / E;
    constexpr bool last = (NS * RS == N);
    constexpr int lxk = lane_exchange_kind<N, E>();
    constexpr bool swap2 = SWP != 0 && !last && lxk == 2 && 2 * NS * RS == N;
    constexpr bool swap4 = SWP == 32 && !last && lxk == 4 && 4 * NS * RS == N;
    constexpr bool swap_next = swap2 || swap4;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int b = j + T * i;
      cpx<R> in[RS], out[RS];
#pragma unroll
      for (int t = 0; t < RS; ++t) in[t] = x[i + B * t];
      const int k = (NS > 1) ? (b % NS) : 0;
      if constexpr (NS > 1) {
#pragma unroll
        for (int t = 1; t < RS; ++t) {
          cpx<R> w = tw[k * t * (N / (NS * RS))];
          in[t] = DIR < 0 ? cmul(in[t], w) : cmulc(in[t], w);
        }
      }
      Dft<R, RS, DIR>::run(in, out);
      if constexpr (last) {
#pragma unroll
        for (int t = 0; t < RS; ++t) x[i + B * t] = out[t];
      } else if constexpr (swap2) {
#pragma unroll
        for (int u = 0; u < E / 2; ++u) {
          cpx<R> a = out[2 * u], c = out[2 * u + 1];
          lane_swap<SWP>(a, c);
          x[u] = a;
          x[u + E / 2] = c;
        }
      } else if constexpr (swap4) {
#pragma unroll
        for (int t = 0; t < E; ++t)
          if (t % 4 < 2) lane_swap32(out[t], out[t + 2]);
#pragma unroll
        for (int t = 0; t < E; t += 2) lane_swap16(out[t], out[t + 1]);
#pragma unroll
        for (int t = 0; t < E; ++t) x[t] = out[(t % (E / 4)) * 4 + t / (E / 4)];
      } else {
        const int base = (b / NS) * NS * RS + k;
#pragma unroll
        for (int t = 0; t < RS; ++t) lds[lidx<sizeof(cpx<R>), E>(base + t * NS) * ILV] = out[t];
      }
    }
    if constexpr (swap_next) {
      Stage<R, N, E, DIR, NS * RS, WAVE, ILV, RELOAD, SWP>::run(x, lds, j, tw);
    } else if constexpr (!last) {
      xsync<WAVE>();
#pragma unroll
      for (int s = 0; s < E; ++s) x[s] = lds[lidx<sizeof(cpx<R>), E>(j + T * s) * ILV];
      xsync<WAVE>();
      Stage<R, N, E, DIR, NS * RS, WAVE, ILV, RELOAD, SWP>::run(x, lds, j, tw);
    }
  }
};

template <typename R>
__host__ __device__ constexpr int lds_elems(int n) { return lds_elems_e<elems_per_thread<R>(8192)>(n); }

// Full transform.  All threads of the workgroup must call it together (it
// contains workgroup barriers when N > E, unless CONTIG says that the T threads
// of a transform are consecutive, in which case transforms of at most 64
// threads synchronise within their wavefront only).
// fft_e takes the elements per thread E explicitly (LDS: lds_elems_e<E>(N) per transform).
// RELOAD: each stage reads its twiddles through reload_each_time (wave-resident
// lines of many elements per lane, whose registers cannot hold every stage's).
// SWP: the exchange before the last stage goes through lanes where it can (see Stage).
template <typename R, int N, int E, int DIR, bool CONTIG = false, int ILV = 1, bool RELOAD = false, int SWP = 0>
__device__ __forceinline__ void fft_e(cpx<R> (&x)[E], cpx<R>* lds, int j, const cpx<R>* __restrict__ tw) {
  constexpr int T = N / E;
  Stage<R, N, E, DIR, 1, CONTIG && (T <= 64), ILV, RELOAD, SWP>::run(x, lds, j, tw);
}
template <typename R, int N, int DIR, bool CONTIG = false, int ILV = 1>
__device__ __forceinline__ void fft(cpx<R> (&x)[elems_per_thread<R>(N)], cpx<R>* lds, int j,
                                    const cpx<R>* __restrict__ tw) {
  fft_e<R, N, elems_per_thread<R>(N), DIR, CONTIG, ILV>(x, lds, j, tw);
}

}  // namespace hp
