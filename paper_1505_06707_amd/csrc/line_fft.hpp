// Stockham FFT along one "line" (a row or a column of the grid) with the
// line spread over many threads, data in registers between stages and LDS
// exchanges in between.
//
// A line of N = R0 * RR^K points (RR = 4 or 8) is owned by TPL = N/P threads; thread t holds
// element t + TPL*s in register slot s (s < P).  This is the layout in which
// rows and columns are loaded from and stored to HBM, in which the first stage
// reads its inputs and in which the last stage leaves its outputs (natural
// order).  Stage 0 has radix R0 (2, 3, 4, 6 or 8) and no twiddles; stages 1..K have
// radix RR and run in a rolled loop with the stride NS = R0 RR^(s-1) as a
// runtime value, so the code of a whole transform stays small.
//
// Stockham indexing for a stage of radix R and stride NS: butterfly j takes
// elements j + m N/R (slots b + m P/R of thread t when j = t + TPL b),
// multiplies input m by w^(m (j mod NS)) with w = exp(-+2 pi i/(NS R)), and
// writes output m to element (j/NS) NS R + j mod NS + m NS.  The last stage has
// NS R = N and writes back into the same slots.
//
// Forward = sum_j x_j exp(-2 pi i jk/N), inverse = sum_j x_j exp(+2 pi i jk/N);
// neither is scaled.
#pragma once
#include "cx.hpp"

namespace sofft {

// N = R0 * RR^K with RR = 4; P points per thread (a multiple of R0 and of
// RR).  PAD is the LDS padding period (one spare element per PAD), chosen so
// that the stride-R0 writes of stage 0 do not collide in LDS banks; 0 means no
// padding.
template <int N> struct Shape;
// Radix-4 stages, no LDS padding (measured faster than one pad element per R0).
template <> struct Shape<16>   { static constexpr int P = 4,  R0 = 4, RR = 4, K = 1, PAD = 0; };
template <> struct Shape<32>   { static constexpr int P = 4,  R0 = 2, RR = 4, K = 2, PAD = 0; };
template <> struct Shape<64>   { static constexpr int P = 4,  R0 = 4, RR = 4, K = 2, PAD = 0; };
template <> struct Shape<128>  { static constexpr int P = 4,  R0 = 2, RR = 4, K = 3, PAD = 0; };
template <> struct Shape<256>  { static constexpr int P = 4,  R0 = 4, RR = 4, K = 3, PAD = 0; };
template <> struct Shape<512>  { static constexpr int P = 4,  R0 = 2, RR = 4, K = 4, PAD = 0; };
template <> struct Shape<1024> { static constexpr int P = 4,  R0 = 4, RR = 4, K = 4, PAD = 0; };
template <> struct Shape<2048> { static constexpr int P = 4,  R0 = 2, RR = 4, K = 5, PAD = 0; };
template <> struct Shape<4096> { static constexpr int P = 4,  R0 = 4, RR = 4, K = 5, PAD = 0; };
template <> struct Shape<48>   { static constexpr int P = 12, R0 = 3, RR = 4, K = 2, PAD = 0; };
template <> struct Shape<96>   { static constexpr int P = 12, R0 = 6, RR = 4, K = 2, PAD = 6; };
template <> struct Shape<192>  { static constexpr int P = 12, R0 = 3, RR = 4, K = 3, PAD = 0; };
template <> struct Shape<384>  { static constexpr int P = 12, R0 = 6, RR = 4, K = 3, PAD = 6; };
template <> struct Shape<768>  { static constexpr int P = 12, R0 = 3, RR = 4, K = 4, PAD = 0; };

// The same shape data at run time (host side), for table building.
struct ShapeInfo {
  int P, R0, RR, K;
};
template <int N>
constexpr ShapeInfo shape_info_of() {
  return {Shape<N>::P, Shape<N>::R0, Shape<N>::RR, Shape<N>::K};
}
inline ShapeInfo shape_info(long n) {
  switch (n) {
    case 16: return shape_info_of<16>();
    case 32: return shape_info_of<32>();
    case 48: return shape_info_of<48>();
    case 64: return shape_info_of<64>();
    case 96: return shape_info_of<96>();
    case 128: return shape_info_of<128>();
    case 192: return shape_info_of<192>();
    case 256: return shape_info_of<256>();
    case 384: return shape_info_of<384>();
    case 512: return shape_info_of<512>();
    case 768: return shape_info_of<768>();
    case 1024: return shape_info_of<1024>();
    case 2048: return shape_info_of<2048>();
    case 4096: return shape_info_of<4096>();
    default: return {0, 0, 0, 0};
  }
}

// Twiddle tables, one per rolled stage s = 1..K (stride NS_s = R0 RR^(s-1)),
// laid out contiguously so that the lanes of a wave read consecutive entries:
// entry (s, m, k) = exp(-2 pi i m k N/(RR NS_s) / N) for m = 1..RR-1,
// k < NS_s, at offset_s + (m-1) NS_s + k.  In total N - R0 entries.

// LDS elements of the exchange buffer of one line.
template <int N>
constexpr int fft_lds_elems() {
  return Shape<N>::PAD ? N + N / Shape<N>::PAD : N;
}

// Line storage in LDS.  Element e of this thread's line lives at
// lds[base + e*es] for plain use, and at lds[base + (e + e/PAD)*es] for the
// FFT exchanges.
template <typename T>
struct LineLDS {
  cx<T>* lds;
  int base;
  int es;
  __device__ __forceinline__ cx<T>& operator[](int e) const { return lds[base + e * es]; }
  template <int PAD>
  __device__ __forceinline__ cx<T>& padded(int e) const {
    if constexpr (PAD == 0) {
      return lds[base + e * es];
    } else {
      return lds[base + (e + e / PAD) * es];
    }
  }
};

template <int SIGN>
__device__ __forceinline__ cx<double> twiddle_mul(cx<double> a, cx<double> w) {
  return SIGN < 0 ? cmul(a, w) : cmulc(a, w);
}

// The butterflies, twiddles and registers are FP64 for every state type; the
// LDS exchange buffer has element type X (double, or float for a complex64
// state, which then rounds once per stage output).  FP32 butterflies with
// FP32 twiddles were measured to drift linearly with the number of time steps:
// a rounded twiddle is the same operator error in every step, and adding its
// residual after the rounded product does not remove it.

// Twiddles of one rolled stage (stride ns = R0 << sh) for this thread's B =
// P/RR butterflies: w[b][m-1] = tws[(m-1) ns + (j mod ns)], j = t + TPL b.
template <int N>
__device__ __forceinline__ void stage_twiddle_load(cx<double> (&w)[Shape<N>::P / Shape<N>::RR][Shape<N>::RR - 1],
                                                   const cx<double>* __restrict__ tws, int t, int sh) {
  constexpr int P = Shape<N>::P, R0 = Shape<N>::R0, RR = Shape<N>::RR, TPL = N / P, B = P / RR;
  if constexpr ((R0 & (R0 - 1)) == 0) {
    // Power-of-two lines: j mod ns by a mask, and unsigned 32-bit byte offsets
    // from the table base, so the loads take the scalar-base form without
    // 64-bit address arithmetic per lane.
    const unsigned ns = unsigned(R0) << sh;
    const char* base = reinterpret_cast<const char*>(tws);
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const unsigned k = (unsigned(t) + TPL * b) & (ns - 1);
#pragma unroll
      for (int m = 1; m < RR; ++m)
        w[b][m - 1] = *reinterpret_cast<const cx<double>*>(base + (((m - 1) * ns + k) << 4));
    }
  } else {
    const int ns = R0 << sh;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + TPL * b;
      const int k = j - ((j >> sh) / R0) * ns;
#pragma unroll
      for (int m = 1; m < RR; ++m) w[b][m - 1] = tws[(m - 1) * ns + k];
    }
  }
}

// One rolled stage of radix RR with stride ns = R0 << sh (sh = log2(RR) (s-1));
// w holds this stage's twiddles (stage_twiddle_load).
// XM: the write of element e goes to e ^ xm (the swizzled exchanges of fft2).
template <typename X, int N, int SIGN, bool LAST, bool XM = false>
__device__ __forceinline__ void rolled_stage(cx<double> (&v)[Shape<N>::P], const LineLDS<X>& L, int t,
                                             const cx<double> (&w)[Shape<N>::P / Shape<N>::RR][Shape<N>::RR - 1],
                                             int sh, int xm = 0) {
  constexpr int P = Shape<N>::P, R0 = Shape<N>::R0, RR = Shape<N>::RR, TPL = N / P, B = P / RR;
  constexpr int PAD = Shape<N>::PAD;
  const int ns = R0 << sh;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + TPL * b;
    const int q = (j >> sh) / R0;
    const int k = j - q * ns;
    cx<double> a[RR];
#pragma unroll
    for (int m = 0; m < RR; ++m) a[m] = v[b + m * B];
#pragma unroll
    for (int m = 1; m < RR; ++m) a[m] = twiddle_mul<SIGN>(a[m], w[b][m - 1]);
    DFT<RR, SIGN, double>::run(a);
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < RR; ++m) v[b + m * B] = a[m];
    } else {
      const int o = q * RR * ns + k;
#pragma unroll
      for (int m = 0; m < RR; ++m) {
        if constexpr (XM)
          L[(o + m * ns) ^ xm] = narrow<X>(a[m]);
        else
          L.template padded<PAD>(o + m * ns) = narrow<X>(a[m]);
      }
    }
  }
}

// In-place transform of the line held in v.  Every thread of the block must
// call it (it contains block barriers, or wavefront barriers with WAVE).  The twiddles of each rolled stage are
// fetched one stage ahead, so their latency hides behind the LDS exchange.
// Barrier between the LDS exchanges of a line: the whole block, or only the
// wavefront (WAVE) when the caller guarantees that every line lies within one
// wavefront, so that no exchange crosses wavefronts.
template <bool WAVE>
__device__ __forceinline__ void line_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename X, int N, int SIGN, bool WAVE = false>
__device__ __forceinline__ void fft(cx<double> (&v)[Shape<N>::P], const LineLDS<X>& L, int t,
                                    const cx<double>* __restrict__ tw) {
  constexpr int P = Shape<N>::P, R0 = Shape<N>::R0, RR = Shape<N>::RR, K = Shape<N>::K;
  constexpr int TPL = N / P, PAD = Shape<N>::PAD;
  constexpr int LR = RR == 4 ? 2 : (RR == 8 ? 3 : 4);   // log2(RR)
  static_assert(P % R0 == 0 && P % RR == 0, "bad shape");
  cx<double> w[P / RR][RR - 1];
  stage_twiddle_load<N>(w, tw, t, 0);
  {  // stage 0: radix R0, stride 1, no twiddles
    constexpr int B = P / R0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + TPL * b;
      cx<double> a[R0];
#pragma unroll
      for (int m = 0; m < R0; ++m) a[m] = v[b + m * B];
      DFT<R0, SIGN, double>::run(a);
#pragma unroll
      for (int m = 0; m < R0; ++m) L.template padded<PAD>(j * R0 + m) = narrow<X>(a[m]);
    }
    line_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = widen(L.template padded<PAD>(t + TPL * s));
    line_sync<WAVE>();
  }
  int off = 0;
#pragma unroll 1
  for (int sh = 0; sh < LR * (K - 1); sh += LR) {
    rolled_stage<X, N, SIGN, false>(v, L, t, w, sh);
    off += (RR - 1) * (R0 << sh);
    stage_twiddle_load<N>(w, tw + off, t, sh + LR);   // next stage
    line_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = widen(L.template padded<PAD>(t + TPL * s));
    line_sync<WAVE>();
  }
  rolled_stage<X, N, SIGN, true>(v, L, t, w, LR * (K - 1));
}

// The same transform with two exchange buffers, L and Lb, used alternately:
// a buffer is written again only two exchanges later, after a barrier every
// thread passed once done reading it, so the barrier that follows each read
// is dropped; one barrier at the end leaves both buffers free for the caller.
//
// SWZ (lines contiguous in LDS, radix-4 shapes with R0 = 4 and at least 64
// threads per line): the first two exchanges store element e at
// e ^ 5 ((e >> 4) & 3).  Their writes go to 4t + m (stage 0) and
// 16 (t >> 2) + (t & 3) + 4m (first rolled stage), which put the 16 lanes of
// a group on 4 of the 16 bank slots of 16 bytes; swizzled they cover all 16,
// and the reads at t + TPL s stay conflict-free (the swizzle permutes within
// aligned groups of 16 elements).  Both masks depend on t alone: (e >> 4) & 3
// is (t >> 2) & 3 for those writes and (t >> 4) & 3 for the reads.
template <typename X, int N, int SIGN, bool WAVE = false, bool SWZ = false>
__device__ __forceinline__ void fft2(cx<double> (&v)[Shape<N>::P], const LineLDS<X>& L, const LineLDS<X>& Lb,
                                     int t, const cx<double>* __restrict__ tw) {
  constexpr int P = Shape<N>::P, R0 = Shape<N>::R0, RR = Shape<N>::RR, K = Shape<N>::K;
  constexpr int TPL = N / P, PAD = Shape<N>::PAD;
  constexpr int LR = RR == 4 ? 2 : (RR == 8 ? 3 : 4);
  static_assert(!SWZ || (P == 4 && R0 == 4 && RR == 4 && PAD == 0 && TPL >= 64 && K >= 2), "swizzle shape");
  const int xw = SWZ ? ((t >> 2) & 3) * 5 : 0;
  const int tr = SWZ ? (t ^ (((t >> 4) & 3) * 5)) : t;
  cx<double> w[P / RR][RR - 1];
  stage_twiddle_load<N>(w, tw, t, 0);
  {
    constexpr int B = P / R0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + TPL * b;
      cx<double> a[R0];
#pragma unroll
      for (int m = 0; m < R0; ++m) a[m] = v[b + m * B];
      DFT<R0, SIGN, double>::run(a);
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        if constexpr (SWZ)
          L[(j * R0 + m) ^ xw] = narrow<X>(a[m]);
        else
          L.template padded<PAD>(j * R0 + m) = narrow<X>(a[m]);
      }
    }
    line_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < P; ++s) {
      if constexpr (SWZ)
        v[s] = widen(L[tr + TPL * s]);
      else
        v[s] = widen(L.template padded<PAD>(t + TPL * s));
    }
  }
  int off = 0;
  bool odd = true;
  constexpr int sh0 = SWZ ? LR : 0;
  if constexpr (SWZ) {   // the first rolled stage (stride R0), swizzled
    rolled_stage<X, N, SIGN, false, true>(v, Lb, t, w, 0, xw);
    off += (RR - 1) * R0;
    stage_twiddle_load<N>(w, tw + off, t, LR);
    line_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = widen(Lb[tr + TPL * s]);
    odd = false;
  }
  // Unrolled, each stage's stride is a compile-time constant (shifts and LDS
  // offsets fold into immediates); the longest lines keep one rolled copy,
  // whose unrolled form spills.
  constexpr int kStageUnroll = N > 2048 ? 1 : K;
#pragma unroll kStageUnroll
  for (int sh = sh0; sh < LR * (K - 1); sh += LR) {
    const LineLDS<X>& Lx = odd ? Lb : L;
    rolled_stage<X, N, SIGN, false>(v, Lx, t, w, sh);
    off += (RR - 1) * (R0 << sh);
    stage_twiddle_load<N>(w, tw + off, t, sh + LR);
    line_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = widen(Lx.template padded<PAD>(t + TPL * s));
    odd = !odd;
  }
  rolled_stage<X, N, SIGN, true>(v, L, t, w, LR * (K - 1));
  line_sync<WAVE>();
}

// Whether fft2 may swizzle a line of N points held contiguously in LDS.
template <int N>
constexpr bool fft2_swizzle() {
  return Shape<N>::P == 4 && Shape<N>::R0 == 4 && Shape<N>::RR == 4 && Shape<N>::PAD == 0 && N / 4 >= 64 &&
         Shape<N>::K >= 2;
}

// Copy the stage twiddle tables (N entries) from global memory to LDS (all
// threads of the block cooperate; a barrier must follow).
template <int N>
__device__ __forceinline__ void stage_twiddles(cx<double>* dst, const cx<double>* __restrict__ src) {
  for (int u = threadIdx.x; u < N; u += blockDim.x) dst[u] = src[u];
}

}  // namespace sofft
