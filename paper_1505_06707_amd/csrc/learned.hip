// Learned correction to the FFT preconditioner of Sec. III (not from the
// paper): z = P^-1 r + s N(r/s, P^-1 r/s) with s the root-mean-square of r and
// N three periodic 3x3 convolutions, 4 -> 16 -> 16 -> 2 channels, ReLU after
// the first two.  Activations are FP16 in HBM ([batch][y][x][channel]); the
// forward convolutions run on the matrix cores (v_mfma_f32_16x16x16_f16, FP16
// operands, FP32 accumulation); the backward pass and Adam are FP32 vector
// code.  Weights live as one FP32 master array and are rounded to FP16 where a
// kernel loads them, so forward and backward both see the FP16 values.
//
// Parameter layout (kLpParams floats): W1 [9][16][4], b1 [16], W2 [9][16][16],
// b2 [16], W3 [9][2][16], b3 [2]; tap t = 3 (dy + 1) + (dx + 1) reads the
// input at (y + dy, x + dx), indices periodic.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

struct sofft_plan;

namespace sofft {
Plan& plan_of(sofft_plan* p);

namespace {

constexpr int kOffW1 = 0, kOffB1 = kOffW1 + 9 * 16 * 4, kOffW2 = kOffB1 + 16, kOffB2 = kOffW2 + 9 * 16 * 16,
              kOffW3 = kOffB2 + 16, kOffB3 = kOffW3 + 9 * 2 * 16, kParams = kOffB3 + 2;

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ---------------------------------------------------------------- forward
enum ConvOut : int { kOutReluF16 = 0, kOutF32 = 1, kOutAddZ = 2 };

struct ConvArgs {
  const _Float16* in;      // [B][H][W][CIN]
  const float* params;     // master weights
  int w_off, b_off;
  int H, W;
  const int* active;       // [B] (null: all)
  _Float16* out16;         // [B][H][W][16]      (kOutReluF16)
  float* out32;            // [B][H][W][2]       (kOutF32)
  cx<double>* z;           // [B][H][W]          (kOutAddZ): z += s (y0 + i y1)
  const double* scale;     // [B]                (kOutAddZ)
};

// One wavefront computes 16 consecutive pixels of a row for all output
// channels: D[co][px] = sum over k of A[co][k] B[k][px] with A the weights of
// one tap (co x ci) and B the inputs of that tap (ci x px).  With CIN = 4 one
// MFMA covers four taps (k = 4 (tap - 4 j) + ci).  Lane l supplies A[l % 16]
// [4 (l / 16) .. +3] and B[4 (l / 16) .. +3][l % 16] and receives D[4 (l / 16)
// .. +3][l % 16]: the four output channels 4 (l / 16) .. +3 of pixel l % 16.
template <int CIN, int COUT, int OUT>
__global__ void __launch_bounds__(256) k_lp_conv(ConvArgs a) {
  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int seg = blockIdx.x * 4 + wave;            // 16-pixel segment
  const int segs_per_row = a.W / 16;
  const int y = seg / segs_per_row;
  if (y >= a.H) return;
  const int x0 = (seg - y * segs_per_row) * 16;
  const int n = lane & 15, g = lane >> 4;
  const int px = x0 + n;
  const float* Wt = a.params + a.w_off;
  const size_t plane = size_t(a.H) * a.W;
  const _Float16* in = a.in + size_t(b) * plane * CIN;
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (CIN == 16) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      half4_t A;
      const int co = n;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        A[i] = co < COUT ? _Float16(Wt[(t * COUT + co) * CIN + 4 * g + i]) : _Float16(0.f);
      const size_t pix = size_t(wrap(y + dy, a.H)) * a.W + wrap(px + dx, a.W);
      const half4_t B = *reinterpret_cast<const half4_t*>(in + pix * CIN + 4 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x16f16(A, B, acc, 0, 0, 0);
    }
  } else {
    static_assert(CIN == 4, "CIN must be 4 or 16");
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int t = 4 * j + g;
      half4_t A, B;
      if (t < 9) {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        const int co = n;
#pragma unroll
        for (int i = 0; i < 4; ++i) A[i] = co < COUT ? _Float16(Wt[(t * COUT + co) * CIN + i]) : _Float16(0.f);
        const size_t pix = size_t(wrap(y + dy, a.H)) * a.W + wrap(px + dx, a.W);
        B = *reinterpret_cast<const half4_t*>(in + pix * CIN);
      } else {
        A = half4_t{0, 0, 0, 0};
        B = half4_t{0, 0, 0, 0};
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16f16(A, B, acc, 0, 0, 0);
    }
  }
  const float* bias = a.params + a.b_off;
  const size_t pix = size_t(b) * plane + size_t(y) * a.W + px;
  if constexpr (OUT == kOutReluF16) {
    static_assert(COUT == 16, "hidden layers have 16 channels");
    half4_t o;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = _Float16(fmaxf(acc[i] + bias[4 * g + i], 0.f));
    *reinterpret_cast<half4_t*>(a.out16 + pix * 16 + 4 * g) = o;
  } else {
    static_assert(COUT == 2, "the output layer has 2 channels");
    if (g == 0) {
      const float y0 = acc[0] + bias[0], y1 = acc[1] + bias[1];
      if constexpr (OUT == kOutF32) {
        a.out32[pix * 2] = y0;
        a.out32[pix * 2 + 1] = y1;
      } else {
        const double s = a.scale[b];
        cx<double>& zz = a.z[pix];
        zz = zz + cx<double>{s * double(y0), s * double(y1)};
      }
    }
  }
}

// x0 = (Re r/s, Im r/s, Re pz/s, Im pz/s) as FP16; item b reads pair idx[b]
// (idx null: b) of r and pz.
__global__ void __launch_bounds__(256) k_lp_pack(const cx<double>* r, const cx<double>* pz, const double* scale,
                                                 const int* idx, const int* active, size_t plane, _Float16* x0) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  const int src = idx ? idx[b] : b;
  const double inv = 1.0 / scale[src];
  const cx<double> rv = r[size_t(src) * plane + i], pv = pz[size_t(src) * plane + i];
  half4_t o;
  o[0] = _Float16(rv.re * inv);   // one rounding, FP64 -> FP16
  o[1] = _Float16(rv.im * inv);
  o[2] = _Float16(pv.re * inv);
  o[3] = _Float16(pv.im * inv);
  *reinterpret_cast<half4_t*>(x0 + (size_t(b) * plane + i) * 4) = o;
}

// scale[b] = sqrt(mean |v_b|^2), FP64, one block per item.
__global__ void __launch_bounds__(256) k_lp_rms(const cx<double>* v, size_t plane, double* scale) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < plane; i += 256) {
    const cx<double> u = v[size_t(b) * plane + i];
    acc += u.re * u.re + u.im * u.im;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[b] = sqrt(red[0] / double(plane));
}

// ---------------------------------------------------------------- training
// Loss terms and dL/dy of the output layer: target (e - pz)/s, loss = mean of
// squared differences over items, pixels and both channels.  Partial sums per
// block in part[b][block].
__global__ void __launch_bounds__(256) k_lp_loss(const float* y, const cx<double>* e, const cx<double>* pz,
                                                 const double* scale, const int* idx, size_t plane, double inv_count,
                                                 float* dy, double* part) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < plane) {
    const int src = idx ? idx[b] : b;
    const double inv = 1.0 / scale[src];
    const cx<double> ev = e[size_t(src) * plane + i], pv = pz[size_t(src) * plane + i];
    const size_t o = (size_t(b) * plane + i) * 2;
    const double d0 = double(y[o]) - (ev.re - pv.re) * inv;
    const double d1 = double(y[o + 1]) - (ev.im - pv.im) * inv;
    acc = d0 * d0 + d1 * d1;
    dy[o] = float(2.0 * d0 * inv_count);
    dy[o + 1] = float(2.0 * d1 * inv_count);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + blockIdx.x] = red[0];
}

// dx[q][ci] = (sum over taps and co of W[t][co][ci] dy[q - d_t][co]) * (x[q][ci] > 0),
// FP32, one thread per pixel; x is the layer's (post-ReLU) input.  MASK =
// false (the network's input layer, which has no ReLU before it) leaves the
// gradient unmasked.
template <int CIN, int COUT, bool MASK = true>
__global__ void __launch_bounds__(256) k_lp_bwd_data(const float* dy, const float* params, int w_off,
                                                     const _Float16* x, int H, int W, float* dx) {
  __shared__ float w[9 * COUT * CIN];
  for (int u = threadIdx.x; u < 9 * COUT * CIN; u += blockDim.x) w[u] = float(_Float16(params[w_off + u]));
  __syncthreads();
  const int b = blockIdx.y;
  const size_t plane = size_t(H) * W;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  const int yy = int(i / W), xx = int(i - size_t(yy) * W);
  float acc[CIN];
#pragma unroll
  for (int c = 0; c < CIN; ++c) acc[c] = 0.f;
  for (int t = 0; t < 9; ++t) {
    const int ddy = t / 3 - 1, ddx = t % 3 - 1;
    const size_t q = size_t(b) * plane + size_t(wrap(yy - ddy, H)) * W + wrap(xx - ddx, W);
    float g[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) g[co] = dy[q * COUT + co];
#pragma unroll
    for (int co = 0; co < COUT; ++co)
#pragma unroll
      for (int c = 0; c < CIN; ++c) acc[c] = fmaf(w[(t * COUT + co) * CIN + c], g[co], acc[c]);
  }
  const size_t o = (size_t(b) * plane + i) * CIN;
#pragma unroll
  for (int c = 0; c < CIN; ++c) dx[o + c] = (!MASK || float(x[o + c]) > 0.f) ? acc[c] : 0.f;
}

// Partial weight and bias gradients over a chunk of pixels of every item:
// part[chunk][t][co][ci] = sum dy[p][co] x[p + d_t][ci], then part[chunk]
// [9 COUT CIN + co] = sum dy[p][co].  Thread j < COUT CIN owns (co, ci) for
// all taps; threads j < COUT also sum the bias terms.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_lp_bwd_w(const float* dy, const _Float16* x, int H, int W, int B,
                                                  int chunks, double* part) {
  const int j = threadIdx.x;
  const size_t plane = size_t(H) * W, total = plane * B;
  const size_t per = (total + chunks - 1) / chunks;
  const size_t p0 = per * blockIdx.x, p1 = std::min(total, p0 + per);
  const int co = j / CIN, ci = j - (j / CIN) * CIN;
  double acc[9], bacc = 0.0;
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = 0.0;
  if (j < COUT * CIN) {
    for (size_t p = p0; p < p1; ++p) {
      const size_t b = p / plane, i = p - b * plane;
      const int yy = int(i / W), xx = int(i - size_t(yy) * W);
      const float g = dy[p * COUT + co];
      if (ci == 0) bacc += g;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int ddy = t / 3 - 1, ddx = t % 3 - 1;
        const size_t q = b * plane + size_t(wrap(yy + ddy, H)) * W + wrap(xx + ddx, W);
        acc[t] += double(g) * double(float(x[q * CIN + ci]));
      }
    }
    double* out = part + size_t(blockIdx.x) * (9 * COUT * CIN + COUT);
#pragma unroll
    for (int t = 0; t < 9; ++t) out[(t * COUT + co) * CIN + ci] = acc[t];
    if (ci == 0) out[9 * COUT * CIN + co] = bacc;
  }
}

// grad[w_off + u] (weights) and grad[b_off + co] (biases) = sum over chunks.
__global__ void k_lp_reduce(const double* part, int chunks, int nw, int cout, int w_off, int b_off, float* grad) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nw + cout) return;
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) acc += part[size_t(c) * (nw + cout) + u];
  grad[u < nw ? w_off + u : b_off + (u - nw)] = float(acc);
}

// Adam with bias correction (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t).
__global__ void k_lp_adam(float* params, const float* grad, float* m, float* v, int n, float lr, float bc1,
                          float bc2) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const float g = grad[u];
  const float mm = 0.9f * m[u] + 0.1f * g;
  const float vv = 0.999f * v[u] + 0.001f * g * g;
  m[u] = mm;
  v[u] = vv;
  params[u] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

sofft_status alloc(DevBuf& d, size_t bytes) {
  if (d.p && d.bytes >= bytes) return SOFFT_OK;
  dev_free(d);
  if (hipMalloc(&d.p, bytes) != hipSuccess) {
    d.p = nullptr;
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return SOFFT_ENOMEM;
  }
  d.bytes = bytes;
  return SOFFT_OK;
}

}  // namespace

// Network state: master weights, Adam moments and activation buffers.
struct LpNet {
  DevBuf params, grad, m, v;     // owned: allocated by sofft_lp_create
  // views into the caller's workspace (sofft_lp_bind), laid out per call
  DevBuf x0, h1, h2, y3, dy3, dh2, dh1, part, loss_part, scale, pz, idx;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t adam_t = 0;
  std::vector<double> host_loss;
};

namespace {
constexpr int kLpChunks = 256;
size_t r256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

// Workspace of a call on B items of `plane` pixels that may train on npairs
// pairs: activations, gradients, partial sums, the pairs' P^-1 r and scales.
size_t lp_ws_bytes(int B, size_t plane, int64_t npairs) {
  const size_t pb = (plane + 255) / 256;
  const size_t n = size_t(B) * plane;
  return r256(n * 4 * 2) + 2 * r256(n * 16 * 2) + 2 * r256(n * 2 * 4) + 2 * r256(n * 16 * 4) +
         r256(size_t(kLpChunks) * (9 * 16 * 16 + 16) * 8) + r256(size_t(B) * pb * 8) +
         r256(size_t(std::max<int64_t>(B, npairs)) * 8) + r256(size_t(npairs) * plane * 16) + r256(size_t(B) * 4);
}

// Point the per-call buffers into the bound workspace (SOFFT_EWORKSPACE when
// it is missing or smaller than lp_ws_bytes).
sofft_status lp_carve(LpNet& net, int B, size_t plane, int64_t npairs) {
  const size_t need = lp_ws_bytes(B, plane, npairs);
  if (!net.ws || net.ws_bytes < need) {
    set_error("the correction network needs a bound workspace of " + std::to_string(need) +
              " bytes for this call (sofft_lp_workspace_size, sofft_lp_bind); bound: " +
              std::to_string(net.ws ? net.ws_bytes : 0));
    return SOFFT_EWORKSPACE;
  }
  char* q = static_cast<char*>(net.ws);
  auto take = [&](DevBuf& d, size_t b) {
    d.p = q;
    d.bytes = b;
    q += r256(b);
  };
  const size_t pb = (plane + 255) / 256;
  const size_t n = size_t(B) * plane;
  take(net.x0, n * 4 * 2);
  take(net.h1, n * 16 * 2);
  take(net.h2, n * 16 * 2);
  take(net.y3, n * 2 * 4);
  take(net.dy3, n * 2 * 4);
  take(net.dh2, n * 16 * 4);
  take(net.dh1, n * 16 * 4);
  take(net.part, size_t(kLpChunks) * (9 * 16 * 16 + 16) * 8);
  take(net.loss_part, size_t(B) * pb * 8);
  take(net.scale, size_t(std::max<int64_t>(B, npairs)) * 8);
  take(net.pz, size_t(npairs) * plane * 16);
  take(net.idx, size_t(B) * 4);
  return SOFFT_OK;
}

int lp_param_count() { return kParams; }

namespace {

sofft_status forward_layers(LpNet& net, int B, int H, int W, const int* active, int last, cx<double>* z,
                            const double* scale, hipStream_t s) {
  const size_t plane = size_t(H) * W;
  if (W % 16 != 0) {
    set_error("the correction network needs grid widths that are multiples of 16");
    return SOFFT_EUNSUPPORTED;
  }
  const dim3 grid(unsigned((plane / 16 + 3) / 4), unsigned(B));
  ConvArgs a{};
  a.params = static_cast<const float*>(net.params.p);
  a.H = H;
  a.W = W;
  a.active = active;
  a.in = static_cast<const _Float16*>(net.x0.p);
  a.w_off = kOffW1;
  a.b_off = kOffB1;
  a.out16 = static_cast<_Float16*>(net.h1.p);
  k_lp_conv<4, 16, kOutReluF16><<<grid, 256, 0, s>>>(a);
  a.in = static_cast<const _Float16*>(net.h1.p);
  a.w_off = kOffW2;
  a.b_off = kOffB2;
  a.out16 = static_cast<_Float16*>(net.h2.p);
  k_lp_conv<16, 16, kOutReluF16><<<grid, 256, 0, s>>>(a);
  a.in = static_cast<const _Float16*>(net.h2.p);
  a.w_off = kOffW3;
  a.b_off = kOffB3;
  if (last == kOutF32) {
    a.out32 = static_cast<float*>(net.y3.p);
    k_lp_conv<16, 2, kOutF32><<<grid, 256, 0, s>>>(a);
  } else {
    a.z = z;
    a.scale = scale;
    k_lp_conv<16, 2, kOutAddZ><<<grid, 256, 0, s>>>(a);
  }
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

// The buffers of a forward pass (B items) are carved by the entry points.
sofft_status buffers(LpNet& net, int B, size_t plane) {
  if (!net.x0.p || net.x0.bytes < size_t(B) * plane * 4 * 2) {
    set_error("internal: network buffers not carved");
    return SOFFT_EUNSUPPORTED;
  }
  return SOFFT_OK;
}

sofft_status train_buffers(LpNet& net, int B, size_t plane, int chunks) {
  (void)chunks;
  return buffers(net, B, plane);
}

// Loss and gradient of one batch (items idx[b] of r, pz, e; scales per pair).
sofft_status loss_grad(LpNet& net, const cx<double>* r, const cx<double>* pz, const cx<double>* e,
                       const double* scale, const int* idx, int B, int H, int W, hipStream_t s) {
  const size_t plane = size_t(H) * W;
  constexpr int chunks = kLpChunks;
  sofft_status st = train_buffers(net, B, plane, chunks);
  if (st != SOFFT_OK) return st;
  const unsigned pb = unsigned((plane + 255) / 256);
  k_lp_pack<<<dim3(pb, B), 256, 0, s>>>(r, pz, scale, idx, nullptr, plane, static_cast<_Float16*>(net.x0.p));
  SOFFT_HIP_TRY(hipGetLastError());
  if ((st = forward_layers(net, B, H, W, nullptr, kOutF32, nullptr, nullptr, s)) != SOFFT_OK) return st;
  k_lp_loss<<<dim3(pb, B), 256, 0, s>>>(static_cast<const float*>(net.y3.p), e, pz, scale, idx, plane,
                                        1.0 / (double(B) * double(plane) * 2.0), static_cast<float*>(net.dy3.p),
                                        static_cast<double*>(net.loss_part.p));
  const float* P = static_cast<const float*>(net.params.p);
  float* G = static_cast<float*>(net.grad.p);
  double* part = static_cast<double*>(net.part.p);
  // layer 3: dW3 from h2, dh2 = W3^T dy3 masked by h2 > 0
  k_lp_bwd_w<16, 2><<<chunks, 256, 0, s>>>(static_cast<const float*>(net.dy3.p),
                                           static_cast<const _Float16*>(net.h2.p), H, W, B, chunks, part);
  k_lp_reduce<<<(9 * 2 * 16 + 2 + 255) / 256, 256, 0, s>>>(part, chunks, 9 * 2 * 16, 2, kOffW3, kOffB3, G);
  k_lp_bwd_data<16, 2><<<dim3(pb, B), 256, 0, s>>>(static_cast<const float*>(net.dy3.p), P, kOffW3,
                                                   static_cast<const _Float16*>(net.h2.p), H, W,
                                                   static_cast<float*>(net.dh2.p));
  // layer 2
  k_lp_bwd_w<16, 16><<<chunks, 256, 0, s>>>(static_cast<const float*>(net.dh2.p),
                                            static_cast<const _Float16*>(net.h1.p), H, W, B, chunks, part);
  k_lp_reduce<<<(9 * 16 * 16 + 16 + 255) / 256, 256, 0, s>>>(part, chunks, 9 * 16 * 16, 16, kOffW2, kOffB2, G);
  k_lp_bwd_data<16, 16><<<dim3(pb, B), 256, 0, s>>>(static_cast<const float*>(net.dh2.p), P, kOffW2,
                                                    static_cast<const _Float16*>(net.h1.p), H, W,
                                                    static_cast<float*>(net.dh1.p));
  // layer 1 (no input gradient needed)
  k_lp_bwd_w<4, 16><<<chunks, 256, 0, s>>>(static_cast<const float*>(net.dh1.p),
                                           static_cast<const _Float16*>(net.x0.p), H, W, B, chunks, part);
  k_lp_reduce<<<(9 * 16 * 4 + 16 + 255) / 256, 256, 0, s>>>(part, chunks, 9 * 16 * 4, 16, kOffW1, kOffB1, G);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

// Gradients of the network for a given dL/dy of its output (dy3, FP32
// [B][H][W][2]) after a forward pass that left x0, h1, h2: weights and biases
// into net.grad, and dL/dx0 (FP32 [B][H][W][4], unmasked) into dx0.
sofft_status backward_from(LpNet& net, const float* dy3, int B, int H, int W, float* dx0, hipStream_t s) {
  const size_t plane = size_t(H) * W;
  constexpr int chunks = kLpChunks;
  sofft_status st = train_buffers(net, B, plane, chunks);
  if (st != SOFFT_OK) return st;
  const unsigned pb = unsigned((plane + 255) / 256);
  const float* P = static_cast<const float*>(net.params.p);
  float* G = static_cast<float*>(net.grad.p);
  double* part = static_cast<double*>(net.part.p);
  k_lp_bwd_w<16, 2><<<chunks, 256, 0, s>>>(dy3, static_cast<const _Float16*>(net.h2.p), H, W, B, chunks, part);
  k_lp_reduce<<<(9 * 2 * 16 + 2 + 255) / 256, 256, 0, s>>>(part, chunks, 9 * 2 * 16, 2, kOffW3, kOffB3, G);
  k_lp_bwd_data<16, 2><<<dim3(pb, B), 256, 0, s>>>(dy3, P, kOffW3, static_cast<const _Float16*>(net.h2.p), H, W,
                                                   static_cast<float*>(net.dh2.p));
  k_lp_bwd_w<16, 16><<<chunks, 256, 0, s>>>(static_cast<const float*>(net.dh2.p),
                                            static_cast<const _Float16*>(net.h1.p), H, W, B, chunks, part);
  k_lp_reduce<<<(9 * 16 * 16 + 16 + 255) / 256, 256, 0, s>>>(part, chunks, 9 * 16 * 16, 16, kOffW2, kOffB2, G);
  k_lp_bwd_data<16, 16><<<dim3(pb, B), 256, 0, s>>>(static_cast<const float*>(net.dh2.p), P, kOffW2,
                                                    static_cast<const _Float16*>(net.h1.p), H, W,
                                                    static_cast<float*>(net.dh1.p));
  k_lp_bwd_w<4, 16><<<chunks, 256, 0, s>>>(static_cast<const float*>(net.dh1.p),
                                           static_cast<const _Float16*>(net.x0.p), H, W, B, chunks, part);
  k_lp_reduce<<<(9 * 16 * 4 + 16 + 255) / 256, 256, 0, s>>>(part, chunks, 9 * 16 * 4, 16, kOffW1, kOffB1, G);
  k_lp_bwd_data<4, 16, false><<<dim3(pb, B), 256, 0, s>>>(static_cast<const float*>(net.dh1.p), P, kOffW1,
                                                          static_cast<const _Float16*>(net.x0.p), H, W, dx0);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status read_loss(LpNet& net, int B, size_t plane, double* loss, hipStream_t s) {
  const size_t pb = (plane + 255) / 256;
  net.host_loss.resize(size_t(B) * pb);
  SOFFT_HIP_TRY(hipMemcpyAsync(net.host_loss.data(), net.loss_part.p, net.host_loss.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
  SOFFT_HIP_TRY(hipStreamSynchronize(s));
  double acc = 0.0;
  for (double v : net.host_loss) acc += v;
  *loss = acc / (double(B) * double(plane) * 2.0);
  return SOFFT_OK;
}

}  // namespace

// z += s N(r/s, z/s) for the items whose active flag is set (the solver's
// hook: z holds P^-1 r on entry).  scale[b] must hold the rms of r_b.
sofft_status lp_apply(LpNet& net, const cx<double>* r, cx<double>* z, int B, int H, int W, const int* active,
                      const double* scale, hipStream_t s) {
  const size_t plane = size_t(H) * W;
  sofft_status st = buffers(net, B, plane);
  if (st != SOFFT_OK) return st;
  k_lp_pack<<<dim3(unsigned((plane + 255) / 256), B), 256, 0, s>>>(r, z, scale, nullptr, active, plane,
                                                                     static_cast<_Float16*>(net.x0.p));
  SOFFT_HIP_TRY(hipGetLastError());
  return forward_layers(net, B, H, W, active, kOutAddZ, z, scale, s);
}

sofft_status lp_rms(const cx<double>* v, int B, size_t plane, double* scale, hipStream_t s) {
  k_lp_rms<<<B, 256, 0, s>>>(v, plane, scale);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

}  // namespace sofft

using namespace sofft;

struct sofft_lp : public LpNet {};

extern "C" {

sofft_status sofft_lp_create(sofft_lp** out) {
  if (!out) {
    set_error("out is null");
    return SOFFT_EINVAL;
  }
  sofft_lp* lp = new sofft_lp();
  sofft_status st = alloc(lp->params, kParams * sizeof(float));
  if (st == SOFFT_OK) st = alloc(lp->m, kParams * sizeof(float));
  if (st == SOFFT_OK) st = alloc(lp->v, kParams * sizeof(float));
  if (st == SOFFT_OK) st = alloc(lp->grad, kParams * sizeof(float));
  if (st == SOFFT_OK && (hipMemset(lp->params.p, 0, kParams * sizeof(float)) != hipSuccess ||
                         hipMemset(lp->m.p, 0, kParams * sizeof(float)) != hipSuccess ||
                         hipMemset(lp->v.p, 0, kParams * sizeof(float)) != hipSuccess)) {
    set_error("hipMemset failed");
    st = SOFFT_EHIP;
  }
  if (st != SOFFT_OK) {
    for (DevBuf* b : {&lp->params, &lp->m, &lp->v, &lp->grad}) dev_free(*b);
    delete lp;
    return st;
  }
  *out = lp;
  return SOFFT_OK;
}

sofft_status sofft_lp_destroy(sofft_lp* lp) {
  if (!lp) return SOFFT_OK;
  for (DevBuf* b : {&lp->params, &lp->grad, &lp->m, &lp->v}) dev_free(*b);
  delete lp;
  return SOFFT_OK;
}

int32_t sofft_lp_param_count(void) { return kParams; }

sofft_status sofft_lp_set_weights(sofft_lp* lp, const float* host) {
  if (!lp || !host) {
    set_error("bad argument to sofft_lp_set_weights");
    return SOFFT_EINVAL;
  }
  SOFFT_HIP_TRY(hipMemcpy(lp->params.p, host, kParams * sizeof(float), hipMemcpyHostToDevice));
  SOFFT_HIP_TRY(hipMemset(lp->m.p, 0, kParams * sizeof(float)));
  SOFFT_HIP_TRY(hipMemset(lp->v.p, 0, kParams * sizeof(float)));
  lp->adam_t = 0;
  return SOFFT_OK;
}

sofft_status sofft_lp_get_weights(const sofft_lp* lp, float* host) {
  if (!lp || !host) {
    set_error("bad argument to sofft_lp_get_weights");
    return SOFFT_EINVAL;
  }
  SOFFT_HIP_TRY(hipMemcpy(host, lp->params.p, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return SOFFT_OK;
}

sofft_status sofft_lp_forward(sofft_lp* lp, const void* r, const void* pz, int64_t ny, int64_t nx, int32_t batch,
                              float* out, void* stream) {
  if (!lp || !r || !pz || !out || ny <= 0 || nx <= 0 || batch <= 0) {
    set_error("bad argument to sofft_lp_forward");
    return SOFFT_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t plane = size_t(ny) * size_t(nx);
  sofft_status st = lp_carve(*lp, batch, plane, 0);
  if (st != SOFFT_OK) return st;
  double* scale = static_cast<double*>(lp->scale.p);
  const cx<double>* rv = static_cast<const cx<double>*>(r);
  if ((st = lp_rms(rv, batch, plane, scale, s)) != SOFFT_OK) return st;
  k_lp_pack<<<dim3(unsigned((plane + 255) / 256), batch), 256, 0, s>>>(
      rv, static_cast<const cx<double>*>(pz), scale, nullptr, nullptr, plane, static_cast<_Float16*>(lp->x0.p));
  SOFFT_HIP_TRY(hipGetLastError());
  if ((st = forward_layers(*lp, batch, int(ny), int(nx), nullptr, kOutF32, nullptr, nullptr, s)) != SOFFT_OK)
    return st;
  SOFFT_HIP_TRY(hipMemcpyAsync(out, lp->y3.p, size_t(batch) * plane * 2 * sizeof(float), hipMemcpyDeviceToDevice, s));
  return SOFFT_OK;
}

sofft_status sofft_lp_loss_grad(sofft_lp* lp, const void* r, const void* pz, const void* e, int64_t ny, int64_t nx,
                                int32_t batch, float* grad, double* loss, void* stream) {
  if (!lp || !r || !pz || !e || !grad || !loss || ny <= 0 || nx <= 0 || batch <= 0) {
    set_error("bad argument to sofft_lp_loss_grad");
    return SOFFT_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t plane = size_t(ny) * size_t(nx);
  sofft_status st = lp_carve(*lp, batch, plane, 0);
  if (st != SOFFT_OK) return st;
  double* scale = static_cast<double*>(lp->scale.p);
  const cx<double>* rv = static_cast<const cx<double>*>(r);
  if ((st = lp_rms(rv, batch, plane, scale, s)) != SOFFT_OK) return st;
  if ((st = loss_grad(*lp, rv, static_cast<const cx<double>*>(pz), static_cast<const cx<double>*>(e), scale,
                      nullptr, batch, int(ny), int(nx), s)) != SOFFT_OK)
    return st;
  SOFFT_HIP_TRY(hipMemcpyAsync(grad, lp->grad.p, kParams * sizeof(float), hipMemcpyDeviceToDevice, s));
  return read_loss(*lp, batch, plane, loss, s);
}

sofft_status sofft_lp_backward(sofft_lp* lp, const void* r, const void* pz, const float* dout, int64_t ny,
                               int64_t nx, int32_t batch, float* din, float* dw, void* stream) {
  if (!lp || !r || !pz || !dout || !din || !dw || ny <= 0 || nx <= 0 || batch <= 0) {
    set_error("bad argument to sofft_lp_backward");
    return SOFFT_EINVAL;
  }
  if (nx % 16 != 0) {
    set_error("the correction network needs grid widths that are multiples of 16");
    return SOFFT_EUNSUPPORTED;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t plane = size_t(ny) * size_t(nx);
  sofft_status st = lp_carve(*lp, batch, plane, 0);
  if (st != SOFFT_OK) return st;
  double* scale = static_cast<double*>(lp->scale.p);
  const cx<double>* rv = static_cast<const cx<double>*>(r);
  if ((st = lp_rms(rv, batch, plane, scale, s)) != SOFFT_OK) return st;
  k_lp_pack<<<dim3(unsigned((plane + 255) / 256), batch), 256, 0, s>>>(
      rv, static_cast<const cx<double>*>(pz), scale, nullptr, nullptr, plane, static_cast<_Float16*>(lp->x0.p));
  SOFFT_HIP_TRY(hipGetLastError());
  if ((st = forward_layers(*lp, batch, int(ny), int(nx), nullptr, kOutF32, nullptr, nullptr, s)) != SOFFT_OK)
    return st;
  if ((st = backward_from(*lp, dout, batch, int(ny), int(nx), din, s)) != SOFFT_OK) return st;
  SOFFT_HIP_TRY(hipMemcpyAsync(dw, lp->grad.p, kParams * sizeof(float), hipMemcpyDeviceToDevice, s));
  return SOFFT_OK;
}

sofft_status sofft_lp_train(sofft_lp* lp, sofft_plan* plan, const void* r, const void* e, const double* E_host,
                            int64_t npairs, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                            double* loss_host, void* stream) {
  if (!lp || !plan || !r || !e || !E_host || npairs <= 0 || epochs <= 0 || batch <= 0 || !(lr > 0)) {
    set_error("bad argument to sofft_lp_train");
    return SOFFT_EINVAL;
  }
  Plan& p = plan_of(plan);
  if (p.prob.ndim != 2 || p.prob.dtype != SOFFT_C128) {
    set_error("training pairs come from 2D complex128 plans");
    return SOFFT_EUNSUPPORTED;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int H = int(p.ax[1].n), W = int(p.ax[0].n);
  const size_t plane = size_t(H) * W;
  const cx<double>* rv = static_cast<const cx<double>*>(r);
  const cx<double>* ev = static_cast<const cx<double>*>(e);
  sofft_status st = lp_carve(*lp, batch, plane, npairs);
  if (st != SOFFT_OK) return st;
  cx<double>* pz = static_cast<cx<double>*>(lp->pz.p);
  // P^-1 r of every pair at its energy, and the scales
  for (int64_t k = 0; k < npairs; ++k)
    if ((st = sse_apply(p, 1, rv + size_t(k) * plane, pz + size_t(k) * plane, E_host[k], 0.0, s)) != SOFFT_OK)
      return st;
  double* scale = static_cast<double*>(lp->scale.p);
  if ((st = lp_rms(rv, int(npairs), plane, scale, s)) != SOFFT_OK) return st;
  // epochs over shuffled batches (splitmix64 stream from the seed)
  uint64_t state = seed;
  auto next = [&]() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  std::vector<int> order(npairs);
  std::vector<int> bidx(batch);
  for (int64_t k = 0; k < npairs; ++k) order[k] = int(k);
  int* idx = static_cast<int*>(lp->idx.p);
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t k = npairs - 1; k > 0; --k) std::swap(order[k], order[next() % uint64_t(k + 1)]);
    double ep_loss = 0.0;
    int nb = 0;
    for (int64_t k0 = 0; k0 + batch <= npairs; k0 += batch) {
      for (int b = 0; b < batch; ++b) bidx[b] = order[k0 + b];
      SOFFT_HIP_TRY(hipMemcpyAsync(idx, bidx.data(), batch * sizeof(int), hipMemcpyHostToDevice, s));
      if ((st = loss_grad(*lp, rv, pz, ev, scale, idx, batch, H, W, s)) != SOFFT_OK) return st;
      lp->adam_t += 1;
      const float bc1 = float(1.0 - std::pow(0.9, double(lp->adam_t)));
      const float bc2 = float(1.0 - std::pow(0.999, double(lp->adam_t)));
      k_lp_adam<<<(kParams + 255) / 256, 256, 0, s>>>(static_cast<float*>(lp->params.p),
                                                      static_cast<const float*>(lp->grad.p),
                                                      static_cast<float*>(lp->m.p), static_cast<float*>(lp->v.p),
                                                      kParams, float(lr), bc1, bc2);
      SOFFT_HIP_TRY(hipGetLastError());
      double l = 0.0;
      if ((st = read_loss(*lp, batch, plane, &l, s)) != SOFFT_OK) return st;   // also keeps bidx safe to reuse
      ep_loss += l;
      ++nb;
    }
    if (loss_host) loss_host[ep] = nb ? ep_loss / nb : 0.0;
  }
  return SOFFT_OK;
}

sofft_status sofft_sse_solve_learned(sofft_plan* plan, sofft_lp* lp, const void* f, int32_t f_per_energy,
                                     const double* E_host, int32_t nE, double field, void* x_out, double rtol,
                                     int32_t maxit, int32_t patience, sofft_solve_stats* stats, void* stream) {
  if (!plan || !lp || !f || !E_host || nE <= 0 || !x_out || !(rtol > 0) || maxit <= 0 || patience <= 0 ||
      !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_solve_learned");
    return SOFFT_EINVAL;
  }
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E_host[e])) {
      set_error("energies must be finite");
      return SOFFT_EINVAL;
    }
  Plan& p = plan_of(plan);
  if (p.prob.ndim == 2 && p.ax[0].n % 16 != 0) {
    set_error("the correction network needs grid widths that are multiples of 16");
    return SOFFT_EUNSUPPORTED;
  }
  if (p.prob.ndim == 2) {
    const sofft_status st = lp_carve(*lp, nE, size_t(p.ax[0].n) * size_t(p.ax[1].n), 0);
    if (st != SOFFT_OK) return st;
  }
  return sse_solve(p, f, f_per_energy, E_host, nE, field, x_out, rtol, maxit, stats,
                   reinterpret_cast<hipStream_t>(stream), lp, patience);
}

sofft_status sofft_lp_workspace_size(int64_t ny, int64_t nx, int32_t batch, int64_t npairs, int64_t* bytes) {
  if (ny <= 0 || nx <= 0 || batch <= 0 || npairs < 0 || !bytes) {
    set_error("bad argument to sofft_lp_workspace_size");
    return SOFFT_EINVAL;
  }
  *bytes = int64_t(lp_ws_bytes(batch, size_t(ny) * size_t(nx), npairs));
  return SOFFT_OK;
}

sofft_status sofft_lp_bind(sofft_lp* lp, void* workspace, int64_t bytes) {
  if (!lp || bytes < 0 || (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)) {
    set_error("bad argument to sofft_lp_bind (the workspace must be 256-byte aligned)");
    return SOFFT_EINVAL;
  }
  lp->ws = workspace;
  lp->ws_bytes = workspace ? size_t(bytes) : 0;
  return SOFFT_OK;
}

}  // extern "C"
