// Elementwise CG updates, conversions and the fixed-order reductions (gfx950).
//
// Reductions are two-stage and deterministic: every kernel block writes one FP64 partial sum
// (per-thread sums over a fixed grid-stride sequence, then a fixed butterfly over the wave and
// a fixed combine over the block), and a single-block finalize kernel adds the partials in a
// fixed order.  No floating-point atomics are used, so results are bitwise reproducible.
#include "common.h"
#include "stencil.h"
#include "refine.h"

namespace tbs {

template <typename T>
__device__ __forceinline__ double block_sum_write(double v, double* part) {
  __shared__ double red[4];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    s = (red[0] + red[1]) + (red[2] + red[3]);
    part[blockIdx.x] = s;
  }
  return s;
}

// r <- r - alpha q ; partial sums of r.r   (T = double or float)
template <typename T>
__global__ __launch_bounds__(256) void cg2_kernel(T* __restrict__ r, const T* __restrict__ q, int64_t n,
                                                  double* part, const Scalars* s) {
  if (s->done) return;
  const T alpha = (T)s->alpha;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const T v = r[i] - alpha * q[i];
    r[i] = v;
    acc += (double)v * (double)v;
  }
  block_sum_write<T>(acc, part);
}

// float specialisation with 4-wide accesses (arrays are 256-byte aligned)
template <>
__global__ __launch_bounds__(256) void cg2_kernel<float>(float* __restrict__ r, const float* __restrict__ q, int64_t n,
                                                         double* part, const Scalars* s) {
  if (s->done) return;
  const float alpha = (float)s->alpha;
  const int64_t n4 = n >> 2;
  const int64_t stride = (int64_t)gridDim.x * 256;
  float4* r4 = (float4*)r;
  const float4* q4 = (const float4*)q;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
    float4 a = r4[i];
    const float4 b = q4[i];
    a.x -= alpha * b.x; a.y -= alpha * b.y; a.z -= alpha * b.z; a.w -= alpha * b.w;
    r4[i] = a;
    acc += ((double)a.x * a.x + (double)a.y * a.y) + ((double)a.z * a.z + (double)a.w * a.w);
  }
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
    const int64_t i = (n4 << 2) + threadIdx.x;
    const float v = r[i] - alpha * q[i];
    r[i] = v;
    acc += (double)v * v;
  }
  block_sum_write<float>(acc, part);
}

// r <- b - q ; partial sums of r.r (part0) and b.b (part1)
template <typename T>
__global__ __launch_bounds__(256) void sub_norm_kernel(T* __restrict__ r, const T* __restrict__ b,
                                                       const T* __restrict__ q, int64_t n, double* p0, double* p1) {
  __shared__ double red[2][4];
  const int64_t stride = (int64_t)gridDim.x * 256;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const T bv = b[i];
    const T v = bv - q[i];
    r[i] = v;
    a0 += (double)v * (double)v;
    a1 += (double)bv * (double)bv;
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[0][wave] = a0; red[1][wave] = a1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    p0[blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    p1[blockIdx.x] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// The pending x updates, one rounding each and the older first, as the CG kernels apply them:
// x + alpha2 p_{nit-2} (two pending) and then + alpha p_{nit-1} (p_{nit-1} = (nit odd ? p1 : p0),
// p_{nit-2} the other array).
template <typename T, typename Tp>
__device__ __forceinline__ T apply_pending(T x, int np, T alpha, T alpha2, const Tp* p, const Tp* pp, int64_t i) {
  if (np == 2) x = fma(alpha2, Io<Tp>::template ld<T>(pp, i), x);
  if (np >= 1) x = fma(alpha, Io<Tp>::template ld<T>(p, i), x);
  return x;
}

// x <- x + the pending updates
template <typename T, typename Tp>
__global__ __launch_bounds__(256) void flush_kernel(T* __restrict__ x, const Tp* __restrict__ p0,
                                                    const Tp* __restrict__ p1, int64_t n, const Scalars* s) {
  const int np = s->pending;
  if (!np) return;
  const bool xz = s->xzero;
  const T alpha = (T)s->alpha, alpha2 = (T)s->alpha2;
  const Tp* p = (s->nit & 1) ? p1 : p0;
  const Tp* pp = (s->nit & 1) ? p0 : p1;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    T x0 = (T)0;
    if (!xz) x0 = x[i];
    x[i] = apply_pending<T, Tp>(x0, np, alpha, alpha2, p, pp, i);
  }
}

// out = base + scale (d + the pending updates), the FP32 part formed exactly as flush_kernel forms it
template <typename Tp>
__global__ __launch_bounds__(256) void refine_add_kernel(double* out, const double* base, const float* __restrict__ d,
                                                         const Tp* __restrict__ p0, const Tp* __restrict__ p1,
                                                         int64_t n, const Scalars* s, double scale) {
  const int np = s->pending;
  const bool dz = s->xzero;  // d was never written: zero
  const float alpha = (float)s->alpha, alpha2 = (float)s->alpha2;
  const Tp* p = (s->nit & 1) ? p1 : p0;
  const Tp* pp = (s->nit & 1) ? p0 : p1;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    float d0 = 0.f;
    if (!dz) d0 = d[i];
    const float x = apply_pending<float, Tp>(d0, np, alpha, alpha2, p, pp, i);
    out[i] = fma(scale, (double)x, base[i]);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void dot_kernel(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                  double* part) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) acc += (double)a[i] * (double)b[i];
  block_sum_write<T>(acc, part);
}

template <typename Ts, typename Td>
__global__ __launch_bounds__(256) void convert_kernel(const void* __restrict__ src, void* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    if (sizeof(Td) == 2) {
      // to bf16: round the fp32 value (an f64 source is first rounded to fp32)
      const float v = Io<Ts>::template ld<float>(src, i);
      ((uint16_t*)dst)[i] = f32_to_bf16(v);
    } else {
      using Tc = typename std::conditional<sizeof(Td) == 8, double, float>::type;
      Io<Td>::template st<Tc>(dst, i, Io<Ts>::template ld<Tc>(src, i));
    }
  }
}

__global__ __launch_bounds__(256) void add_f32_to_f64_kernel(double* __restrict__ x, const float* __restrict__ d, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) x[i] += (double)d[i];
}

__global__ __launch_bounds__(256) void guess_combine_kernel(double* __restrict__ x, const double* __restrict__ u,
                                                            const float* __restrict__ du, int64_t n, double scale) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) x[i] = fma(scale, (double)du[i], u[i]);
}

// Streaming copy with 16-byte accesses, four in flight per thread (the bandwidth reference of the
// library's kernels); any byte tail is copied by the first block.
__global__ __launch_bounds__(256) void stream_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          int64_t n16, const unsigned char* __restrict__ s8,
                                                          unsigned char* __restrict__ d8, int64_t nbytes) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
  if (blockIdx.x == 0)
    for (int64_t j = n16 * 16 + threadIdx.x; j < nbytes; j += 256) d8[j] = s8[j];
}

__global__ __launch_bounds__(256) void fill_kernel(uint32_t* __restrict__ x, int64_t nwords) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nwords; i += stride) x[i] = 0u;
}

// out[0] = sqrt(r.r), out[1] = sqrt(b.b) of a FIN_NORMS reduction, to device memory
__global__ void norms_out_kernel(const Scalars* __restrict__ s, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = sqrt(s->out);
    out[1] = sqrt(s->out2);
  }
}

__global__ __launch_bounds__(1024) void finalize_kernel(int op, const double* __restrict__ p0,
                                                        const double* __restrict__ p1,
                                                        const double* __restrict__ p2,
                                                        const double* __restrict__ p3, int count, Scalars* s,
                                                        double rtol) {
  __shared__ double r0[1024], r1[1024], r2[1024], r3[1024];
  if (op == FIN_CLEAR_PENDING) {
    if (threadIdx.x == 0) s->pending = 0;
    return;
  }
  if ((op == FIN_ALPHA || op == FIN_BETA || op == FIN_FUSED) && s->done) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) {
    a0 += p0[i];
    if (p1) a1 += p1[i];
    if (p2) a2 += p2[i];
    if (p3) a3 += p3[i];
  }
  r0[threadIdx.x] = a0;
  r1[threadIdx.x] = a1;
  r2[threadIdx.x] = a2;
  r3[threadIdx.x] = a3;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
      r3[threadIdx.x] += r3[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double v0 = r0[0], v1 = r1[0], v2 = r2[0], v3 = r3[0];
  switch (op) {
    case FIN_INIT:
    case FIN_INIT_XZERO: {
      s->rr = v0; s->rr0 = v0; s->bb = v1; s->tol2 = rtol * rtol * v1;
      s->nit = 0; s->status = 0; s->pending = 0; s->alpha = 0.0; s->alpha2 = 0.0; s->beta = 0.0;
      s->xzero = (op == FIN_INIT_XZERO);
      int done = (v1 == 0.0) || (v0 <= s->tol2);
      if (!isfinite(v0) || !isfinite(v1)) { s->status = -4; done = 1; }
      s->done = done;
      break;
    }
    case FIN_ALPHA: {
      s->pending = 0;
      s->pq = v0;
      if (!(v0 > 0.0) || !isfinite(v0)) { s->status = -4; s->done = 1; break; }
      s->alpha = s->rr / v0;
      break;
    }
    case FIN_BETA: {
      if (!isfinite(v0)) { s->status = -4; s->done = 1; break; }
      s->beta = v0 / s->rr;
      s->rr = v0;
      s->nit += 1;
      s->pending = 1;
      if (v0 <= s->tol2) s->done = 1;
      break;
    }
    case FIN_FUSED: {
      // v0 = p_k.q_k, v1 = r_k.q_k, v2 = q_k.q_k, v3 = r_k.r_k of the iteration's recursive residual.
      // alpha from the explicit r_k.r_k; r_{k+1}.r_{k+1} = r.r - 2 alpha r.q + alpha^2 q.q (one step
      // ahead, restarted from the explicit value every iteration) gives beta and the stopping test.
      // The kernel applied the pending x updates only if there were two; this iteration's is added.
      if (s->pending == 2) { s->pending = 0; s->xzero = 0; }  // x was written
      s->pq = v0;
      if (!(v0 > 0.0) || !isfinite(v0) || !isfinite(v1) || !isfinite(v2) || !isfinite(v3)) {
        s->status = -4; s->done = 1; break;
      }
      const double alpha = v3 / v0;
      double rn = v3 - 2.0 * alpha * v1 + alpha * alpha * v2;
      if (rn < 0.0) rn = 0.0;
      s->alpha2 = s->alpha;
      s->alpha = alpha;
      s->beta = v3 > 0.0 ? rn / v3 : 0.0;
      s->rr = rn;
      s->nit += 1;
      s->pending += 1;
      if (rn <= s->tol2) s->done = 1;
      break;
    }
    case FIN_DOT: s->out = v0; break;
    case FIN_NORMS: s->out = v0; s->out2 = v1; break;
  }
}

// ------------------------------------------------------------------------------------------

static inline int vec_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > kVecBlocks) b = kVecBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_cg2(void* r, const void* q, int64_t n, int dt, double* part, const Scalars* s, hipStream_t st) {
  // fixed grid so that the number of partial sums is always kVecBlocks
  if (dt == 0)
    hipLaunchKernelGGL(cg2_kernel<double>, dim3(kVecBlocks), dim3(256), 0, st, (double*)r, (const double*)q, n, part, s);
  else
    hipLaunchKernelGGL(cg2_kernel<float>, dim3(kVecBlocks), dim3(256), 0, st, (float*)r, (const float*)q, n, part, s);
  return hipGetLastError();
}

hipError_t launch_sub_norm(void* r, const void* b, const void* q, int64_t n, int dt, double* p0, double* p1,
                           hipStream_t st) {
  if (dt == 0)
    hipLaunchKernelGGL(sub_norm_kernel<double>, dim3(kVecBlocks), dim3(256), 0, st, (double*)r, (const double*)b,
                       (const double*)q, n, p0, p1);
  else
    hipLaunchKernelGGL(sub_norm_kernel<float>, dim3(kVecBlocks), dim3(256), 0, st, (float*)r, (const float*)b,
                       (const float*)q, n, p0, p1);
  return hipGetLastError();
}

hipError_t launch_flush(void* x, const void* p0, const void* p1, int64_t n, int dt, const Scalars* s, hipStream_t st) {
  const int b = vec_blocks(n);
  if (dt == 0)
    hipLaunchKernelGGL((flush_kernel<double, double>), dim3(b), dim3(256), 0, st, (double*)x, (const double*)p0,
                       (const double*)p1, n, s);
  else if (dt == 1)
    hipLaunchKernelGGL((flush_kernel<float, float>), dim3(b), dim3(256), 0, st, (float*)x, (const float*)p0,
                       (const float*)p1, n, s);
  else
    hipLaunchKernelGGL((flush_kernel<float, uint16_t>), dim3(b), dim3(256), 0, st, (float*)x, (const uint16_t*)p0,
                       (const uint16_t*)p1, n, s);
  return hipGetLastError();
}

hipError_t launch_refine_add(double* out, const double* base, const float* d, const void* p0, const void* p1,
                             int64_t n, int dt, const Scalars* s, double scale, hipStream_t st) {
  const int b = vec_blocks(n);
  if (dt == 1)
    hipLaunchKernelGGL(refine_add_kernel<float>, dim3(b), dim3(256), 0, st, out, base, d, (const float*)p0,
                       (const float*)p1, n, s, scale);
  else
    hipLaunchKernelGGL(refine_add_kernel<uint16_t>, dim3(b), dim3(256), 0, st, out, base, d, (const uint16_t*)p0,
                       (const uint16_t*)p1, n, s, scale);
  return hipGetLastError();
}

hipError_t launch_dot(const void* a, const void* b, int64_t n, int dt, double* part, hipStream_t st) {
  if (dt == 0)
    hipLaunchKernelGGL(dot_kernel<double>, dim3(kVecBlocks), dim3(256), 0, st, (const double*)a, (const double*)b, n, part);
  else
    hipLaunchKernelGGL(dot_kernel<float>, dim3(kVecBlocks), dim3(256), 0, st, (const float*)a, (const float*)b, n, part);
  return hipGetLastError();
}

hipError_t launch_convert(const void* src, int sdt, void* dst, int ddt, int64_t n, hipStream_t st) {
  const int b = vec_blocks(n);
#define CONV(S, D) hipLaunchKernelGGL((convert_kernel<S, D>), dim3(b), dim3(256), 0, st, src, dst, n)
  if (sdt == 0 && ddt == 1) CONV(double, float);
  else if (sdt == 0 && ddt == 2) CONV(double, uint16_t);
  else if (sdt == 1 && ddt == 0) CONV(float, double);
  else if (sdt == 1 && ddt == 2) CONV(float, uint16_t);
  else if (sdt == 2 && ddt == 1) CONV(uint16_t, float);
  else if (sdt == 2 && ddt == 0) CONV(uint16_t, double);
  else return hipErrorInvalidValue;
#undef CONV
  return hipGetLastError();
}

hipError_t launch_add_f32_to_f64(double* x, const float* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(add_f32_to_f64_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, x, d, n);
  return hipGetLastError();
}

hipError_t launch_guess_combine(double* x, const double* u, const float* du, int64_t n, double scale, hipStream_t st) {
  hipLaunchKernelGGL(guess_combine_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, x, u, du, n, scale);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t nbytes, hipStream_t st) {
  const int64_t n16 = nbytes / 16;
  // enough workgroups to keep every CU's memory pipeline full (8 per CU on 256 CUs)
  int64_t b = (n16 + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)b), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n16,
                     (const unsigned char*)src, (unsigned char*)dst, nbytes);
  return hipGetLastError();
}

hipError_t launch_fill(void* x, int dt, int64_t n, hipStream_t st) {
  const int64_t bytes = n * (dt == 0 ? 8 : (dt == 1 ? 4 : 2));
  const int64_t words = (bytes + 3) / 4;
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(words)), dim3(256), 0, st, (uint32_t*)x, words);
  return hipGetLastError();
}

hipError_t launch_norms_out(const Scalars* s, double* out, hipStream_t st) {
  hipLaunchKernelGGL(norms_out_kernel, dim3(1), dim3(64), 0, st, s, out);
  return hipGetLastError();
}

hipError_t launch_finalize(int op, const double* p0, const double* p1, int count, Scalars* s, double rtol,
                           hipStream_t st, const double* p2, const double* p3) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1024), 0, st, op, p0, p1, p2, p3, count, s, rtol);
  return hipGetLastError();
}

}  // namespace tbs
