// Learned initial guess for the implicit step: a 4-layer 3x3x3 CNN (2 -> 16 -> 16 -> 16 -> 1,
// exact-erf GELU) with bf16 operands on the gfx950 matrix cores and FP32 accumulation.  Not in
// the paper (which warm-starts CG from a coarse-grid solution); the network predicts
// u^{k+1} - u^k from (u^k, f) and the solver keeps its guess only if the FP64 residual drops.
//
// Activations are channels-last [voxel][16] bf16 (32 B per voxel); the first layer's input has
// 2 channels, the last layer's output 1.  Every convolution is an implicit GEMM on
// v_mfma_f32_16x16x32_bf16 computing Out^T = W^T In^T: M = 16 output channels (zero padded),
// N = 16 voxels along x, K = 2 taps x 16 input channels per instruction (27 taps padded to 28).
// A workgroup stages its input tile (halo 1) in LDS with 16 channels per voxel and each wave
// accumulates 16-voxel rows.  The same kernel runs the backward data pass with flipped,
// transposed weights.  Weight gradients are a deterministic two-stage reduction on the vector
// ALUs (per-workgroup partial sums, then a fixed-order sum).  Optimiser: Adam on FP32 master
// weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>

#include "../../include/tbs.h"
#include "common.h"
#include "net.h"

namespace tbs {
namespace net {

constexpr int NL = 4;
constexpr int CIN[NL] = {2, 16, 16, 16};
constexpr int COUT[NL] = {16, 16, 16, 1};
constexpr int NSTEP = 15;         // MFMA K-steps of the 16-channel layout (27 taps + 3 zero partners) / 2
constexpr int PACK = NSTEP * 64 * 8;  // bf16 per packed layer
constexpr int WG_PARTS = 6928;    // max partial-gradient row: 16*16*27 weights + 16 biases
constexpr int SMOOTH_PASSES = 2;  // passes of the separable binomial low-pass after the last layer

__host__ __device__ constexpr int woff(int l) {  // offset of W_l in the flat parameter vector
  return l == 0 ? 0 : woff(l - 1) + CIN[l - 1] * COUT[l - 1] * 27 + COUT[l - 1];
}
__host__ __device__ constexpr int boff(int l) { return woff(l) + CIN[l] * COUT[l] * 27; }
static_assert(woff(NL) == TBS_NET_PARAMS, "parameter count");

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// GELU(x) = x Phi(x) = max(x, 0) - |x| Phi(-|x|), with the normal tail Phi(-y) = t 2^(P(t) - y^2 /
// (2 ln 2)), t = 1 / (1 + c y), P of degree 6 fitted by fit_gelu.py (relative error of Phi(-y)
// below 1.3e-6 for all y >= 0), so the negative tail keeps its relative accuracy.
__device__ __forceinline__ float gelu_f(float x) {
  const float y = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(2.700000107e-01f, y, 1.0f));
  float p = 3.957020044e-01f;
  p = fmaf(p, t, -1.359942675e+00f);
  p = fmaf(p, t, 1.348554134e+00f);
  p = fmaf(p, t, -3.906427920e-01f);
  p = fmaf(p, t, 8.047851324e-01f);
  p = fmaf(p, t, 1.414555073e+00f);
  p = fmaf(p, t, -3.213009119e+00f);
  const float q = t * __builtin_amdgcn_exp2f(fmaf(y * y, -0.72134752044448170f, p));  // Phi(-y)
  return fmaf(-y, q, fmaxf(x, 0.f));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

struct Grid3 {
  int nx, ny, nz;
  int periodic;
};

// ------------------------------------------------------------------------------------------
// convolution on the matrix cores

enum Epi { EPI_GELU = 0, EPI_LINEAR = 1, EPI_BWD = 2, EPI_RAW = 3 };

// Geometry of the z-marching convolution: a workgroup owns a 32 x 8 column of output voxels and
// marches through a chunk of zc planes, keeping the three input planes a output plane needs in an
// LDS ring (one-voxel halo in x and y) and fetching the next plane into registers meanwhile.
constexpr int CTX = 32, CTY = 8;                  // output tile per plane (x, y)
constexpr int SX = CTX + 2, SY = CTY + 2;          // staged plane
constexpr int PLV = SX * SY;                       // voxels per staged plane
constexpr int WROWS = 2 * CTY / 4;                 // 16-voxel rows per wave per plane

struct ConvGeo {
  int tx, ty, nch, zc;
};
// z-chunk length: about 2048 workgroups in flight on small grids, at most 96 planes per chunk
__host__ __device__ inline ConvGeo conv_geo(const Grid3& g) {
  ConvGeo c;
  c.tx = (g.nx + CTX - 1) / CTX;
  c.ty = (g.ny + CTY - 1) / CTY;
  int64_t zc = (int64_t)g.nz * c.tx * c.ty / 2048;
  c.zc = (int)(zc < 4 ? 4 : (zc > 96 ? 96 : zc));
  c.nch = (g.nz + c.zc - 1) / c.zc;
  return c;
}

// 16-channel K order.  Tap index t = 9 dz + 3 dy + dx.  K-step s holds taps tap16(s, 0) and
// tap16(s, 1): steps 3 dy + dx pair (0, dy, dx) with (1, dy, dx); steps 9 + dy pair (2, dy, 0) with
// (2, dy, 1); steps 12 + dy hold (2, dy, 2) and a zero-weight partner.  For a fixed dz-pair and dx
// the B operand depends only on the staged row y + dy, so one LDS read serves the three output
// rows it touches (dy = 0, 1, 2), each with its own A operand.
__host__ __device__ constexpr int tap16(int s, int half) {
  return s < 9 ? s + 9 * half : (s < 12 ? 18 + 3 * (s - 9) + half : 18 + 3 * (s - 12) + 2);
}
__host__ __device__ constexpr bool pad16(int s, int half) { return s >= 12 && half == 1; }

typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
// two floats to packed bf16 (round to nearest even) with the gfx950 conversion instruction
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  bf16x2 v;
  v[0] = (__bf16)lo;
  v[1] = (__bf16)hi;
  return __builtin_bit_cast(uint32_t, v);
}

// in: [voxel][CIS] bf16; wpk: packed A operands [steps][64 lanes][8]; out per epilogue:
//   EPI_GELU:   zout (f32 [voxel][16], nullable) = acc + bias; yout (bf16 [voxel][16]) = GELU(z)
//   EPI_LINEAR: fout (f32 [voxel]) = (acc[0] + bias[0]) * (*scale)          (last layer, 1 channel)
//   EPI_BWD:    yout (bf16 [voxel][16]) = acc * GELU'(zprev[voxel][c])       (backward data)
//   EPI_RAW:    fout (f32 [voxel][COS]) = acc (+ bias if bias != NULL)       (parity probes)
// Two K layouts: with 16 (or zero-padded 1) input channels each K-step holds 2 taps x 16
// channels (15 steps, order tap16); with 2 input channels it holds 16 taps x 2 channels (2 steps,
// 27 taps padded to 32), and the ring keeps only the 2 channels.  Each wave owns 4 consecutive
// rows (y) of 16 voxels (x) per plane; the plane loop is unrolled by the ring period so all LDS
// reads of the B operands use immediate offsets.
template <int CIS, int COS, int EPI>
__global__ __launch_bounds__(256) void conv_mfma(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wpk,
                                                 const float* __restrict__ bias, Grid3 g,
                                                 float* __restrict__ zout, uint16_t* __restrict__ yout,
                                                 float* __restrict__ fout, const float* __restrict__ zprev,
                                                 const double* __restrict__ scale) {
  constexpr bool TWO = (CIS == 2);
  constexpr int STEPS = TWO ? 2 : NSTEP;
  constexpr int VW = TWO ? 2 : 16;                  // bf16 per staged voxel
  constexpr int UNITS = CIS == 16 ? 2 * PLV : PLV;  // load units per plane (16 B, or one voxel)
  constexpr int UPT = (UNITS + 255) / 256;          // units per thread
  using Unit = typename std::conditional<CIS == 16, uint4, typename std::conditional<TWO, uint32_t, uint16_t>::type>::type;
  __shared__ __attribute__((aligned(16))) uint16_t st[3 * PLV * VW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const ConvGeo geo = conv_geo(g);
  const int64_t plane = (int64_t)g.nx * g.ny;

  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = bid % geo.tx, by = (bid / geo.tx) % geo.ty, ch = bid / (geo.tx * geo.ty);
  const int x0 = bx * CTX, y0 = by * CTY, z0 = ch * geo.zc;
  const int zc = min(geo.zc, g.nz - z0);

  // A operands (weights) for all K-steps, loaded once and kept in registers
  bf16x8 wa[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) wa[s] = *(const bf16x8*)(wpk + (s * 64 + lane) * 8);
  float bz[4] = {0.f, 0.f, 0.f, 0.f};
  const int grp = lane >> 4;          // K-group of this lane
  const int vx = lane & 15;           // voxel (x) of this lane's B column / D column
  const int c0 = 4 * grp;             // D rows (output channels) held by this lane
  if (bias)
#pragma unroll
    for (int r = 0; r < 4; ++r) bz[r] = (c0 + r < COS) ? bias[c0 + r] : 0.f;

  // this thread's load units: plane-relative global voxel offsets (-1: outside a Dirichlet grid)
  int uoff[UPT];
#pragma unroll
  for (int q = 0; q < UPT; ++q) {
    const int u = tid + 256 * q;
    const int v = CIS == 16 ? (u >> 1) : u;
    int gx = x0 - 1 + v % SX, gy = y0 - 1 + v / SX;
    bool ok = u < UNITS;
    if (g.periodic) {
      gx = (gx + g.nx) % g.nx;
      gy = (gy + g.ny) % g.ny;
    } else {
      ok = ok && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny;
    }
    uoff[q] = ok ? gy * g.nx + gx : -1;
  }
  if (CIS == 1) {  // channels 1..15 of the ring stay zero
    for (int i = tid; i < 3 * PLV * VW / 8; i += 256) ((uint4*)st)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
  }
  Unit pre[UPT];
  // fetch relative plane j (global plane z0 - 1 + j) into pre
  auto fetch = [&](int j) {
    int gz = z0 - 1 + j;
    bool pv = true;
    if (g.periodic) gz = (gz + g.nz) % g.nz;
    else pv = gz >= 0 && gz < g.nz;
    const int64_t pb = (int64_t)gz * plane;
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      pre[q] = Unit{};
      if (pv && uoff[q] >= 0) {
        if constexpr (CIS == 16) pre[q] = ((const uint4*)(in + (pb + uoff[q]) * 16))[(tid + 256 * q) & 1];
        else if constexpr (TWO) pre[q] = *(const uint32_t*)(in + (pb + uoff[q]) * 2);
        else pre[q] = in[pb + uoff[q]];
      }
    }
  };
  auto stash = [&](int slot) {
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int u = tid + 256 * q;
      if (UNITS % 256 == 0 || u < UNITS) {
        if constexpr (CIS == 16) ((uint4*)st)[slot * PLV * 2 + u] = pre[q];
        else if constexpr (TWO) ((uint32_t*)st)[slot * PLV + u] = pre[q];
        else st[(slot * PLV + u) * 16] = pre[q];
      }
    }
  };

  // B operand lane offsets (bf16 elements of st) for the wave's first row: wave w owns rows
  // y = 4 (w >> 1) + r (r = 0..3) of x half w & 1
  const int yb = 4 * (wave >> 1), xh = wave & 1;
  const int lb = yb * SX + xh * 16 + vx;
  int loff[TWO ? 24 : 5];
  if (TWO) {
    // k = 8 grp + j: tap 16 s + 4 grp + j/2, channel j % 2; padding taps (> 26) read tap 13
#pragma unroll
    for (int ph = 0; ph < 3; ++ph)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int tap = 16 * s + 4 * grp + t;
          if (tap > 26) tap = 13;
          loff[8 * ph + 4 * s + t] = (lb + ((ph + tap / 9) % 3) * PLV + ((tap / 3) % 3) * SX + tap % 3) * 2;
        }
  } else {
    // k = 8 grp + j: tap tap16(s, grp >> 1), channel 8 (grp & 1) + j
    const int l0 = lb * 16 + (grp & 1) * 8, h = grp >> 1;
#pragma unroll
    for (int ph = 0; ph < 3; ++ph) loff[ph] = l0 + h * ((ph == 2 ? -2 : 1) * PLV * 16);  // dz 0 -> dz 1
    loff[3] = l0 + h * 16;                                                           // dx 0 -> dx 1
    loff[4] = l0;                                                                    // partner unused
  }

  // prologue: ring slots 0..2 hold planes z0-1, z0, z0+1; registers hold plane z0+2
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    fetch(j);
    stash(j);
  }
  fetch(3);

  for (int i0 = 0; i0 < zc; i0 += 3) {
#pragma unroll
    for (int ph = 0; ph < 3; ++ph) {
      const int i = i0 + ph;
      if (i < zc) {  // uniform
        __syncthreads();  // plane z0 + i + 1 is in the ring
        const int gz = z0 + i;
        f32x4 acc[WROWS];
#pragma unroll
        for (int r = 0; r < WROWS; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (TWO) {
#pragma unroll
          for (int r = 0; r < WROWS; ++r)
#pragma unroll
            for (int s = 0; s < STEPS; ++s) {
              uint32_t w4[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) w4[t] = *(const uint32_t*)(st + loff[8 * ph + 4 * s + t] + r * SX * 2);
              bf16x8 bv;
              __builtin_memcpy(&bv, w4, 16);
              acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], bv, acc[r], 0, 0, 0);
            }
        } else {
          // staged rows yb + yy, yy = 0..5, feed output rows r = yy - dy
#pragma unroll
          for (int yy = 0; yy < WROWS + 2; ++yy) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
              // q < 3: planes (k-1, k) at dx = q; q = 3: plane k+1 at dx (0, 1); q = 4: plane k+1 at dx 2
              const int pl = q < 3 ? ph : (ph + 2) % 3;
              const int dx = q < 3 ? q : (q == 3 ? 0 : 2);
              const int lo = q < 3 ? loff[ph] : loff[q];
              const bf16x8 bv = *(const bf16x8*)(st + lo + (pl * PLV + yy * SX + dx) * 16);
#pragma unroll
              for (int dy = 0; dy < 3; ++dy) {
                const int r = yy - dy;
                if (r >= 0 && r < WROWS) {
                  const int sidx = q < 3 ? 3 * dy + q : (q == 3 ? 9 + dy : 12 + dy);
                  acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[sidx], bv, acc[r], 0, 0, 0);
                }
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < WROWS; ++r) {
          // D layout: acc[r] = Out[channel 4 grp + r][voxel vx]
          const f32x4 A = acc[r];
          const int gx = x0 + xh * 16 + vx, gy = y0 + yb + r;
          if (gx < g.nx && gy < g.ny) {
            const int64_t vi = (int64_t)gz * plane + (int64_t)gy * g.nx + gx;
            if (EPI == EPI_GELU) {
              float z[4];
#pragma unroll
              for (int c = 0; c < 4; ++c) z[c] = A[c] + bz[c];
              if (zout) *(float4*)(zout + vi * 16 + c0) = make_float4(z[0], z[1], z[2], z[3]);
              uint2 packed;
              packed.x = pack_bf16x2(gelu_f(z[0]), gelu_f(z[1]));
              packed.y = pack_bf16x2(gelu_f(z[2]), gelu_f(z[3]));
              *(uint2*)(yout + vi * 16 + c0) = packed;
            } else if (EPI == EPI_LINEAR) {
              if (grp == 0) fout[vi] = (float)(((double)A[0] + (double)bz[0]) * scale[0]);
            } else if (EPI == EPI_BWD) {
              const float4 zp = *(const float4*)(zprev + vi * 16 + c0);
              uint2 packed;
              packed.x = pack_bf16x2(A[0] * gelu_grad_f(zp.x), A[1] * gelu_grad_f(zp.y));
              packed.y = pack_bf16x2(A[2] * gelu_grad_f(zp.z), A[3] * gelu_grad_f(zp.w));
              *(uint2*)(yout + vi * 16 + c0) = packed;
            } else {
#pragma unroll
              for (int c = 0; c < 4; ++c)
                if (c0 + c < COS) fout[vi * COS + c0 + c] = A[c] + bz[c];
            }
          }
        }
        __syncthreads();  // every wave is done with slot ph (plane z0 + i - 1)
        if (i + 3 <= zc + 1) {
          stash(ph);                         // plane z0 + i + 2 (relative plane i + 3)
          if (i + 4 <= zc + 1) fetch(i + 4);
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// weight gradient: dW[co][ci][tap] = sum_v X[v + off(tap)][ci] G[v][co], dB[co] = sum_v G[v][co]
// Each block accumulates its tiles (grid-stride over tiles) in registers, then writes one row of
// partial sums; a second kernel adds the rows in a fixed order.  Work item = (co, ci) pair x row
// group; tile = 16 (x) x 4 (y) x 4 (z) voxels staged as FP32 in LDS, channel-major.

constexpr int WTX = 16, WTY = 4, WTZ = 4;
constexpr int WSX = 20, WSY = WTY + 2, WSZ = WTZ + 2;  // x staged as -2..17 (16-byte aligned rows)

template <int CIS, int COS>
__global__ __launch_bounds__(256) void wgrad_partial(const uint16_t* __restrict__ xin, const uint16_t* __restrict__ gin,
                                                     Grid3 g, float* __restrict__ part, int accumulate) {
  constexpr int P = CIS * COS;                 // weight pairs
  constexpr int NG = 256 / P;                  // row groups
  constexpr int ROWS = WTY * WTZ;
  __shared__ __attribute__((aligned(16))) float xs[CIS][WSZ][WSY][WSX];
  __shared__ __attribute__((aligned(16))) float gs[COS][ROWS][WTX];
  __shared__ float red[NG > 1 ? NG : 1][NG > 1 ? P : 1][28];
  const int tid = threadIdx.x;
  const int pair = tid % P, rg = tid / P;
  const int co = pair / CIS, ci = pair % CIS;
  const int tx = (g.nx + WTX - 1) / WTX, ty = (g.ny + WTY - 1) / WTY, tz = (g.nz + WTZ - 1) / WTZ;
  const int ntiles = tx * ty * tz;
  const int64_t plane = (int64_t)g.nx * g.ny;
  float acc[27];
  float accb = 0.f;
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = 0.f;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
    const int x0 = bx * WTX, y0 = by * WTY, z0 = bz * WTZ;
    __syncthreads();
    for (int v = tid; v < WSX * WSY * WSZ; v += 256) {
      const int sx = v % WSX, sy = (v / WSX) % WSY, sz = v / (WSX * WSY);
      int gx = x0 + sx - 2, gy = y0 + sy - 1, gz = z0 + sz - 1;
      bool ok = true;
      if (g.periodic) {
        gx = (gx + g.nx) % g.nx; gy = (gy + g.ny) % g.ny; gz = (gz + g.nz) % g.nz;
      } else {
        ok = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
      }
      const int64_t vi = (int64_t)gz * plane + (int64_t)gy * g.nx + gx;
#pragma unroll
      for (int c = 0; c < CIS; ++c) xs[c][sz][sy][sx] = ok ? bf16_to_f32(xin[vi * CIS + c]) : 0.f;
    }
    for (int v = tid; v < ROWS * WTX; v += 256) {
      const int vx = v % WTX, r = v / WTX;
      const int gx = x0 + vx, gy = y0 + r % WTY, gz = z0 + r / WTY;
      const bool ok = gx < g.nx && gy < g.ny && gz < g.nz;  // outputs outside the grid contribute 0
      const int64_t vi = (int64_t)gz * plane + (int64_t)gy * g.nx + gx;
#pragma unroll
      for (int c = 0; c < COS; ++c) gs[c][r][vx] = ok ? bf16_to_f32(gin[vi * COS + c]) : 0.f;
    }
    __syncthreads();
    for (int r = rg; r < ROWS; r += NG) {
      const int ry = r % WTY, rz = r / WTY;
      float gv[WTX];
#pragma unroll
      for (int q = 0; q < WTX; q += 4) {
        const float4 t4 = *(const float4*)&gs[co][r][q];
        gv[q] = t4.x; gv[q + 1] = t4.y; gv[q + 2] = t4.z; gv[q + 3] = t4.w;
      }
      if (ci == 0) {
#pragma unroll
        for (int q = 0; q < WTX; ++q) accb += gv[q];
      }
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          float xr[WSX];
#pragma unroll
          for (int q = 0; q < WSX; q += 4) {
            const float4 t4 = *(const float4*)&xs[ci][rz + dz][ry + dy][q];
            xr[q] = t4.x; xr[q + 1] = t4.y; xr[q + 2] = t4.z; xr[q + 3] = t4.w;
          }
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            float s = acc[dz * 9 + dy * 3 + dx];
#pragma unroll
            for (int q = 0; q < WTX; ++q) s = __builtin_fmaf(xr[q + dx + 1], gv[q], s);
            acc[dz * 9 + dy * 3 + dx] = s;
          }
        }
    }
  }
  // combine row groups in a fixed order, then one partial row per block
  if (NG > 1) {
#pragma unroll
    for (int t = 0; t < 27; ++t) red[NG > 1 ? rg : 0][pair][t] = acc[t];
    red[NG > 1 ? rg : 0][pair][27] = accb;
    __syncthreads();
    if (rg == 0) {
      for (int q = 1; q < NG; ++q) {
#pragma unroll
        for (int t = 0; t < 27; ++t) acc[t] += red[q][pair][t];
        accb += red[q][pair][27];
      }
    }
  }
  if (rg == 0) {
    float* row = part + (int64_t)blockIdx.x * WG_PARTS;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int j = (co * CIS + ci) * 27 + t;
      row[j] = accumulate ? row[j] + acc[t] : acc[t];
    }
    if (ci == 0) {
      const int j = COS * CIS * 27 + co;
      row[j] = accumulate ? row[j] + accb : accb;
    }
  }
}

// grad[woff + j] (+)= sum over partial rows (fixed order, FP64)
__global__ __launch_bounds__(256) void wgrad_reduce(const float* __restrict__ part, int rows, int count,
                                                    float* __restrict__ grad, int accumulate) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += part[(int64_t)r * WG_PARTS + j];
  grad[j] = accumulate ? (float)((double)grad[j] + s) : (float)s;
}

// ------------------------------------------------------------------------------------------
// inputs, loss, optimiser, weight packing

// sum of squares of u (and q) into sc[0], sc[1] (fixed order: per-block partials then one block)
template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                     double* part) {
  __shared__ double red[2][4];
  double s0 = 0, s1 = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double x = (double)a[i];
    s0 = fma(x, x, s0);
    if (b) { const double y = (double)b[i]; s1 = fma(y, y, s1); }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = s0; red[1][threadIdx.x >> 6] = s1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// sc[0] = 1/rms(u), sc[1] = 1/rms(q) (1 where the rms is 0), sc[2] = output scale tau*rms(u)*out_scale
__global__ void scales_final(const double* __restrict__ part, int blocks, int64_t n, double tau, double out_scale,
                             double* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s0 = 0, s1 = 0;
  for (int i = 0; i < blocks; ++i) { s0 += part[2 * i]; s1 += part[2 * i + 1]; }
  const double ru = sqrt(s0 / (double)n), rq = sqrt(s1 / (double)n);
  sc[0] = ru > 0 ? 1.0 / ru : 1.0;
  sc[1] = rq > 0 ? 1.0 / rq : 1.0;
  sc[2] = tau * (ru > 0 ? ru : 1.0) * out_scale;
  sc[3] = 1.0;
}

// x0[v] = (bf16(u * sc0), bf16(q * sc1)): the product is formed in FP64, rounded to fp32, then bf16
template <typename T>
__global__ __launch_bounds__(256) void prep_input(const T* __restrict__ u, const T* __restrict__ q, int64_t n,
                                                  const double* __restrict__ sc, uint32_t* __restrict__ x0) {
  const double a = sc[0], b = sc[1];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t c0 = f32_to_bf16((float)((double)u[i] * a));
    const uint32_t c1 = q ? f32_to_bf16((float)((double)q[i] * b)) : 0u;
    x0[i] = c0 | (c1 << 16);
  }
}

// loss partials and output gradient: t = du / sc2, diff = o - t, g = 2 diff / total (fp32; it is
// smoothed by the adjoint of the output filter and rounded to bf16 afterwards)
__global__ __launch_bounds__(256) void mse_grad(const float* __restrict__ o, const float* __restrict__ du, int64_t n,
                                                const double* __restrict__ sc, double inv_total,
                                                float* __restrict__ gout, double* part) {
  __shared__ double red[4];
  const double s = sc[2];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double d = (double)o[i] - (double)du[i] / s;
    acc = fma(d, d, acc);
    gout[i] = (float)(2.0 * d * inv_total);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One full pass B = Bx By Bz of the binomial low-pass on a 32 x 8 x 8 output tile staged with a
// one-voxel halo in LDS (the three separable passes share the tile).
// One pass of the separable binomial low-pass [1/4, 1/2, 1/4] along x, then y, then z (zero
// fill outside a Dirichlet box, wrap-around on a periodic one).  A workgroup owns a 64 x 16
// column of outputs and marches through a chunk of z-planes: each input plane is staged with its
// one-point x and y halo in a double-buffered LDS tile (the next plane is fetched into registers
// while the current one is filtered), the x- and y-passes run from LDS, and the z-pass keeps the
// xy-filtered values of the two previous planes in registers.
constexpr int SMX = 64, SMY = 16, SMR = SMY + 2, SMROWS = (SMR + 3) / 4;

__global__ __launch_bounds__(256) void smooth3(const float* __restrict__ src, float* __restrict__ dst, Grid3 g,
                                               int zc) {
  __shared__ float t[2][SMR][SMX + 2];
  const int tid = threadIdx.x, lx = tid & 63, ly = tid >> 6;
  const int tx = (g.nx + SMX - 1) / SMX, ty = (g.ny + SMY - 1) / SMY;
  int b = blockIdx.x;
  const int x0 = (b % tx) * SMX;
  b /= tx;
  const int y0 = (b % ty) * SMY;
  const int z0 = (b / ty) * zc;
  const int z1 = min(z0 + zc, g.nz);
  const int nplanes = z1 - z0 + 2;  // the chunk plus one halo plane on each side
  const int64_t plane = (int64_t)g.nx * g.ny;
  // wrapped (periodic) or range-checked (Dirichlet) index along one axis; -1 = outside
  auto fold = [&](int i, int n) -> int {
    if (g.periodic) return ((i % n) + n) % n;
    return (i >= 0 && i < n) ? i : -1;
  };
  // staged points this thread loads: its column x0 + lx on rows ly, ly + 4, ... of the tile, and
  // for the first 2 SMR threads one halo column point (left for tid < SMR, right otherwise)
  const int cx = fold(x0 + lx, g.nx);
  int64_t rowoff[SMROWS];
#pragma unroll
  for (int i = 0; i < SMROWS; ++i) {
    const int r = ly + 4 * i;
    const int gy = r < SMR ? fold(y0 + r - 1, g.ny) : -1;
    rowoff[i] = (gy < 0 || cx < 0) ? -1 : (int64_t)gy * g.nx + cx;
  }
  const bool halo = tid < 2 * SMR;
  const int hr = tid % SMR, hc = tid < SMR ? 0 : SMX + 1;
  int64_t hoff = -1;
  if (halo) {
    const int gy = fold(y0 + hr - 1, g.ny), gx = fold(x0 + (hc == 0 ? -1 : SMX), g.nx);
    hoff = (gy < 0 || gx < 0) ? -1 : (int64_t)gy * g.nx + gx;
  }
  float pm[SMROWS], ph = 0.f;
  auto fetch = [&](int k) {
    const int gz = fold(z0 - 1 + k, g.nz);
    const float* sp = src + (int64_t)(gz < 0 ? 0 : gz) * plane;
#pragma unroll
    for (int i = 0; i < SMROWS; ++i) pm[i] = (gz >= 0 && rowoff[i] >= 0) ? sp[rowoff[i]] : 0.f;
    if (halo) ph = (gz >= 0 && hoff >= 0) ? sp[hoff] : 0.f;
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < SMROWS; ++i)
      if (ly + 4 * i < SMR) t[buf][ly + 4 * i][lx + 1] = pm[i];
    if (halo) t[buf][hr][hc] = ph;
  };
  // output rows 4 ly .. 4 ly + 3 of the column; their xy-filtered values on the two previous planes
  float s0[4] = {0.f, 0.f, 0.f, 0.f}, s1[4] = {0.f, 0.f, 0.f, 0.f};
  const int gxo = x0 + lx;
  fetch(0);
  for (int k = 0; k < nplanes; ++k) {
    const int buf = k & 1;
    stash(buf);
    if (k + 1 < nplanes) fetch(k + 1);
    __syncthreads();
    float xr[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const float* row = &t[buf][4 * ly + i][lx];
      xr[i] = 0.25f * row[0] + 0.5f * row[1] + 0.25f * row[2];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float s2 = 0.25f * xr[j] + 0.5f * xr[j + 1] + 0.25f * xr[j + 2];
      const int gy = y0 + 4 * ly + j;
      if (k >= 2 && gxo < g.nx && gy < g.ny)
        dst[(int64_t)(z0 + k - 2) * plane + (int64_t)gy * g.nx + gxo] = 0.25f * s0[j] + 0.5f * s1[j] + 0.25f * s2;
      s0[j] = s1[j];
      s1[j] = s2;
    }
  }
}

// z-planes per workgroup of the low-pass: enough workgroups to fill the chip several times over
static int smooth_zchunk(Grid3 g) {
  const int64_t cols = (int64_t)((g.nx + SMX - 1) / SMX) * ((g.ny + SMY - 1) / SMY);
  return (int)std::max<int64_t>(8, std::min<int64_t>(64, (int64_t)g.nz * cols / 8192));
}

__global__ __launch_bounds__(256) void f32_to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                          int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = f32_to_bf16(src[i]);
}

__global__ void loss_final(const double* __restrict__ part, int blocks, double inv_total, double* loss_acc,
                           int accumulate) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0;
  for (int i = 0; i < blocks; ++i) s += part[i];
  loss_acc[0] = (accumulate ? loss_acc[0] : 0.0) + s * inv_total;
}

// Adam (Kingma & Ba 2015) on the FP32 master weights; t is the 1-based step
__global__ __launch_bounds__(256) void adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                            const float* __restrict__ g, int n, int t, float lr, float b1, float b2,
                                            float eps) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)t));
  const float vh = vi / (1.0f - powf(b2, (float)t));
  w[i] = w[i] - lr * mh / (sqrtf(vh) + eps);
}

// Packed A operands of layer l.  Forward: A[m][k] = W[m][ci][tap] with tap = tap16(s, k >> 4),
// ci = k & 15 (zero outside the layer's channels and for the padding partners of steps 12-14).  Backward data (flip = 1):
// the transposed convolution's weights W'[ci][co][tap] = W[co][ci][26 - tap], M = ci, K = (tap, co).
// Lane layout of v_mfma_f32_16x16x32_bf16 A: lane holds row (lane & 15), k = 8 (lane >> 4) + j.
__global__ __launch_bounds__(64) void pack_weights(const float* __restrict__ w, int l, int flip,
                                                   uint16_t* __restrict__ out, float* __restrict__ bias_out) {
  const int lane = threadIdx.x;
  const int ci_n = flip ? COUT[l] : CIN[l];   // K-channel count of this convolution
  const int m_n = flip ? CIN[l] : COUT[l];    // output channels
  const float* W = w + woff(l);
  const int mrow = lane & 15, grp = lane >> 4;
  for (int s = 0; s < NSTEP; ++s) {
    for (int j = 0; j < 8; ++j) {
      float val = 0.f;
      if (!flip && ci_n == 2) {
        // two-channel layout: k = 8 grp + j -> tap 16 s + 4 grp + j/2, channel j % 2 (2 steps)
        const int tap = 16 * s + 4 * grp + (j >> 1), kc = j & 1;
        if (s < 2 && tap < 27 && mrow < m_n) val = W[(mrow * CIN[l] + kc) * 27 + tap];
      } else {
        const int half = grp >> 1;
        const int tap = tap16(s, half);
        const int kc = (grp & 1) * 8 + j;
        if (!pad16(s, half) && mrow < m_n && kc < ci_n) {
          if (!flip) val = W[(mrow * CIN[l] + kc) * 27 + tap];
          else val = W[(kc * CIN[l] + mrow) * 27 + (26 - tap)];
        }
      }
      out[(s * 64 + lane) * 8 + j] = f32_to_bf16(val);
    }
  }
  if (bias_out && lane < 16) bias_out[lane] = (!flip && lane < COUT[l]) ? w[boff(l) + lane] : 0.f;
}

}  // namespace net
}  // namespace tbs

// ==========================================================================================
// host side

using namespace tbs;
using namespace tbs::net;

namespace {

constexpr int kPartBlocks = 1024;   // weight-gradient partial rows
constexpr int kRedBlocks = 1024;    // blocks of the sum-of-squares / loss reductions

struct NetWs {
  // parameter block
  float* master; float* m; float* v; float* grad;
  uint16_t* wf;     // packed forward A operands, NL x PACK
  uint16_t* wb;     // packed backward-data A operands, NL x PACK
  float* bias;      // NL x 16
  double* sc;       // scales: 1/rms u, 1/rms q, output scale; loss accumulator at sc[4]
  double* red;      // reduction partials (2 x kRedBlocks)
  float* part;      // weight-gradient partial rows kPartBlocks x WG_PARTS
  // activations (per sample)
  uint32_t* x0;     // N x 2 bf16
  uint16_t* y[3];   // N x 16 bf16 (inference uses y[0], y[1] as ping-pong)
  float* z[3];      // N x 16 f32 (training)
  uint16_t* gz[2];  // N x 16 bf16 (training: gradients of pre-activations)
  uint16_t* gout;   // N bf16 (training)
  float* o;         // N f32 (network output / guess)
};

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t layout(NetWs* L, char* base, int64_t N, int training) {
  size_t o = 0;
  auto take = [&](size_t bytes) { char* p = base ? base + o : nullptr; o += a256(bytes); return p; };
  const size_t P = TBS_NET_PARAMS;
  NetWs w{};
  w.master = (float*)take(P * 4); w.m = (float*)take(P * 4); w.v = (float*)take(P * 4); w.grad = (float*)take(P * 4);
  w.wf = (uint16_t*)take((size_t)NL * PACK * 2); w.wb = (uint16_t*)take((size_t)NL * PACK * 2);
  w.bias = (float*)take(NL * 16 * 4);
  w.sc = (double*)take(8 * 8);
  w.red = (double*)take(2 * kRedBlocks * 8);
  w.part = (float*)take(training ? (size_t)kPartBlocks * WG_PARTS * 4 : 0);
  w.x0 = (uint32_t*)take((size_t)N * 4);
  w.y[0] = (uint16_t*)take((size_t)N * 32);
  w.y[1] = (uint16_t*)take((size_t)N * 32);
  w.y[2] = (uint16_t*)take(training ? (size_t)N * 32 : 0);
  for (int i = 0; i < 3; ++i) w.z[i] = (float*)take(training ? (size_t)N * 64 : 0);
  for (int i = 0; i < 2; ++i) w.gz[i] = (uint16_t*)take(training ? (size_t)N * 32 : 0);
  w.gout = (uint16_t*)take(training ? (size_t)N * 2 : 0);
  w.o = (float*)take((size_t)N * 4);
  if (L) *L = w;
  return o;
}

thread_local char g_err[256];
int err(int code, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return code;
}

}  // namespace

struct tbs_net {
  hipStream_t st;
  char* ws;
  size_t ws_bytes;
  int64_t grid[3];
  int batch, training;
  NetWs w;
  int step;           // Adam step count
  double out_scale;
  double lr;
  int weights_set;
};

#define NCHK(expr)                                                        \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) return err(TBS_E_HIP, hipGetErrorString(e_));   \
  } while (0)

static bool aligned256(const void* p) { return p && ((uintptr_t)p & 255u) == 0; }

extern "C" int tbs_net_create(tbs_net** out, void* stream) {
  if (!out) return TBS_E_INVAL;
  tbs_net* n = new (std::nothrow) tbs_net();
  if (!n) return TBS_E_INVAL;
  n->st = (hipStream_t)stream;
  n->out_scale = 1.0;
  n->lr = 1e-3;
  *out = n;
  return TBS_OK;
}

extern "C" void tbs_net_destroy(tbs_net* n) { delete n; }

extern "C" size_t tbs_net_workspace_bytes(const int64_t grid[3], int batch, int training) {
  if (!grid || grid[0] < 1 || grid[1] < 1 || grid[2] < 1 || batch < 1) return 0;
  return layout(nullptr, nullptr, grid[0] * grid[1] * grid[2], training);
}

extern "C" int tbs_net_bind_workspace(tbs_net* n, const int64_t grid[3], int batch, int training, void* p,
                                      size_t bytes) {
  if (!n || !grid || batch < 1) return TBS_E_INVAL;
  if (!aligned256(p)) return TBS_E_INVAL;
  const size_t need = tbs_net_workspace_bytes(grid, batch, training);
  if (need == 0 || bytes < need) return TBS_E_NOMEM;
  const bool keep = n->ws && n->weights_set;
  float host_params[TBS_NET_PARAMS];
  float host_m[TBS_NET_PARAMS], host_v[TBS_NET_PARAMS];
  if (keep) {
    // carry the parameter block (weights and Adam moments) over to the new workspace
    NCHK(hipMemcpyAsync(host_params, n->w.master, sizeof(host_params), hipMemcpyDeviceToHost, n->st));
    NCHK(hipMemcpyAsync(host_m, n->w.m, sizeof(host_m), hipMemcpyDeviceToHost, n->st));
    NCHK(hipMemcpyAsync(host_v, n->w.v, sizeof(host_v), hipMemcpyDeviceToHost, n->st));
    NCHK(hipStreamSynchronize(n->st));
  }
  n->ws = (char*)p;
  n->ws_bytes = bytes;
  for (int d = 0; d < 3; ++d) n->grid[d] = grid[d];
  n->batch = batch;
  n->training = training;
  layout(&n->w, n->ws, grid[0] * grid[1] * grid[2], training);
  if (keep) {
    NCHK(hipMemcpyAsync(n->w.master, host_params, sizeof(host_params), hipMemcpyHostToDevice, n->st));
    NCHK(hipMemcpyAsync(n->w.m, host_m, sizeof(host_m), hipMemcpyHostToDevice, n->st));
    NCHK(hipMemcpyAsync(n->w.v, host_v, sizeof(host_v), hipMemcpyHostToDevice, n->st));
    for (int l = 0; l < NL; ++l) {
      hipLaunchKernelGGL(pack_weights, dim3(1), dim3(64), 0, n->st, n->w.master, l, 0, n->w.wf + l * PACK, n->w.bias + l * 16);
      hipLaunchKernelGGL(pack_weights, dim3(1), dim3(64), 0, n->st, n->w.master, l, 1, n->w.wb + l * PACK, nullptr);
    }
    NCHK(hipStreamSynchronize(n->st));
  } else {
    n->weights_set = 0;
  }
  return TBS_OK;
}

static int repack(tbs_net* n) {
  for (int l = 0; l < NL; ++l) {
    hipLaunchKernelGGL(pack_weights, dim3(1), dim3(64), 0, n->st, n->w.master, l, 0, n->w.wf + l * PACK, n->w.bias + l * 16);
    hipLaunchKernelGGL(pack_weights, dim3(1), dim3(64), 0, n->st, n->w.master, l, 1, n->w.wb + l * PACK, nullptr);
  }
  NCHK(hipGetLastError());
  return TBS_OK;
}

extern "C" int tbs_net_set_weights(tbs_net* n, const float* host, size_t count) {
  if (!n || !host || count != TBS_NET_PARAMS) return TBS_E_INVAL;
  if (!n->ws) return TBS_E_NOMEM;
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(host[i])) return err(TBS_E_INVAL, "non-finite weight");
  NCHK(hipMemcpyAsync(n->w.master, host, count * 4, hipMemcpyHostToDevice, n->st));
  NCHK(hipMemsetAsync(n->w.m, 0, count * 4, n->st));
  NCHK(hipMemsetAsync(n->w.v, 0, count * 4, n->st));
  n->step = 0;
  int rc = repack(n);
  if (rc) return rc;
  NCHK(hipStreamSynchronize(n->st));
  n->weights_set = 1;
  return TBS_OK;
}

extern "C" int tbs_net_get_weights(const tbs_net* n, float* host, size_t count) {
  if (!n || !host || count != TBS_NET_PARAMS) return TBS_E_INVAL;
  if (!n->ws || !n->weights_set) return TBS_E_STATE;
  NCHK(hipMemcpyAsync(host, n->w.master, count * 4, hipMemcpyDeviceToHost, n->st));
  NCHK(hipStreamSynchronize(n->st));
  return TBS_OK;
}

extern "C" int tbs_net_set_hparams(tbs_net* n, double out_scale, double lr) {
  if (!n || !(out_scale > 0) || !(lr > 0) || !std::isfinite(out_scale) || !std::isfinite(lr)) return TBS_E_INVAL;
  n->out_scale = out_scale;
  n->lr = lr;
  return TBS_OK;
}

static int check_grid(const tbs_net* n, const int64_t grid[3]) {
  if (!n->ws) return err(TBS_E_NOMEM, "no workspace bound");
  if (!n->weights_set) return err(TBS_E_STATE, "weights not set");
  for (int d = 0; d < 3; ++d)
    if (grid[d] != n->grid[d]) return err(TBS_E_INVAL, "grid differs from the bound workspace");
  return TBS_OK;
}

// one workgroup per (32 x 8 column, z-chunk)
static int conv_blocks(const int64_t grid[3]) {
  const Grid3 g{(int)grid[0], (int)grid[1], (int)grid[2], 0};
  const ConvGeo c = conv_geo(g);
  return c.tx * c.ty * c.nch;
}

static int smooth(tbs_net* n, float* buf, float* tmp, Grid3 g);

// forward of one sample; x0 already prepared.  keep = training (store z and all y, and leave the
// network output unscaled for the loss); otherwise the output is the guess du = o * sc[2].
static int forward_layers(tbs_net* n, Grid3 g, int keep) {
  const int64_t grid[3] = {g.nx, g.ny, g.nz};
  const int nb = conv_blocks(grid);
  NetWs& w = n->w;
  uint16_t* y0 = keep ? w.y[0] : w.y[0];
  uint16_t* y1 = keep ? w.y[1] : w.y[1];
  uint16_t* y2 = keep ? w.y[2] : w.y[0];
  hipLaunchKernelGGL((conv_mfma<2, 16, EPI_GELU>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)w.x0, w.wf,
                     w.bias, g, keep ? w.z[0] : nullptr, y0, nullptr, nullptr, nullptr);
  hipLaunchKernelGGL((conv_mfma<16, 16, EPI_GELU>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)y0,
                     w.wf + PACK, w.bias + 16, g, keep ? w.z[1] : nullptr, y1, nullptr, nullptr, nullptr);
  hipLaunchKernelGGL((conv_mfma<16, 16, EPI_GELU>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)y1,
                     w.wf + 2 * PACK, w.bias + 32, g, keep ? w.z[2] : nullptr, y2, nullptr, nullptr, nullptr);
  hipLaunchKernelGGL((conv_mfma<16, 1, EPI_LINEAR>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)y2,
                     w.wf + 3 * PACK, w.bias + 48, g, nullptr, nullptr, w.o, nullptr,
                     (const double*)(w.sc + (keep ? 3 : 2)));
  NCHK(hipGetLastError());
  // output low-pass (linear, so it commutes with the output scale); scratch: a free activation buffer
  return smooth(n, w.o, keep ? (float*)w.gz[0] : (float*)w.y[1], g);
}

// buf <- B^SMOOTH_PASSES buf with B = Bx By Bz the binomial low-pass; tmp is scratch of N floats
static int smooth(tbs_net* n, float* buf, float* tmp, Grid3 g) {
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  const int zc = smooth_zchunk(g);
  const int sblocks = ((g.nx + SMX - 1) / SMX) * ((g.ny + SMY - 1) / SMY) * ((g.nz + zc - 1) / zc);
  float* a = buf;
  float* b = tmp;
  for (int p = 0; p < SMOOTH_PASSES; ++p) {
    hipLaunchKernelGGL(smooth3, dim3(sblocks), dim3(256), 0, n->st, (const float*)a, b, g, zc);
    float* t = a; a = b; b = t;
  }
  if (a != buf) NCHK(hipMemcpyAsync(buf, a, (size_t)N * 4, hipMemcpyDeviceToDevice, n->st));
  NCHK(hipGetLastError());
  return TBS_OK;
}

template <typename T>
static int prepare(tbs_net* n, const T* u, const T* q, int64_t N, double tau, double out_scale) {
  NetWs& w = n->w;
  hipLaunchKernelGGL(sumsq_partial<T>, dim3(kRedBlocks), dim3(256), 0, n->st, u, q, N, w.red);
  hipLaunchKernelGGL(scales_final, dim3(1), dim3(64), 0, n->st, (const double*)w.red, kRedBlocks, N, tau, out_scale,
                     w.sc);
  hipLaunchKernelGGL(prep_input<T>, dim3(2048), dim3(256), 0, n->st, u, q, N, (const double*)w.sc, w.x0);
  NCHK(hipGetLastError());
  return TBS_OK;
}

extern "C" int tbs_net_forward(tbs_net* n, const void* u, const void* q, int dtype, float* du, int periodic,
                               double tau) {
  if (!n || !aligned256(u) || !aligned256(du) || (q && !aligned256(q))) return TBS_E_INVAL;
  if (dtype != TBS_F64 && dtype != TBS_F32) return TBS_E_INVAL;
  if (!(tau > 0)) return TBS_E_INVAL;
  int rc = check_grid(n, n->grid);
  if (rc) return rc;
  const int64_t N = n->grid[0] * n->grid[1] * n->grid[2];
  Grid3 g{(int)n->grid[0], (int)n->grid[1], (int)n->grid[2], periodic ? 1 : 0};
  rc = dtype == TBS_F64 ? prepare(n, (const double*)u, (const double*)q, N, tau, n->out_scale)
                        : prepare(n, (const float*)u, (const float*)q, N, tau, n->out_scale);
  if (rc) return rc;
  rc = forward_layers(n, g, 0);
  if (rc) return rc;
  if (du != n->w.o) NCHK(hipMemcpyAsync(du, n->w.o, (size_t)N * 4, hipMemcpyDeviceToDevice, n->st));
  return TBS_OK;
}

int tbs_net_guess_internal(tbs_net* n, const int64_t grid[3], int periodic, double tau, hipStream_t st,
                           const double* u_prev, const double* q, const float** du_out) {
  if (!n) return TBS_E_INVAL;
  int rc = check_grid(n, grid);
  if (rc) return rc;
  if (n->st != st) return err(TBS_E_INVAL, "network and solver must share one stream");
  const int64_t N = grid[0] * grid[1] * grid[2];
  Grid3 g{(int)grid[0], (int)grid[1], (int)grid[2], periodic ? 1 : 0};
  rc = prepare(n, u_prev, q, N, tau, n->out_scale);
  if (rc) return rc;
  rc = forward_layers(n, g, 0);
  if (rc) return rc;
  *du_out = n->w.o;
  return TBS_OK;
}

extern "C" int tbs_net_train_step(tbs_net* n, const float* u, const float* q, const float* du_t, int batch,
                                  int periodic, double tau, float* loss_out) {
  if (!n || !aligned256(u) || !aligned256(du_t) || (q && !aligned256(q)) || batch < 1) return TBS_E_INVAL;
  if (!(tau > 0)) return TBS_E_INVAL;
  int rc = check_grid(n, n->grid);
  if (rc) return rc;
  if (!n->training) return err(TBS_E_STATE, "workspace bound without training buffers");
  const int64_t N = n->grid[0] * n->grid[1] * n->grid[2];
  Grid3 g{(int)n->grid[0], (int)n->grid[1], (int)n->grid[2], periodic ? 1 : 0};
  NetWs& w = n->w;
  const int nb = conv_blocks(n->grid);
  const double inv_total = 1.0 / ((double)N * batch);
  const int wblocks = kPartBlocks;
  for (int b = 0; b < batch; ++b) {
    const float* ub = u + (size_t)b * N;
    const float* qb = q ? q + (size_t)b * N : nullptr;
    const float* tb = du_t + (size_t)b * N;
    rc = prepare(n, ub, qb, N, tau, n->out_scale);
    if (rc) return rc;
    rc = forward_layers(n, g, 1);
    if (rc) return rc;
    float* gtmp = (float*)w.gz[0];
    hipLaunchKernelGGL(mse_grad, dim3(kRedBlocks), dim3(256), 0, n->st, (const float*)w.o, tb, N,
                       (const double*)w.sc, inv_total, gtmp, w.red);
    rc = smooth(n, gtmp, (float*)w.gz[1], g);  // adjoint of the output filter (it is symmetric)
    if (rc) return rc;
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(2048), dim3(256), 0, n->st, (const float*)gtmp, w.gout, N);
    hipLaunchKernelGGL(loss_final, dim3(1), dim3(64), 0, n->st, (const double*)w.red, kRedBlocks, inv_total,
                       w.sc + 4, b > 0);
    const int acc = b > 0;
    // layer 4: dW4 = sum y3 (x) g ; dZ3 = convT(g, W4) * GELU'(z3)
    hipLaunchKernelGGL((wgrad_partial<16, 1>), dim3(wblocks), dim3(256), 0, n->st, (const uint16_t*)w.y[2],
                       (const uint16_t*)w.gout, g, w.part, 0);
    hipLaunchKernelGGL(wgrad_reduce, dim3((16 * 27 + 1 + 255) / 256), dim3(256), 0, n->st, (const float*)w.part,
                       wblocks, 16 * 27 + 1, w.grad + woff(3), acc);
    hipLaunchKernelGGL((conv_mfma<1, 16, EPI_BWD>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)w.gout,
                       w.wb + 3 * PACK, nullptr, g, nullptr, w.gz[0], nullptr, (const float*)w.z[2], nullptr);
    // layer 3: dW3 = sum y2 (x) dZ3 ; dZ2 = convT(dZ3, W3) * GELU'(z2)
    hipLaunchKernelGGL((wgrad_partial<16, 16>), dim3(wblocks), dim3(256), 0, n->st, (const uint16_t*)w.y[1],
                       (const uint16_t*)w.gz[0], g, w.part, 0);
    hipLaunchKernelGGL(wgrad_reduce, dim3((16 * 16 * 27 + 16 + 255) / 256), dim3(256), 0, n->st,
                       (const float*)w.part, wblocks, 16 * 16 * 27 + 16, w.grad + woff(2), acc);
    hipLaunchKernelGGL((conv_mfma<16, 16, EPI_BWD>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)w.gz[0],
                       w.wb + 2 * PACK, nullptr, g, nullptr, w.gz[1], nullptr, (const float*)w.z[1], nullptr);
    // layer 2: dW2 = sum y1 (x) dZ2 ; dZ1 = convT(dZ2, W2) * GELU'(z1)
    hipLaunchKernelGGL((wgrad_partial<16, 16>), dim3(wblocks), dim3(256), 0, n->st, (const uint16_t*)w.y[0],
                       (const uint16_t*)w.gz[1], g, w.part, 0);
    hipLaunchKernelGGL(wgrad_reduce, dim3((16 * 16 * 27 + 16 + 255) / 256), dim3(256), 0, n->st,
                       (const float*)w.part, wblocks, 16 * 16 * 27 + 16, w.grad + woff(1), acc);
    hipLaunchKernelGGL((conv_mfma<16, 16, EPI_BWD>), dim3(nb), dim3(256), 0, n->st, (const uint16_t*)w.gz[1],
                       w.wb + PACK, nullptr, g, nullptr, w.gz[0], nullptr, (const float*)w.z[0], nullptr);
    // layer 1: dW1 = sum x0 (x) dZ1
    hipLaunchKernelGGL((wgrad_partial<2, 16>), dim3(wblocks), dim3(256), 0, n->st, (const uint16_t*)w.x0,
                       (const uint16_t*)w.gz[0], g, w.part, 0);
    hipLaunchKernelGGL(wgrad_reduce, dim3((2 * 16 * 27 + 16 + 255) / 256), dim3(256), 0, n->st,
                       (const float*)w.part, wblocks, 2 * 16 * 27 + 16, w.grad + woff(0), acc);
    NCHK(hipGetLastError());
  }
  n->step += 1;
  hipLaunchKernelGGL(adam, dim3((TBS_NET_PARAMS + 255) / 256), dim3(256), 0, n->st, w.master, w.m, w.v,
                     (const float*)w.grad, TBS_NET_PARAMS, n->step, (float)n->lr, 0.9f, 0.999f, 1e-8f);
  rc = repack(n);
  if (rc) return rc;
  if (loss_out) {
    double l = 0;
    NCHK(hipMemcpyAsync(&l, w.sc + 4, 8, hipMemcpyDeviceToHost, n->st));
    NCHK(hipStreamSynchronize(n->st));
    *loss_out = (float)l;
  }
  return TBS_OK;
}

// ------------------------------------------------------------------------------------------
// kernel-level probes for parity tests (use the bound workspace's grid)

extern "C" int tbs_net_conv_layer(tbs_net* n, int layer, int mode, const uint16_t* x, const uint16_t* gin,
                                  int periodic, float* out) {
  if (!n || layer < 0 || layer >= NL || mode < 0 || mode > 2 || !aligned256(out)) return TBS_E_INVAL;
  int rc = check_grid(n, n->grid);
  if (rc) return rc;
  Grid3 g{(int)n->grid[0], (int)n->grid[1], (int)n->grid[2], periodic ? 1 : 0};
  const int nb = conv_blocks(n->grid);
  NetWs& w = n->w;
  const int ci = CIN[layer], co = COUT[layer];
  if (mode == 0) {  // forward pre-activation z = conv(x, W) + b, out [voxel][co]
    if (!aligned256(x)) return TBS_E_INVAL;
#define FWD(CI, CO) hipLaunchKernelGGL((conv_mfma<CI, CO, EPI_RAW>), dim3(nb), dim3(256), 0, n->st, x, \
                                       w.wf + layer * PACK, w.bias + layer * 16, g, nullptr, nullptr, out, nullptr, nullptr)
    if (ci == 2) FWD(2, 16);
    else if (co == 16) FWD(16, 16);
    else FWD(16, 1);
#undef FWD
  } else if (mode == 1) {  // data gradient dx = convT(g, W), out [voxel][ci]
    if (!aligned256(gin)) return TBS_E_INVAL;
#define BWD(CI, CO) hipLaunchKernelGGL((conv_mfma<CI, CO, EPI_RAW>), dim3(nb), dim3(256), 0, n->st, gin, \
                                       w.wb + layer * PACK, nullptr, g, nullptr, nullptr, out, nullptr, nullptr)
    if (co == 1) BWD(1, 16);
    else if (ci == 2) BWD(16, 2);
    else BWD(16, 16);
#undef BWD
  } else {  // weight gradient: out [co][ci][27] then [co] biases
    if (!n->training) return err(TBS_E_STATE, "weight gradients need a training workspace");
    if (!aligned256(x) || !aligned256(gin)) return TBS_E_INVAL;
    if (ci == 2) hipLaunchKernelGGL((wgrad_partial<2, 16>), dim3(kPartBlocks), dim3(256), 0, n->st, x, gin, g, w.part, 0);
    else if (co == 16) hipLaunchKernelGGL((wgrad_partial<16, 16>), dim3(kPartBlocks), dim3(256), 0, n->st, x, gin, g, w.part, 0);
    else hipLaunchKernelGGL((wgrad_partial<16, 1>), dim3(kPartBlocks), dim3(256), 0, n->st, x, gin, g, w.part, 0);
    const int cnt = ci * co * 27 + co;
    hipLaunchKernelGGL(wgrad_reduce, dim3((cnt + 255) / 256), dim3(256), 0, n->st, (const float*)w.part,
                       kPartBlocks, cnt, out, 0);
  }
  NCHK(hipGetLastError());
  return TBS_OK;
}

// gradient of the last train step (flat parameter order) for parity tests
extern "C" int tbs_net_get_grad(const tbs_net* n, float* host, size_t count) {
  if (!n || !host || count != TBS_NET_PARAMS) return TBS_E_INVAL;
  if (!n->ws || !n->training) return TBS_E_STATE;
  NCHK(hipMemcpyAsync(host, n->w.grad, count * 4, hipMemcpyDeviceToHost, n->st));
  NCHK(hipStreamSynchronize(n->st));
  return TBS_OK;
}
