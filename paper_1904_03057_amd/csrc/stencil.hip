// On-the-fly tensor B-spline operator for gfx950: the paper's separable domain kernels
// (Sec. 2.4: w = (1/h^2)(w x f x f + f x w x f + f x f x w), f = f x f x f) applied as a
// cascade of 1-D filters (Fig. FiltAlg), computed at run time (Sec. 2.5, strategy (c)).
//
// Factorisation used here (7 filter passes instead of the 12 of the plain cascade):
//   x-pass  U = Mx u,            V = (Mx + ax Kx) u
//   y-pass  P = My U,            R = My V + ay Ky U
//   z-pass  y = Mz R + az Kz P
// which expands to (Mx My Mz + ax Kx My Mz + ay Mx Ky Mz + az Mx My Kz) u.  Symmetric taps are
// applied to pair sums (u_{i-j} + u_{i+j}).
//
// Execution ("2.5-D" streaming): a 256-thread workgroup owns a 64 x TY tile of the x-y plane
// and marches along z through its chunk.  Each input plane tile (with an n-wide halo) is staged
// in LDS, the x-pass and y-pass run from LDS, and the z-pass is accumulated in registers into
// the 2n+1 output planes a plane touches (ring of 2n+1 register slots, loop unrolled by 2n+1).
// The next plane's global loads are issued before the current plane is filtered.
#include "common.h"
#include "stencil.h"

namespace tbs {

template <int N>
struct TapReg {
  // taps in compute precision, kept in scalar registers
  double m[N + 1], mx[N + 1], ays[N + 1], azs[N + 1];
};

template <int N, int TY, int MODE, typename Tin, typename Tc, typename Tout, int BC>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs a) {
  constexpr int TX = 64;
  constexpr int R = TY + 2 * N;      // staged rows
  constexpr int C = TX + 2 * N;      // staged columns
  constexpr int T = 2 * N + 1;       // taps
  constexpr int NE = (R * C + 255) / 256;
  constexpr int RPW = TY / 4;        // output rows per wave
  static_assert(TY % 4 == 0, "TY must be a multiple of 4");

  __shared__ Tc stage[R * C];
  __shared__ Tc su[R * TX];
  __shared__ Tc sv[R * TX];
  __shared__ double red[2][4];

  if (MODE == M_CG1 && a.scal->done) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  const int bid = xcd_remap(blockIdx.x, a.nblocks);
  const int tyi = bid % a.tiles_y;
  const int rest = bid / a.tiles_y;
  const int txi = rest % a.tiles_x;
  const int czi = rest / a.tiles_x;
  const int x0 = txi * TX, y0 = tyi * TY, z0 = czi * a.zc;
  const int zc_eff = min(a.zc, a.nz - z0);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane = (int64_t)nx * ny;

  // taps in compute precision
  Tc m[N + 1], mx[N + 1], ays[N + 1], azs[N + 1];
#pragma unroll
  for (int j = 0; j <= N; ++j) {
    m[j] = (Tc)a.t.m[j];
    mx[j] = (Tc)(a.t.m[j] + a.t.ax * a.t.s[j]);
    ays[j] = (Tc)(a.t.ay * a.t.s[j]);
    azs[j] = (Tc)(a.t.az * a.t.s[j]);
  }

  // plane-invariant staging offsets of this thread's elements
  int off[NE];
  uint32_t valid = 0, own = 0;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int idx = tid + 256 * e;
    off[e] = 0;
    if (idx < R * C) {
      const int r = idx / C, c = idx - (idx / C) * C;
      int gx = x0 - N + c, gy = y0 - N + r;
      bool ok;
      if (BC == BC_PERIODIC) {
        gx %= nx; if (gx < 0) gx += nx;
        gy %= ny; if (gy < 0) gy += ny;
        ok = true;
      } else {
        ok = (gx >= 0 && gx < nx && gy >= 0 && gy < ny);
      }
      if (ok) {
        valid |= 1u << e;
        off[e] = gy * nx + gx;
      }
      if (r >= N && r < N + TY && c >= N && c < N + TX && x0 + c - N < nx && y0 + r - N < ny) own |= 1u << e;
    }
  }

  const Tc beta = (MODE == M_CG1 && !a.first) ? (Tc)a.scal->beta : (Tc)0;
  const Tc alpha_prev = (MODE == M_CG1) ? (Tc)a.scal->alpha : (Tc)0;
  const bool xupd = (MODE == M_CG1) && a.io0 != nullptr && !a.first && a.scal->pending;
  const Tc tauc = (Tc)a.t.tau;

  Tc pre[NE];
  // Load (and transform) input plane k into pre[]; own-point side effects for CG1.
  auto load_plane = [&](int k) {
    bool pvalid = true;
    int kk = k;
    if (BC == BC_PERIODIC) {
      kk %= nz; if (kk < 0) kk += nz;
    } else {
      pvalid = (k >= 0 && k < nz);
    }
    const bool inchunk = (k >= z0 && k < z0 + zc_eff);
    const int64_t base = (int64_t)kk * plane;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      Tc v = (Tc)0;
      if (pvalid && ((valid >> e) & 1u)) {
        const int64_t gi = base + off[e];
        if (MODE == M_APPLY) {
          v = Io<Tin>::template ld<Tc>(a.in0, gi);
        } else if (MODE == M_RHS) {
          v = Io<Tin>::template ld<Tc>(a.in0, gi);
          if (a.in1) v += tauc * Io<Tin>::template ld<Tc>(a.in1, gi);
        } else if (MODE == M_CG1) {
          const Tc r = Io<Tc>::template ld<Tc>(a.in0, gi);
          Tc pold = (Tc)0;
          if (!a.first) pold = Io<Tin>::template ld<Tc>(a.in1, gi);
          v = storage_round<Tin, Tc>(r + beta * pold);
          if (inchunk && ((own >> e) & 1u)) {
            Io<Tin>::template st<Tc>(a.out1, gi, v);
            if (xupd) {
              Tc* x = (Tc*)a.io0;
              x[gi] = x[gi] + alpha_prev * pold;
            }
          }
        } else {  // M_RESID
          v = Io<Tin>::template ld<Tc>(a.in0, gi);
        }
      }
      pre[e] = v;
    }
  };

  Tc acc[T][RPW];
  Tc cq[T][RPW];
#pragma unroll
  for (int s = 0; s < T; ++s)
#pragma unroll
    for (int i = 0; i < RPW; ++i) { acc[s][i] = (Tc)0; cq[s][i] = (Tc)0; }

  double part0 = 0.0, part1 = 0.0;
  const int gxo = x0 + lane;
  const bool colown = gxo < nx;

  const int kbeg = z0 - N, kend = z0 + zc_eff + N;
  load_plane(kbeg);
  for (int kb = kbeg; kb < kend; kb += T) {
#pragma unroll
    for (int ph = 0; ph < T; ++ph) {
      const int k = kb + ph;
      if (k >= kend) break;
      const bool active = (BC == BC_PERIODIC) || (k >= 0 && k < nz);
      if (active) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          const int idx = tid + 256 * e;
          if (idx < R * C) stage[idx] = pre[e];
        }
      }
      __syncthreads();
      if (k + 1 < kend) load_plane(k + 1);
      if (active) {
        if (MODE == M_CG1) {
#pragma unroll
          for (int i = 0; i < RPW; ++i) cq[ph][i] = stage[(wave * RPW + i + N) * C + lane + N];
        }
        // x-pass over all R staged rows (rows dealt to waves round-robin)
        for (int r = wave; r < R; r += 4) {
          const Tc* row = stage + r * C + lane;
          const Tc c0 = row[N];
          Tc U = m[0] * c0, V = mx[0] * c0;
#pragma unroll
          for (int j = 1; j <= N; ++j) {
            const Tc sm = row[N - j] + row[N + j];
            U += m[j] * sm;
            V += mx[j] * sm;
          }
          su[r * TX + lane] = U;
          sv[r * TX + lane] = V;
        }
      }
      __syncthreads();
      if (active) {
        Tc uc[RPW + 2 * N], vc[RPW + 2 * N];
#pragma unroll
        for (int j = 0; j < RPW + 2 * N; ++j) {
          uc[j] = su[(wave * RPW + j) * TX + lane];
          vc[j] = sv[(wave * RPW + j) * TX + lane];
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          Tc P = m[0] * uc[i + N];
          Tc Rr = m[0] * vc[i + N] + ays[0] * uc[i + N];
#pragma unroll
          for (int j = 1; j <= N; ++j) {
            const Tc pu = uc[i + N - j] + uc[i + N + j];
            const Tc pv = vc[i + N - j] + vc[i + N + j];
            P += m[j] * pu;
            Rr += m[j] * pv + ays[j] * pu;
          }
          // plane k adds to outputs k+d, d = -N..N, in ring slot (ph + d) mod T
#pragma unroll
          for (int d = -N; d <= N; ++d) {
            const int s = (ph + d + 2 * T) % T;
            const int ad = d < 0 ? -d : d;
            if (MODE == M_RHS) acc[s][i] += m[ad] * P;
            else acc[s][i] += m[ad] * Rr + azs[ad] * P;
          }
        }
      }
      // output plane o = k - N is complete
      {
        constexpr int dummy = 0;
        (void)dummy;
        const int so = (ph - N + 2 * T) % T;
        const int o = k - N;
        if (o >= z0) {
          const int64_t obase = (int64_t)o * plane;
#pragma unroll
          for (int i = 0; i < RPW; ++i) {
            const int gy = y0 + wave * RPW + i;
            if (colown && gy < ny) {
              const int64_t gi = obase + (int64_t)gy * nx + gxo;
              const Tc val = acc[so][i];
              if (MODE == M_APPLY || MODE == M_RHS) {
                Io<Tout>::template st<Tc>(a.out0, gi, val);
              } else if (MODE == M_CG1) {
                Io<Tout>::template st<Tc>(a.out0, gi, val);
                part0 += (double)cq[so][i] * (double)val;
              } else {
                const double b = a.bvec[gi];
                const double r = b - (double)val;
                if (a.out0) Io<Tout>::template st<double>(a.out0, gi, r);
                part0 += r * r;
                part1 += b * b;
              }
            }
          }
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) acc[so][i] = (Tc)0;
      }
    }
  }

  if (MODE == M_CG1 || MODE == M_RESID) {
    part0 = wave_sum(part0);
    part1 = wave_sum(part1);
    if (lane == 0) { red[0][wave] = part0; red[1][wave] = part1; }
    __syncthreads();
    if (tid == 0) {
      a.part0[blockIdx.x] = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
      if (MODE == M_RESID) a.part1[blockIdx.x] = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
    }
  }
}

// ------------------------------------------------------------------------------------------
// host-side launch helpers

template <int N, int TY, int MODE, typename Tin, typename Tc, typename Tout>
static hipError_t launch_bc(const StencilArgs& a, int bc, hipStream_t st) {
  dim3 grid(a.nblocks), block(256);
  if (bc == BC_PERIODIC)
    hipLaunchKernelGGL((stencil_kernel<N, TY, MODE, Tin, Tc, Tout, BC_PERIODIC>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((stencil_kernel<N, TY, MODE, Tin, Tc, Tout, BC_DIRICHLET>), grid, block, 0, st, a);
  return hipGetLastError();
}

template <int MODE, typename Tin, typename Tc, typename Tout>
static hipError_t launch_n(const StencilArgs& a, int n, int bc, hipStream_t st) {
  constexpr int TY = STENCIL_TY;
  switch (n) {
    case 1: return launch_bc<1, TY, MODE, Tin, Tc, Tout>(a, bc, st);
    case 2: return launch_bc<2, TY, MODE, Tin, Tc, Tout>(a, bc, st);
    case 3: return launch_bc<3, TY, MODE, Tin, Tc, Tout>(a, bc, st);
    case 4: return launch_bc<4, TY, MODE, Tin, Tc, Tout>(a, bc, st);
    case 5: return launch_bc<5, TY, MODE, Tin, Tc, Tout>(a, bc, st);
  }
  return hipErrorInvalidValue;
}

// dtype codes: 0 = f64, 1 = f32, 2 = bf16
hipError_t launch_apply(const StencilArgs& a, int n, int bc, int in_dt, int out_dt, hipStream_t st) {
  if (in_dt == 0 && out_dt == 0) return launch_n<M_APPLY, double, double, double>(a, n, bc, st);
  if (in_dt == 1 && out_dt == 1) return launch_n<M_APPLY, float, float, float>(a, n, bc, st);
  if (in_dt == 2 && out_dt == 1) return launch_n<M_APPLY, uint16_t, float, float>(a, n, bc, st);
  if (in_dt == 1 && out_dt == 0) return launch_n<M_APPLY, float, double, double>(a, n, bc, st);
  if (in_dt == 2 && out_dt == 0) return launch_n<M_APPLY, uint16_t, double, double>(a, n, bc, st);
  return hipErrorInvalidValue;
}

hipError_t launch_rhs(const StencilArgs& a, int n, int bc, int dt, hipStream_t st) {
  if (dt == 0) return launch_n<M_RHS, double, double, double>(a, n, bc, st);
  if (dt == 1) return launch_n<M_RHS, float, float, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

// CG1: dt = 0 (all f64), 1 (all f32), 2 (f32 with p stored as bf16)
hipError_t launch_cg1(const StencilArgs& a, int n, int bc, int dt, hipStream_t st) {
  if (dt == 0) return launch_n<M_CG1, double, double, double>(a, n, bc, st);
  if (dt == 1) return launch_n<M_CG1, float, float, float>(a, n, bc, st);
  if (dt == 2) return launch_n<M_CG1, uint16_t, float, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

// RESID: FP64 x and b; r written as f64 (r_dt 0) or f32 (r_dt 1) when out0 != NULL
hipError_t launch_resid(const StencilArgs& a, int n, int bc, int r_dt, hipStream_t st) {
  if (r_dt == 0) return launch_n<M_RESID, double, double, double>(a, n, bc, st);
  if (r_dt == 1) return launch_n<M_RESID, double, double, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

}  // namespace tbs
