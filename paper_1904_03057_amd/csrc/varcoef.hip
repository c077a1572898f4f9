// Variable-coefficient system operator on gfx950 (Sec. 2.3: D and mu_a expanded in the solution's
// B-spline basis; Sec. 2.4: the domain kernels c_k d_m w^{klm} + c_k m_m f^{klm} of the tensor
// form; Sec. 2.5 strategy (c): computed on the fly):
//
//   F(c)_l = sum_k sum_m c_k (m_m f^{klm} + d_m w^{klm})
//          = int [ mu phi b_l + D (phi_x b_l,x / hx^2 + phi_y b_l,y / hy^2 + phi_z b_l,z / hz^2) ],
//
// phi = sum c_k b_k, mu = sum m_m b_m, D = sum d_m b_m, integrated cell by cell (grid units, the
// operator divided by hx hy hz) with Q = ceil((3n + 1) / 2) Gauss points per cell and axis, which is
// exact for the degree-3n products.  The integrals are evaluated by sum factorisation: the fields
// are interpolated to the Gauss points one axis at a time (z, then y, then x), multiplied there,
// and projected back onto the test functions in the reverse order (x, y, z).  Per cell (= per
// coefficient) this is about 6.7 k multiply-adds for cubic splines, against the (2n+1)^3 products
// of three-index kernels per output.
//
// Execution: one wave owns a strip of 64 coefficient columns (64 - 2n output columns and an
// n-column halo on each side) and kVcTileY output rows, and marches through a z-chunk cell by
// cell.  For each z-cell and z-point it marches along y: a ring of n+1 rows of the z-interpolated
// fields (per lane: its column), the y-interpolation, the x-interpolation from the n neighbouring
// lanes (cross-lane shuffles), the point products, the x-projection (partial sums handed back to
// the output lanes by shuffles), the y-projection into a ring of n+1 output rows, and finally the
// z-projection into an LDS accumulator of n+1 output planes x kVcTileY rows per lane.  A plane is
// written to memory once the z-march has passed it.  Every output sums its terms in one fixed
// order: results are independent of the launch geometry's z-chunking only up to rounding of the
// (identical) per-cell terms, and bitwise reproducible for a given geometry.
#include "common.h"
#include "varcoef.h"

namespace tbs {

template <typename T> __device__ __forceinline__ T vfma(T a, T b, T c);
template <> __device__ __forceinline__ float vfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double vfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int N, typename T, int BC>
__global__ __launch_bounds__(64) void varcoef_kernel(VarcoefArgs a, VarcoefTabF tf) {
  constexpr int Q = (3 * N + 2) / 2;
  constexpr int NB = N + 1;
  constexpr int H = N / 2;
  constexpr int TXO = 64 - 2 * N;
  constexpr int TY = kVcTileY;
  __shared__ T acc[TY * NB * 64];  // [output row][plane slot][lane]: each lane owns its column

  const int lane = threadIdx.x;
  const int bid = xcd_remap(blockIdx.x, a.nblocks);
  const int txi = bid % a.tiles_x;
  const int rest = bid / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int czi = rest / a.tiles_y;
  const int x0 = txi * TXO, y0 = tyi * TY, z0 = czi * a.zc;
  const int zc_eff = min(a.zc, a.nz - z0);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane = (int64_t)nx * ny;
  const T* __restrict__ Cc = (const T*)a.c;
  const T* __restrict__ Dc = (const T*)a.d;
  const T* __restrict__ Mc = (const T*)a.m;
  T* __restrict__ Y = (T*)a.y;

  // basis tables (uniform): value / derivative of B-spline t of a cell at Gauss point q, weights
  auto BV = [&](int q, int t) -> T { return sizeof(T) == 8 ? (T)a.bv[q * kVcMaxB + t] : (T)tf.bv[q * kVcMaxB + t]; };
  auto BD = [&](int q, int t) -> T { return sizeof(T) == 8 ? (T)a.bd[q * kVcMaxB + t] : (T)tf.bd[q * kVcMaxB + t]; };
  auto WQ = [&](int q) -> T { return sizeof(T) == 8 ? (T)a.w[q] : (T)tf.w[q]; };
  const T ihx2 = (T)a.ihx2, ihy2 = (T)a.ihy2, ihz2 = (T)a.ihz2;

  // this lane's coefficient column: c is read there (zero outside a Dirichlet box), mu and D at
  // the nearest column inside (their expansions continue by the edge coefficients)
  const int xp = x0 - N + lane;
  int xcc, xcm;
  bool xok;
  if (BC == BC_PERIODIC) {
    xcc = ((xp % nx) + nx) % nx;
    xcm = xcc;
    xok = true;
  } else {
    xok = xp >= 0 && xp < nx;
    xcc = xok ? xp : 0;
    xcm = min(max(xp, 0), nx - 1);
  }

  for (int i = lane; i < TY * NB * 64; i += 64) acc[i] = (T)0;

  const int jz0 = z0 + H - N, jz1 = z0 + zc_eff + H;  // z-cells whose support meets the chunk
  const int jy0 = y0 + H - N;                        // first y-cell of the strip's rows
  for (int jz = jz0; jz < jz1; ++jz) {
    // the n+1 coefficient planes of this z-cell
    int64_t pcz[NB], pmz[NB];
    bool zok[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int kz = jz - H + t;
      int kc, km;
      if (BC == BC_PERIODIC) {
        kc = ((kz % nz) + nz) % nz;
        km = kc;
        zok[t] = true;
      } else {
        zok[t] = kz >= 0 && kz < nz;
        kc = zok[t] ? kz : 0;
        km = min(max(kz, 0), nz - 1);
      }
      pcz[t] = (int64_t)kc * plane;
      pmz[t] = (int64_t)km * plane;
    }
    for (int zq = 0; zq < Q; ++zq) {
      T bzv[NB], bzd[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        bzv[t] = BV(zq, t);
        bzd[t] = BD(zq, t);
      }
      const T wz = WQ(zq);
      // fields at (z-point zq, coefficient row ky, this column): c value, c z-derivative, mu, D
      auto load_row = [&](int ky, T* out) {
        int kc, km;
        bool yok;
        if (BC == BC_PERIODIC) {
          kc = ((ky % ny) + ny) % ny;
          km = kc;
          yok = true;
        } else {
          yok = ky >= 0 && ky < ny;
          kc = yok ? ky : 0;
          km = min(max(ky, 0), ny - 1);
        }
        const int64_t oc = (int64_t)kc * nx + xcc, om = (int64_t)km * nx + xcm;
        T cv = (T)0, cd = (T)0, mu = (T)0, dd = (T)0;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const T c = (yok && xok && zok[t]) ? Cc[pcz[t] + oc] : (T)0;
          cv = vfma(bzv[t], c, cv);
          cd = vfma(bzd[t], c, cd);
          mu = vfma(bzv[t], Mc[pmz[t] + om], mu);
          dd = vfma(bzv[t], Dc[pmz[t] + om], dd);
        }
        out[0] = cv;
        out[1] = cd;
        out[2] = mu;
        out[3] = dd;
      };
      T zr[NB][4];   // ring of coefficient rows jy - H + t
      T ya[NB], yc[NB];  // y-projection ring of output rows jy - H + t (z-value and z-derivative parts)
#pragma unroll
      for (int t = 0; t < N; ++t) load_row(jy0 - H + t, zr[t]);
#pragma unroll
      for (int t = 0; t < NB; ++t) ya[t] = yc[t] = (T)0;
      for (int s = 0; s < TY + N; ++s) {
        const int jy = jy0 + s;
        load_row(jy - H + N, zr[N]);
#pragma unroll
        for (int yq = 0; yq < Q; ++yq) {
          // y-interpolation: c (value, y-derivative), c_z, mu, D at (yq, zq) in this column
          T f0 = (T)0, f1 = (T)0, f2 = (T)0, f3 = (T)0, f4 = (T)0;
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const T bv = BV(yq, t), bd = BD(yq, t);
            f0 = vfma(bv, zr[t][0], f0);
            f1 = vfma(bd, zr[t][0], f1);
            f2 = vfma(bv, zr[t][1], f2);
            f3 = vfma(bv, zr[t][2], f3);
            f4 = vfma(bv, zr[t][3], f4);
          }
          // the cell of this lane uses columns lane .. lane + n
          T nb[NB][5];
          nb[0][0] = f0; nb[0][1] = f1; nb[0][2] = f2; nb[0][3] = f3; nb[0][4] = f4;
#pragma unroll
          for (int t = 1; t < NB; ++t) {
            nb[t][0] = __shfl_down(f0, t, 64);
            nb[t][1] = __shfl_down(f1, t, 64);
            nb[t][2] = __shfl_down(f2, t, 64);
            nb[t][3] = __shfl_down(f3, t, 64);
            nb[t][4] = __shfl_down(f4, t, 64);
          }
          const T wyz = WQ(yq) * wz;
          T pa[NB], pb[NB], pc[NB];
#pragma unroll
          for (int t = 0; t < NB; ++t) pa[t] = pb[t] = pc[t] = (T)0;
#pragma unroll
          for (int xq = 0; xq < Q; ++xq) {
            T phi = (T)0, phx = (T)0, phy = (T)0, phz = (T)0, mu = (T)0, dd = (T)0;
#pragma unroll
            for (int t = 0; t < NB; ++t) {
              const T bv = BV(xq, t), bd = BD(xq, t);
              phi = vfma(bv, nb[t][0], phi);
              phx = vfma(bd, nb[t][0], phx);
              phy = vfma(bv, nb[t][1], phy);
              phz = vfma(bv, nb[t][2], phz);
              mu = vfma(bv, nb[t][3], mu);
              dd = vfma(bv, nb[t][4], dd);
            }
            const T wq = WQ(xq) * wyz;
            const T g0 = wq * mu * phi;
            const T wd = wq * dd;
            const T g1 = wd * ihx2 * phx, g2 = wd * ihy2 * phy, g3 = wd * ihz2 * phz;
#pragma unroll
            for (int t = 0; t < NB; ++t) {
              const T bv = BV(xq, t), bd = BD(xq, t);
              pa[t] = vfma(bv, g0, vfma(bd, g1, pa[t]));
              pb[t] = vfma(bv, g2, pb[t]);
              pc[t] = vfma(bv, g3, pc[t]);
            }
          }
          // x-projection: output column o collects partial t of the cell in lane o - t
          T ax = pa[0], bx = pb[0], cx = pc[0];
#pragma unroll
          for (int t = 1; t < NB; ++t) {
            ax += __shfl_up(pa[t], t, 64);
            bx += __shfl_up(pb[t], t, 64);
            cx += __shfl_up(pc[t], t, 64);
          }
          // y-projection onto the cell's n+1 output rows
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const T bv = BV(yq, t), bd = BD(yq, t);
            ya[t] = vfma(bv, ax, vfma(bd, bx, ya[t]));
            yc[t] = vfma(bv, cx, yc[t]);
          }
        }
        // output row jy - H has all its y-cells for this z-point: z-projection into its planes
        const int r = jy - H - y0;
        if (r >= 0 && r < TY) {
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const int slot = (((jz - H + t) % NB) + NB) % NB;
            T* p = &acc[(r * NB + slot) * 64 + lane];
            *p = vfma(bzv[t], ya[0], vfma(bzd[t], yc[0], *p));
          }
        }
#pragma unroll
        for (int t = 0; t < N; ++t) {
#pragma unroll
          for (int f = 0; f < 4; ++f) zr[t][f] = zr[t + 1][f];
          ya[t] = ya[t + 1];
          yc[t] = yc[t + 1];
        }
        ya[N] = yc[N] = (T)0;
      }
    }
    // output plane jz - H has all its z-cells: write it and clear its slot
    const int kz = jz - H;
    const int slot = ((kz % NB) + NB) % NB;
    const bool wcol = lane >= N && lane < N + TXO && xp < nx && kz >= z0 && kz < z0 + zc_eff;
    for (int r = 0; r < TY; ++r) {
      T* p = &acc[(r * NB + slot) * 64 + lane];
      if (wcol && y0 + r < ny) Y[(int64_t)kz * plane + (int64_t)(y0 + r) * nx + xp] = *p;
      *p = (T)0;
    }
  }
}

template <int N, typename T>
static hipError_t launch_nt(const VarcoefArgs& a, const VarcoefTabF& tf, int bc, hipStream_t st) {
  if (bc == BC_PERIODIC)
    hipLaunchKernelGGL((varcoef_kernel<N, T, BC_PERIODIC>), dim3(a.nblocks), dim3(64), 0, st, a, tf);
  else
    hipLaunchKernelGGL((varcoef_kernel<N, T, BC_DIRICHLET>), dim3(a.nblocks), dim3(64), 0, st, a, tf);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(const VarcoefArgs& a, int n, int bc, hipStream_t st) {
  VarcoefTabF tf;
  for (int i = 0; i < kVcMaxQ * kVcMaxB; ++i) {
    tf.bv[i] = (float)a.bv[i];
    tf.bd[i] = (float)a.bd[i];
  }
  for (int i = 0; i < kVcMaxQ; ++i) tf.w[i] = (float)a.w[i];
  switch (n) {
    case 1: return launch_nt<1, T>(a, tf, bc, st);
    case 2: return launch_nt<2, T>(a, tf, bc, st);
    case 3: return launch_nt<3, T>(a, tf, bc, st);
    case 4: return launch_nt<4, T>(a, tf, bc, st);
    case 5: return launch_nt<5, T>(a, tf, bc, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_varcoef(const VarcoefArgs& a, int n, int bc, int dt, hipStream_t st) {
  if (dt == 0) return launch_t<double>(a, n, bc, st);
  if (dt == 1) return launch_t<float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

}  // namespace tbs
