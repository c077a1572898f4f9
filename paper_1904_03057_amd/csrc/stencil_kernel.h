#pragma once
// Stencil kernel template (private to the stencil translation units: stencil_inst.hip instantiates
// it once per basis degree and boundary condition, so those compile in parallel; the dtype / mode
// dispatch lives in stencil.hip).
//
// On-the-fly tensor B-spline operator for gfx950: the paper's separable domain kernels
// (Sec. 2.4: w = (1/h^2)(w x f x f + f x w x f + f x f x w), f = f x f x f) applied as a
// cascade of 1-D filters (Fig. FiltAlg), computed at run time (Sec. 2.5, strategy (c)).
//
// Factorisation used here (7 filter passes instead of the 12 of the plain cascade):
//   x-pass  U = Mx u,            V = (Mx + ax Kx) u
//   y-pass  P = My U,            R = My V + ay Ky U
//   z-pass  y = Mz R + az Kz P
// which expands to (Mx My Mz + ax Kx My Mz + ay Mx Ky Mz + az Mx My Kz) u.  Symmetric taps are
// applied to pair sums (u_{i-j} + u_{i+j}), and every accumulation is an explicit FMA chain.
//
// Execution ("2.5-D" streaming): a workgroup of WX x WY waves (WX column groups of 64 lanes, WY row
// groups of TY / WY rows) owns a 64 WX x TY tile of the x-y plane and marches along z through its chunk of planes.  Each input plane tile (halo n rows in y, halo HX
// columns in x, HX = n rounded up to the 16-byte vector width) is fetched with 16-byte loads
// one plane ahead into registers, converted/transformed and staged in LDS.  The x-pass (lanes =
// columns) and the y-pass (a register column window per thread) run from LDS; the z-pass is
// accumulated in registers into the 2n+1 output planes each input plane touches (a ring of 2n+1
// register slots, loop unrolled by 2n+1 so every slot index is a compile-time constant).
#include "common.h"
#include "stencil.h"

namespace tbs {

template <typename T> __device__ __forceinline__ T fmad(T a, T b, T c);
template <> __device__ __forceinline__ float fmad<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmad<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// VE consecutive elements (one 16-byte access for the staged input, or a single element).
template <typename T, int VE> struct alignas(sizeof(T) * VE) VecN { T x[VE]; };

template <typename Ts, typename Tc> __device__ __forceinline__ Tc to_c(Ts v) { return (Tc)v; }
template <> __device__ __forceinline__ float to_c<uint16_t, float>(uint16_t v) { return bf16_to_f32(v); }
template <> __device__ __forceinline__ double to_c<uint16_t, double>(uint16_t v) { return (double)bf16_to_f32(v); }
template <typename Ts, typename Tc> __device__ __forceinline__ Ts from_c(Tc v) { return (Ts)v; }
template <> __device__ __forceinline__ uint16_t from_c<uint16_t, float>(float v) { return f32_to_bf16(v); }

template <int N, int TY, int MODE, typename Tin, typename Tc, typename Tout, int BC, bool VEC, int WX, int WY>
__global__ __launch_bounds__(64 * WX * WY) __attribute__((amdgpu_waves_per_eu(BC == BC_ROBIN ? 2 : 1))) void stencil_kernel(StencilArgs a) {
  constexpr int NT = 64 * WX * WY;                 // threads: WX column groups of 64 x WY row waves
  constexpr int VE = VEC ? 16 / (int)sizeof(Tin) : 1;
  using Raw = VecN<Tin, VE>;   // staged input (u, u_prev, x, p_old)
  using RawC = VecN<Tc, VE>;   // companion compute-precision vectors (q of RHS; r and x of CG1)
  constexpr int TX = 64 * WX;
  constexpr int HX = ((N + VE - 1) / VE) * VE;   // x-halo rounded to whole vectors
  constexpr int R = TY + 2 * N;                   // staged rows
  constexpr int C = TX + 2 * HX;                  // staged columns
  constexpr int CV = C / VE;                      // vectors per staged row
  constexpr int T = 2 * N + 1;                    // taps
  constexpr int CORE = TY * (TX / VE);            // vectors of the tile's own points
  constexpr int HALO = R * CV - CORE;              // halo vectors
  constexpr int NVC = (CORE + NT - 1) / NT;        // core vectors per thread (slots 0..NVC-1)
  constexpr int NVH = (HALO + NT - 1) / NT;        // halo vectors per thread
  constexpr int NV = NVC + NVH;
  constexpr int RPW = TY / WY;                     // output rows per wave
  constexpr bool CG = (MODE == M_CG1 || MODE == M_CGF);
  constexpr bool RR = (MODE == M_RHSRES);  // b = M u and r = b - A u in one pass (no Robin corners)
  constexpr bool RES = (MODE == M_RESID || RR);
  static_assert(!(RR && BC == BC_ROBIN), "the fused rhs and residual has no Robin corner terms");
  constexpr bool FUSED = (MODE == M_CGF);
  constexpr int QD = CG ? N + 1 : 1;  // depth of the centre-value rings (CG1, CGF)
  static_assert(TY % WY == 0, "TY must be a multiple of the row waves");

  __shared__ Tc stage[R * C];
  __shared__ Tc su[R * TX];
  __shared__ Tc sv[R * TX];
  __shared__ Tc cring[QD * TY * TX];  // p at the own points of the last n+1 planes (p.q)
  // CGF: r at the own points of the last n+2 planes (r.q).  It is written while a plane is staged,
  // before the barrier that follows, so it keeps one plane more than cring: the slot being written
  // is never the one the previous plane's outputs are still reading.
  constexpr int RQD = FUSED ? N + 2 : 1;
  __shared__ Tc rring[FUSED ? RQD * TY * TX : 1];
  __shared__ double red[4][WY * WX];
  // BC_ROBIN: corner blocks in compute precision (cm, cvx, cwy, cwz, each kRobinMaxZ^2)
  constexpr int RBT = kRobinMaxZ * kRobinMaxZ;
  __shared__ Tc rbt[BC == BC_ROBIN ? 4 * RBT : 1];
  __shared__ Tc zl[BC == BC_ROBIN ? (2 * (N / 2) + 1) * TY * TX : 1];
  static_assert(sizeof(stage) + sizeof(su) + sizeof(sv) + sizeof(cring) + sizeof(rring) + sizeof(red) + sizeof(rbt) +
                        sizeof(zl) <= (FUSED ? cgf_lds_bytes(N, TY, BC, (int)sizeof(Tc)) : kLdsMax),
                "LDS of the workgroup");

  if (CG && a.scal->done) return;

  if constexpr (BC == BC_ROBIN) {
    // static indices only (uniform loads of the argument block); read after the loop's first barrier
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < RBT; ++i) {
        rbt[i] = (Tc)a.rb.cm[i];
        rbt[RBT + i] = (Tc)a.rb.cvx[i];
        rbt[2 * RBT + i] = (Tc)a.rb.cwy[i];
        rbt[3 * RBT + i] = (Tc)a.rb.cwz[i];
      }
    }
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int col = (wv % WX) * 64 + lane;           // tile column of this lane
  const int wave = __builtin_amdgcn_readfirstlane(wv / WX);  // row group 0..WY-1 (wave-uniform)

  const int bid = xcd_remap(blockIdx.x, a.nblocks);
  // logical tile order (x- or y-tiles fastest, then the other, then z-chunks): the tiles an XCD
  // runs at the same time are neighbours whose halo cache lines meet in that XCD's L2
  int txi, tyi, czi;
  if (a.order == 0) {
    txi = bid % a.tiles_x;
    const int rest = bid / a.tiles_x;
    tyi = rest % a.tiles_y;
    czi = rest / a.tiles_y;
  } else {
    tyi = bid % a.tiles_y;
    const int rest = bid / a.tiles_y;
    txi = rest % a.tiles_x;
    czi = rest / a.tiles_x;
  }
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

  // plane-invariant placement of this thread's staged vectors: core (own-point) vectors in
  // slots 0..NVC-1, halo vectors (top/bottom rows, then left/right columns) after them
  int off[NV], soff[NV];
  int coff[NVC];  // CGF: tile-relative position (row * TX + column) of each core vector
  uint32_t valid = 0, own = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    int r = 0, cv = 0;
    bool present;
    if (v < NVC) {
      const int idx = tid + NT * v;
      present = idx < CORE;
      r = N + idx / (TX / VE);
      cv = HX / VE + idx % (TX / VE);
      coff[v < NVC ? v : 0] = (r - N) * TX + (cv - HX / VE) * VE;
    } else {
      int idx = tid + NT * (v - NVC);
      present = idx < HALO;
      if (idx < 2 * N * CV) {
        const int rr = idx / CV;
        r = rr < N ? rr : rr + TY;
        cv = idx % CV;
      } else {
        idx -= 2 * N * CV;
        constexpr int SV = 2 * HX / VE;
        r = N + idx / SV;
        const int sc = idx % SV;
        cv = sc < HX / VE ? sc : sc + TX / VE;
      }
    }
    off[v] = 0;
    soff[v] = present ? r * C + cv * VE : -1;
    if (present) {
      int gx = x0 - HX + cv * VE, gy = y0 - N + r;
      bool ok;
      if (BC == BC_PERIODIC) {
        gx %= nx; if (gx < 0) gx += nx;
        gy %= ny; if (gy < 0) gy += ny;
        ok = true;
      } else {
        ok = (gx >= 0 && gx < nx && gy >= 0 && gy < ny);
      }
      if (ok) {
        valid |= 1u << v;
        off[v] = gy * nx + gx;
      }
      if (v < NVC && x0 + cv * VE - HX < nx && y0 + r - N < ny) own |= 1u << v;
    }
  }

  const Tc beta = (CG && !a.first) ? (Tc)a.scal->beta : (Tc)0;
  const Tc alpha_prev = CG ? (Tc)a.scal->alpha : (Tc)0;
  // lazy x update: CG1 applies the one pending update alpha p_{k-1}; CGF advances x every second
  // iteration, applying alpha2 p_{k-2} (read from the array p_k is about to overwrite, at the own
  // points only) and then alpha p_{k-1}, one rounding each, so x is bitwise that of one update per
  // iteration while it is read and written half as often
  const int npend = CG ? a.scal->pending : 0;
  const bool xupd = CG && a.io0 != nullptr && !a.first && (FUSED ? npend == 2 : npend != 0);
  const bool xload = xupd && !(CG && a.scal->xzero);  // x known to be zero: not read
  const Tc alpha2 = FUSED ? (Tc)a.scal->alpha2 : (Tc)0;
  const Tc tauc = (Tc)a.t.tau;

  // prefetch registers: primary input vector (u / u_prev / p_old / x), secondary (q / r), x (CG1)
  // two prefetch slots: plane k is staged from slot (k - kbeg) & 1 while plane k+1 is in flight
  // prefetch distance (planes); 1 keeps the registers of the residual (and CG1) low
  constexpr int PF = RES ? 1 : (CG ? STENCIL_CG_PF : 2);
  Raw pa[PF][NV];
  RawC pb[PF][NV];
  RawC px[PF][NVC];
  RawC pq[FUSED ? PF : 1][FUSED ? NV : 1];  // CGF: q_old
  Raw pp2[FUSED ? PF : 1][FUSED ? NVC : 1];  // CGF: p_{k-2} at the own points (x update)
  int pk[PF] = {};  // plane index held in each prefetch slot
  double part0 = 0.0, part1 = 0.0, part2 = 0.0, part3 = 0.0;

  auto fetch = [&](int k, const int sl) {
    bool pvalid = true;
    int kk = k;
    if (BC == BC_PERIODIC) {
      kk %= nz; if (kk < 0) kk += nz;
    } else {
      pvalid = (k >= 0 && k < nz);
    }
    const bool inchunk = (k >= z0 && k < z0 + zc_eff);
    const int64_t base = (int64_t)kk * plane;
    pk[sl] = k;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int e = 0; e < VE; ++e) {
        pa[sl][v].x[e] = (Tin)0;
        pb[sl][v].x[e] = (Tc)0;
        if (v < NVC) px[sl][v < NVC ? v : 0].x[e] = (Tc)0;
        if (FUSED) pq[FUSED ? sl : 0][FUSED ? v : 0].x[e] = (Tc)0;
        if (FUSED && v < NVC) pp2[FUSED ? sl : 0][FUSED && v < NVC ? v : 0].x[e] = (Tin)0;
      }
      if (pvalid && ((valid >> v) & 1u)) {
        const int64_t gi = base + off[v];
        if (MODE == M_APPLY || RES) {
          pa[sl][v] = *(const Raw*)((const Tin*)a.in0 + gi);
        } else if (MODE == M_RHS) {
          pa[sl][v] = *(const Raw*)((const Tin*)a.in0 + gi);
          if (a.in1) pb[sl][v] = *(const RawC*)((const Tc*)a.in1 + gi);
        } else {  // CG1, CGF: in0 = r (Tc), in1 = p_old (Tin), in2 = q_old (Tc, CGF), io0 = x (Tc)
          pb[sl][v] = *(const RawC*)((const Tc*)a.in0 + gi);
          if (!a.first) pa[sl][v] = *(const Raw*)((const Tin*)a.in1 + gi);
          if (FUSED && !a.first) pq[FUSED ? sl : 0][FUSED ? v : 0] = *(const RawC*)((const Tc*)a.in2 + gi);
          if (v < NVC && xupd && inchunk && ((own >> v) & 1u)) {
            if (xload) px[sl][v < NVC ? v : 0] = *(const RawC*)((const Tc*)a.io0 + gi);
            if (FUSED) pp2[FUSED ? sl : 0][FUSED && v < NVC ? v : 0] = *(const Raw*)((const Tin*)a.out1 + gi);
          }
        }
      }
    }
  };

  // Transform the prefetched plane into LDS (and do the own-point side effects of CG1).
  auto stage_plane = [&](const int sl) {
    const int k = pk[sl];
    int kk = k;
    if (BC == BC_PERIODIC) { kk %= nz; if (kk < 0) kk += nz; }
    const bool inchunk = (k >= z0 && k < z0 + zc_eff);
    const int64_t base = (int64_t)kk * plane;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (soff[v] >= 0) {
        Tc* dst = stage + soff[v];
        if (MODE == M_APPLY || RES) {
#pragma unroll
          for (int e = 0; e < VE; ++e) dst[e] = to_c<Tin, Tc>(pa[sl][v].x[e]);
        } else if (MODE == M_RHS) {
#pragma unroll
          for (int e = 0; e < VE; ++e) dst[e] = fmad(tauc, pb[sl][v].x[e], to_c<Tin, Tc>(pa[sl][v].x[e]));
        } else {
          Raw pn;
          RawC xn, rn;
          const bool ow = v < NVC && inchunk && ((own >> v) & 1u) && ((valid >> v) & 1u);
#pragma unroll
          for (int e = 0; e < VE; ++e) {
            const Tc pold = to_c<Tin, Tc>(pa[sl][v].x[e]);
            Tc rv = pb[sl][v].x[e];
            // CGF: r_k = r_{k-1} - alpha_{k-1} q_{k-1} at every staged point (halo included)
            if (FUSED && !a.first) rv = fmad(-alpha_prev, pq[FUSED ? sl : 0][FUSED ? v : 0].x[e], rv);
            const Tc val = storage_round<Tin, Tc>(fmad(beta, pold, rv));
            dst[e] = val;
            pn.x[e] = from_c<Tin, Tc>(val);
            rn.x[e] = rv;
            if (v < NVC) {
              Tc xv = px[sl][v < NVC ? v : 0].x[e];
              if (FUSED) xv = fmad(alpha2, to_c<Tin, Tc>(pp2[FUSED ? sl : 0][FUSED && v < NVC ? v : 0].x[e]), xv);
              xn.x[e] = fmad(alpha_prev, pold, xv);
            }
          }
          if (FUSED && v < NVC) {
            const int rs = ((k % RQD) + RQD) % RQD;
#pragma unroll
            for (int e = 0; e < VE; ++e) rring[rs * TY * TX + coff[v < NVC ? v : 0] + e] = rn.x[e];
          }
          if (ow) {
            const int64_t gi = base + off[v];
            *(Raw*)((Tin*)a.out1 + gi) = pn;
            if (xupd) *(RawC*)((Tc*)a.io0 + gi) = xn;
            if (FUSED) {
              *(RawC*)((Tc*)a.out2 + gi) = rn;
#pragma unroll
              for (int e = 0; e < VE; ++e) part3 = fma((double)rn.x[e], (double)rn.x[e], part3);
            }
          }
        }
      }
    }
  };

  Tc acc[T][RPW];
  Tc accb[RR ? T : 1][RR ? RPW : 1];  // RHSRES: M u (= Mz P), the right-hand side
#pragma unroll
  for (int s = 0; s < T; ++s)
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      acc[s][i] = (Tc)0;
      if (RR) accb[RR ? s : 0][RR ? i : 0] = (Tc)0;
    }
  // BC_ROBIN: z-corner contributions to the output planes j-th from an end, j < ZM, kept in LDS
  // (each thread only touches its own column and rows)
  constexpr int ZM = BC == BC_ROBIN ? 2 * (N / 2) + 1 : 1;
  if constexpr (BC == BC_ROBIN) {
#pragma unroll
    for (int j = 0; j < ZM; ++j)
#pragma unroll
      for (int i = 0; i < RPW; ++i) zl[(j * TY + wave * RPW + i) * TX + col] = (Tc)0;
  }

  const int gxo = x0 + col;
  const bool colown = gxo < nx;

  const int kbeg = z0 - N, kend = z0 + zc_eff + N;
  fetch(kbeg, 0);
  if (PF == 2 && kbeg + 1 < kend) fetch(kbeg + 1, PF - 1);
  // unrolled over 2T planes: ring slot (ph + d) mod T and prefetch slot ph & 1 are static
  for (int kb = kbeg; kb < kend; kb += 2 * T) {
#pragma clang loop unroll(full)
    for (int ph = 0; ph < 2 * T; ++ph) {
      const int k = kb + ph;
      if (k < kend) {  // uniform: keeps the trip count constant so the ring indices are static
      const bool active = (BC == BC_PERIODIC) || (k >= 0 && k < nz);
      if (active) stage_plane(ph % PF);
      __syncthreads();
      if (k + PF < kend) fetch(k + PF, ph % PF);
      // RESID: b at the points of the output plane this iteration completes, loaded now so the
      // loads are in flight during the filter passes instead of at the output
      double bpre[MODE == M_RESID ? RPW : 1];
      if constexpr (MODE == M_RESID) {
        const int o = k - N;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int gy = y0 + wave * RPW + i;
          bpre[i] = (o >= z0 && colown && gy < ny) ? a.bvec[(int64_t)o * plane + (int64_t)gy * nx + gxo] : 0.0;
        }
      }
      if (active) {
        if constexpr (CG) {
          const int qs = ((k % QD) + QD) % QD;
#pragma unroll
          for (int i = 0; i < RPW; ++i)
            cring[(qs * TY + wave * RPW + i) * TX + col] = stage[(wave * RPW + i + N) * C + col + HX];
        }
        // x-pass over all R staged rows (rows dealt to the waves round-robin)
#pragma unroll 2
        for (int r = wave; r < R; r += WY) {
          const Tc* row = stage + r * C + HX + col;
          const Tc c0 = row[0];
          Tc U = m[0] * c0;
          Tc Vv = mx[0] * c0;
#pragma unroll
          for (int j = 1; j <= N; ++j) {
            const Tc sm = row[-j] + row[j];
            U = fmad(m[j], sm, U);
            Vv = fmad(mx[j], sm, Vv);
          }
          if constexpr (BC == BC_ROBIN) {
            // corner blocks of Mx and Mx + Wx: output column gx in the first / last z columns
            constexpr int zr = 2 * (N / 2) + 1;
            const int gx = x0 + col;
            if (gx < zr) {
#pragma unroll
              for (int cc = 0; cc < zr; ++cc) {
                const Tc v = row[cc - gx];
                U = fmad(rbt[gx * kRobinMaxZ + cc], v, U);
                Vv = fmad(rbt[RBT + gx * kRobinMaxZ + cc], v, Vv);
              }
            } else if (gx >= nx - zr && gx < nx) {
              const int rr = nx - 1 - gx;
#pragma unroll
              for (int cc = 0; cc < zr; ++cc) {
                const Tc v = row[rr - cc];
                U = fmad(rbt[rr * kRobinMaxZ + cc], v, U);
                Vv = fmad(rbt[RBT + rr * kRobinMaxZ + cc], v, Vv);
              }
            }
          }
          su[r * TX + col] = U;
          sv[r * TX + col] = Vv;
        }
      }
      __syncthreads();
      if (active) {
        Tc uc[RPW + 2 * N], vc[RPW + 2 * N];
#pragma unroll
        for (int j = 0; j < RPW + 2 * N; ++j) {
          uc[j] = su[(wave * RPW + j) * TX + col];
          if (MODE != M_RHS) vc[j] = sv[(wave * RPW + j) * TX + col];
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          Tc P = m[0] * uc[i + N];
          Tc Rr = (Tc)0;
          if (MODE != M_RHS) Rr = fmad(ays[0], uc[i + N], m[0] * vc[i + N]);
#pragma unroll
          for (int j = 1; j <= N; ++j) {
            const Tc pu = uc[i + N - j] + uc[i + N + j];
            P = fmad(m[j], pu, P);
            if (MODE != M_RHS) {
              const Tc pv = vc[i + N - j] + vc[i + N + j];
              Rr = fmad(m[j], pv, Rr);
              Rr = fmad(ays[j], pu, Rr);
            }
          }
          if constexpr (BC == BC_ROBIN) {
            // corner blocks of My (on U, V) and Wy (on U): output row gy in the first / last z rows
            // (wave-uniform); the x-pass results of the other rows are read back from LDS
            constexpr int zr = 2 * (N / 2) + 1;
            const int gy = y0 + wave * RPW + i;
            if (gy < zr || (gy >= ny - zr && gy < ny)) {
              const bool lo = gy < zr;
              const int rr = lo ? gy : ny - 1 - gy;
#pragma unroll
              for (int cc = 0; cc < zr; ++cc) {
                const int sr = (lo ? cc : ny - 1 - cc) - y0 + N;  // staged row of the input row
                const Tc Uc = su[sr * TX + col];
                const Tc cmv = rbt[rr * kRobinMaxZ + cc];
                P = fmad(cmv, Uc, P);
                if (MODE != M_RHS) {
                  Rr = fmad(cmv, sv[sr * TX + col], Rr);
                  Rr = fmad(rbt[2 * RBT + rr * kRobinMaxZ + cc], Uc, Rr);
                }
              }
            }
          }
          // plane k adds to outputs k+d, d = -N..N, held in ring slot (ph + d) mod T
#pragma unroll
          for (int d = -N; d <= N; ++d) {
            const int s = (ph + d + 3 * T) % T;
            const int ad = d < 0 ? -d : d;
            if (MODE == M_RHS) {
              acc[s][i] = fmad(m[ad], P, acc[s][i]);
            } else {
              acc[s][i] = fmad(m[ad], Rr, acc[s][i]);
              acc[s][i] = fmad(azs[ad], P, acc[s][i]);
              if (RR) accb[RR ? s : 0][RR ? i : 0] = fmad(m[ad], P, accb[RR ? s : 0][RR ? i : 0]);
            }
          }
          if constexpr (BC == BC_ROBIN) {
            // corner blocks of Mz (on R) and Wz (on P): an input plane k among the first / last z
            // planes adds to the output plane j-th from the same end (j < z) through zacc[j], which
            // the output step adds in and clears (the low end's are all cleared before the high
            // end's first input plane: nz >= 2z + n)
            if (k < ZM || k >= nz - ZM) {
              const int ri = k < ZM ? k : nz - 1 - k;
#pragma unroll
              for (int j = 0; j < ZM; ++j) {
                Tc* zp = zl + (j * TY + wave * RPW + i) * TX + col;
                Tc zv = fmad(rbt[j * kRobinMaxZ + ri], MODE == M_RHS ? P : Rr, *zp);
                if (MODE != M_RHS) zv = fmad(rbt[3 * RBT + j * kRobinMaxZ + ri], P, zv);
                *zp = zv;
              }
            }
          }
        }
      }
      // output plane o = k - N is complete
      {
        const int so = (ph - N + 3 * T) % T;
        const int o = k - N;
        Tc zadd[BC == BC_ROBIN ? RPW : 1];
        if constexpr (BC == BC_ROBIN) {
          const int zj = (o >= 0 && o < ZM) ? o : ((o >= nz - ZM && o < nz) ? nz - 1 - o : -1);
#pragma unroll
          for (int i = 0; i < RPW; ++i) {
            zadd[i] = (Tc)0;
            if (zj >= 0) {
              Tc* zp = zl + (zj * TY + wave * RPW + i) * TX + col;
              zadd[i] = *zp;
              *zp = (Tc)0;
            }
          }
        }
        if (o >= z0) {
          const int64_t obase = (int64_t)o * plane;
          const int qo = ((o % QD) + QD) % QD;
#pragma unroll
          for (int i = 0; i < RPW; ++i) {
            const int gy = y0 + wave * RPW + i;
            if (colown && gy < ny) {
              const int64_t gi = obase + (int64_t)gy * nx + gxo;
              Tc val = acc[so][i];
              if constexpr (BC == BC_ROBIN) val += zadd[i];
              if (MODE == M_APPLY || MODE == M_RHS) {
                if (a.nt_store) Io<Tout>::template st_nt<Tc>(a.out0, gi, val);
                else Io<Tout>::template st<Tc>(a.out0, gi, val);
              } else if (CG) {
                if (a.nt_store) Io<Tout>::template st_nt<Tc>(a.out0, gi, val);
                else Io<Tout>::template st<Tc>(a.out0, gi, val);
                const double qv = (double)val;
                part0 = fma((double)cring[(qo * TY + wave * RPW + i) * TX + col], qv, part0);
                if (FUSED) {
                  const int ro = ((o % RQD) + RQD) % RQD;
                  part1 = fma((double)rring[(ro * TY + wave * RPW + i) * TX + col], qv, part1);
                  part2 = fma(qv, qv, part2);
                }
              } else {
                // rscale (a power of two, 1 unless the refinement keeps r inside FP32 range) scales
                // the stored residual and both sums alike: their ratio is unchanged
                double b0;
                if constexpr (RR) {
                  b0 = (double)accb[RR ? so : 0][RR ? i : 0];
                  ((double*)a.out1)[gi] = b0;  // the step's right-hand side, as the rhs kernel forms it
                } else {
                  b0 = bpre[MODE == M_RESID ? i : 0];
                }
                const double b = b0 * a.rscale;
                const double r = b - (double)val * a.rscale;
                if (a.out0) Io<Tout>::template st<double>(a.out0, gi, r);
                part0 = fma(r, r, part0);
                part1 = fma(b, b, part1);
              }
            }
          }
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          acc[so][i] = (Tc)0;
          if (RR) accb[RR ? so : 0][RR ? i : 0] = (Tc)0;
        }
      }
      }
    }
  }

  if (CG || RES) {
    part0 = wave_sum(part0);
    part1 = wave_sum(part1);
    if (FUSED) {
      part2 = wave_sum(part2);
      part3 = wave_sum(part3);
    }
    if (lane == 0) { red[0][wv] = part0; red[1][wv] = part1; red[2][wv] = part2; red[3][wv] = part3; }
    __syncthreads();
    if (tid == 0) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int q = 0; q < WY * WX; ++q) { s0 += red[0][q]; s1 += red[1][q]; s2 += red[2][q]; s3 += red[3][q]; }
      a.part0[blockIdx.x] = s0;
      if (RES || FUSED) a.part1[blockIdx.x] = s1;
      if (FUSED) { a.part2[blockIdx.x] = s2; a.part3[blockIdx.x] = s3; }
    }
  }
}

// ------------------------------------------------------------------------------------------
// host-side launch helpers

// Tile shape per (degree, mode, compute type, boundary): heights and row waves from stencil.h (the
// host sizes the partial-sum buffers for the smallest height); the FP32 apply may take WX column
// groups (STENCIL_APPLY_WX, one by default).
template <int N, int MODE, typename Tc, int BC> constexpr int tile_y() {
  return stencil_tile_y(MODE, (int)sizeof(Tc), N, BC);
}
template <int N, int MODE, typename Tc, int BC> constexpr int tile_wy() {
  return stencil_tile_wy(MODE, (int)sizeof(Tc), N, BC);
}
template <int MODE, typename Tc> constexpr int tile_wx() {
  return (MODE == M_APPLY && sizeof(Tc) == 4) ? STENCIL_APPLY_WX : 1;
}

// One launch for boundary condition BC (one object per degree and boundary condition, so the
// instances compile in parallel; stencil.h dispatches on the run-time boundary condition).
template <int N, int MODE, typename Tin, typename Tc, typename Tout, int BC>
hipError_t launch_bcx(const StencilArgs& a0, bool vec, hipStream_t st) {
  constexpr int TY = tile_y<N, MODE, Tc, BC>();
  constexpr int WX = tile_wx<MODE, Tc>();
  constexpr int WY = tile_wy<N, MODE, Tc, BC>();
  static_assert(TY >= kTileY, "the partial-sum buffers hold one sum per tile of kTileY rows");
  StencilArgs a = a0;  // geometry for this tile shape
  a.tiles_x = (a.nx + 64 * WX - 1) / (64 * WX);
  a.tiles_y = (a.ny + TY - 1) / TY;
  a.nblocks = a.tiles_x * a.tiles_y * a.nchunks;
  dim3 grid(a.nblocks), block(64 * WX * WY);
  if (vec)
    hipLaunchKernelGGL((stencil_kernel<N, TY, MODE, Tin, Tc, Tout, BC, true, WX, WY>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((stencil_kernel<N, TY, MODE, Tin, Tc, Tout, BC, false, WX, WY>), grid, block, 0, st, a);
  return hipGetLastError();
}

// The fused rhs and residual for degree N and boundary BC (no Robin instance: the caller falls back
// to the rhs and residual kernels there).
template <int N, int BC>
hipError_t launch_rhsres_bc(const StencilArgs& a, bool vec, hipStream_t st) {
  if constexpr (BC == BC_ROBIN) {
    return hipErrorInvalidValue;
  } else {
    return launch_bcx<N, M_RHSRES, double, double, float, BC>(a, vec, st);
  }
}

}  // namespace tbs

// Every (mode, dtype) combination the dispatch in stencil.hip uses, for degree N and boundary BC.
#define TBS_STENCIL_INSTANTIATE(N, BC)                                                                        \
  namespace tbs {                                                                                             \
  template hipError_t launch_bcx<N, M_APPLY, double, double, double, BC>(const StencilArgs&, bool, hipStream_t);   \
  template hipError_t launch_bcx<N, M_APPLY, float, float, float, BC>(const StencilArgs&, bool, hipStream_t);      \
  template hipError_t launch_bcx<N, M_APPLY, uint16_t, float, float, BC>(const StencilArgs&, bool, hipStream_t);   \
  template hipError_t launch_bcx<N, M_APPLY, float, double, double, BC>(const StencilArgs&, bool, hipStream_t);    \
  template hipError_t launch_bcx<N, M_APPLY, uint16_t, double, double, BC>(const StencilArgs&, bool, hipStream_t); \
  template hipError_t launch_bcx<N, M_RHS, double, double, double, BC>(const StencilArgs&, bool, hipStream_t);     \
  template hipError_t launch_bcx<N, M_RHS, float, float, float, BC>(const StencilArgs&, bool, hipStream_t);        \
  template hipError_t launch_bcx<N, M_CG1, double, double, double, BC>(const StencilArgs&, bool, hipStream_t);     \
  template hipError_t launch_bcx<N, M_CG1, float, float, float, BC>(const StencilArgs&, bool, hipStream_t);        \
  template hipError_t launch_bcx<N, M_CG1, uint16_t, float, float, BC>(const StencilArgs&, bool, hipStream_t);     \
  template hipError_t launch_bcx<N, M_CGF, double, double, double, BC>(const StencilArgs&, bool, hipStream_t);     \
  template hipError_t launch_bcx<N, M_CGF, float, float, float, BC>(const StencilArgs&, bool, hipStream_t);        \
  template hipError_t launch_bcx<N, M_CGF, uint16_t, float, float, BC>(const StencilArgs&, bool, hipStream_t);     \
  template hipError_t launch_bcx<N, M_RESID, double, double, double, BC>(const StencilArgs&, bool, hipStream_t);   \
  template hipError_t launch_bcx<N, M_RESID, double, double, float, BC>(const StencilArgs&, bool, hipStream_t);    \
  template hipError_t launch_rhsres_bc<N, BC>(const StencilArgs&, bool, hipStream_t);                               \
  }
