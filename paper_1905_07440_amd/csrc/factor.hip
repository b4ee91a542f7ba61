// FP64 dense factorizations for the stabilised recomputation of G.
//
// The paper defines G through M = I + B_L ... B_1 and refers to the standard
// DQMC literature for computing it without overflow: the running product is
// kept as U D T, re-factored with a pivoted QR after every block of n_stab
// slices, and G comes from one more solve at the end.  Two factorizations
// serve that scheme, one workgroup (4 waves) per matrix, in panels of NB = 16
// columns:
//
//  QR           Householder QR with the columns pre-sorted by decreasing norm
//               (pre-pivoting keeps the graded scales of Z = (C U) D in order
//               without per-step pivot searches).  Each panel is factored by
//               all four waves (factor_panel: one column per step through
//               LDS, one butterfly per column for the norm and the dots); the
//               block reflector I - V T V^T (compact WY, T by recursive
//               doubling from the Gram matrix V^T V) is applied to the
//               trailing columns with MFMA.  Q is accumulated backwards the
//               same way, in a launch of its own that gives every 16-column
//               tile of Q its own wave (qr_formq_kernel).
//               Outputs Q, D = |diag R| and Rt = D^-1 R P^T (over Z), so
//               Z = Q diag(D) Rt.
//  Gauss-Jordan in-place inversion with partial (row) pivoting, blocked the
//               same way: the four waves eliminate a panel (eliminate_panel:
//               pivot over all unused rows), then every other column gets the
//               rank-NB update
//                   A[r][C] = [r not a pivot row of the panel] A[r][C] + F[r][:] A_old[P][C]
//               (F: the eliminated panel, P: its pivot rows).  Output
//               diag(rs) M^-1 diag(cs) (over M) and log|det M|.
//
// Up to N = 144 the matrix lives in the accumulators of the four waves
// (qr_regs_kernel, gj_regs_kernel); beyond, in global memory, where it stays
// in L2 (qr_blocked_kernel, inv_blocked_kernel).
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

constexpr int NB = 16;           // panel width
constexpr int MAXN = 256;        // largest N (lattices up to 16 x 16)
constexpr int VLD = MAXN + 16;   // panel row length in LDS (zero tail)
// kernels are instantiated for N <= MX with MX in {64, 112, 144, 256}: panel
// rows per lane and 16-row tiles per strip are sized for MX
template <int MX> struct Cap { enum { rpl = (MX + 63) / 64, tiles = (MX + 15) / 16 }; };

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// data-parallel-primitive moves of a double (both 32-bit halves); lanes whose
// source is outside the enabled rows read 0
template <int CTRL, int ROWMASK = 0xF>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
// sum over the 64 lanes, returned uniform: within rows of 16 by quad
// permutations and mirrors, then across rows by the row broadcasts
__device__ inline double wave_total(double v) {
  v += dpp_move<0xB1>(v);          // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);          // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);         // row_half_mirror
  v += dpp_move<0x140>(v);         // row_mirror
  v += dpp_move<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
  return lane_value(v, 63);
}

// 1 / x by the hardware estimate and two Newton steps (x finite, nonzero,
// not subnormal): within an ulp or so of the correctly rounded quotient
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// maximum over the 64 lanes of an unsigned key, returned uniform (the same
// exchange pattern as wave_total)
template <int CTRL, int ROWMASK = 0xF>
__device__ inline uint32_t dpp_move_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, false);
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  v = max(v, dpp_move_u32<0xB1>(v));
  v = max(v, dpp_move_u32<0x4E>(v));
  v = max(v, dpp_move_u32<0x141>(v));
  v = max(v, dpp_move_u32<0x140>(v));
  v = max(v, dpp_move_u32<0x142, 0xA>(v));
  v = max(v, dpp_move_u32<0x143, 0xC>(v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Totals over the 64 lanes of several values at once, returned
// wave-uniform: a butterfly in which every exchange halves the values a lane
// carries, none through LDS.  Lane halves (bit 5) and row pairs (bit 4) trade
// through the permlane swaps: after swapping the upper lanes of x with the
// lower lanes of y, x + y is, on every lane, the kept value plus the
// partner's matching one.  Bit 3 pairs lanes by a row rotation of 8 and the
// last halving by the half-row mirror (lane ^ 7), whose partners agree on
// every bit already reduced.
__device__ inline double swap_sum32(double lo_half, double hi_half) {
  // x: values the lower lanes keep; y: values the upper lanes keep
  const auto l = __builtin_amdgcn_permlane32_swap(__double2loint(lo_half), __double2loint(hi_half), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(__double2hiint(lo_half), __double2hiint(hi_half), false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
__device__ inline double swap_sum16(double lo_half, double hi_half) {
  const auto l = __builtin_amdgcn_permlane16_swap(__double2loint(lo_half), __double2loint(hi_half), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(__double2hiint(lo_half), __double2hiint(hi_half), false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
// 8 values: after the butterfly lane l holds the total of value (l >> 3) & 7,
// and t[c] reads value c from lane 8 c
__device__ inline void wave_totals8(const double (&v)[8], double (&t)[8]) {
  const int lane = threadIdx.x & 63;
  double a4[4], a2[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) a4[i] = swap_sum32(v[i], v[4 + i]);
#pragma unroll
  for (int i = 0; i < 2; ++i) a2[i] = swap_sum16(a4[i], a4[2 + i]);
  const bool h = (lane & 8) != 0;
  double a1 = (h ? a2[1] : a2[0]) + dpp_move<0x128>(h ? a2[0] : a2[1]);   // row_ror:8, lane ^ 8
  a1 += dpp_move<0x141>(a1);                          // row_half_mirror, lane ^ 7
  a1 += dpp_move<0xB1>(a1);                           // quad_perm [1,0,3,2]
  a1 += dpp_move<0x4E>(a1);                           // quad_perm [2,3,0,1]
#pragma unroll
  for (int c = 0; c < 8; ++c) t[c] = lane_value(a1, 8 * c);
}

// ---------------------------------------------------------------------------
// Householder factorisation of one panel of 16 columns (rows relative to the
// panel's diagonal block, m of them) by all four waves: wave w holds panel
// columns w, w + 4, w + 8, w + 12, one row per lane and slot.  Column j goes
// to every wave through LDS (Colj, alternating per column); each wave reduces
// the column's norm below the diagonal together with its dots against its
// own columns in one butterfly, forms the same reflector, and updates its own
// columns.  load(c, r) gives the panel; store(c, r, v) receives R on and
// above the diagonal and the reflectors below it, for every c < 16 and every
// row slot r; tau[j] the reflectors' scales.
// ---------------------------------------------------------------------------
template <int RPL, int CAP, typename Load, typename Store>
__device__ inline void factor_panel(int nbw, int m, double (*Colj)[CAP], double* tau, Load load, Store store) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double a[4][RPL];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + 64 * t, c = wave + 4 * q;
      a[q][t] = (c < nbw && r < m) ? load(c, r) : 0.0;
    }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nbw) {
      const int jq = j >> 2;
      if (wave == (j & 3)) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = lane + 64 * t;
          if (r < CAP) Colj[j & 1][r] = a[jq][t];
        }
      }
      __syncthreads();
      // slot 0: the squared norm of column j below the diagonal; slot 1 + q:
      // the dot of that tail with own column w + 4q (if right of j).  The
      // reflector's scale enters afterwards, since
      // v^T a_c = a_c[j] + scl * (tail . a_c[tail])
      // the column as loaded (row j too: its diagonal entry then comes from
      // lane j's register instead of a second LDS round trip), and its tail
      double raw[RPL], tail[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        raw[t] = (r < CAP) ? Colj[j & 1][r] : 0.0;
        tail[t] = (r > j && r < m) ? raw[t] : 0.0;
      }
      double part[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) part[c] = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) part[0] += tail[t] * tail[t];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (wave + 4 * q > j) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) part[1 + q] += tail[t] * a[q][t];
        }
      double tot[8];
      wave_totals8(part, tot);
      const double sg = tot[0];
      const double al = lane_value(raw[0], j);   // row j < 16 lives in slot 0 of lane j
      double be = al, tj = 0.0, scl = 0.0;
      if (sg > 0.0) {
        const double nrm = sqrt(al * al + sg);
        be = (al >= 0.0) ? -nrm : nrm;
        tj = (be - al) * rcp_nr(be);
        scl = rcp_nr(al - be);             // |al - be| = |al| + nrm > 0
      }
      double vr[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        vr[t] = (r == j) ? 1.0 : tail[t] * scl;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (wave + 4 * q > j) {
          const double w = tj * (lane_value(a[q][0], j) + scl * tot[1 + q]);   // row j lives in lane j
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[q][t] -= vr[t] * w;
        }
      if (wave == (j & 3)) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = lane + 64 * t;
          if (r >= j) a[jq][t] = (r == j) ? be : vr[t];
        }
      }
      if (tid == 0) tau[j] = tj;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < RPL; ++t) store(wave + 4 * q, lane + 64 * t, a[q][t]);
}

// ---------------------------------------------------------------------------
// Gauss-Jordan elimination of one panel of 16 columns (all n rows) by all four
// waves: wave w holds panel columns w, w + 4, w + 8, w + 12, one row per lane
// and slot.  Column j goes to every wave through LDS; every wave finds the
// same pivot (the unused row of largest |a| by a DPP maximum over 32-bit keys:
// |a| rounded to FP32 with its low 9 bits replaced by 511 - row, so
// near-equal magnitudes go to the lower row) and updates its own columns:
// rows other than the pivot row lose a multiple of it, the pivot row is
// divided by the pivot, and column j becomes -a / pivot with 1 / pivot on the
// pivot row.  used[] marks this lane's pivoted rows (the same in every wave).
// load(c, r) gives the panel (called for c < nbw, r < n only); store(c, r, v)
// receives it eliminated, for every c < 16 and row slot r;
// perm[p0 + j], pinv[row] and pivot[p0 + j] record the pivots.
// ---------------------------------------------------------------------------
template <int RPL, int CAP, typename Load, typename Store>
__device__ inline void eliminate_panel(int p0, int nbw, int n, double (*Colj)[CAP], bool (&used)[RPL], int* perm,
                                       int* pinv, double* pivot, Load load, Store store) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double a[4][RPL];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + 64 * t, c = wave + 4 * q;
      a[q][t] = (r < n && c < nbw) ? load(c, r) : 0.0;
    }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nbw) {
      const int jq = j >> 2;
      if (wave == (j & 3)) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = lane + 64 * t;
          if (r < CAP) Colj[j & 1][r] = a[jq][t];
        }
      }
      __syncthreads();
      double aj[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        aj[t] = (r < CAP) ? Colj[j & 1][r] : 0.0;
      }
      uint32_t key = 0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        const uint32_t kt = (__float_as_uint((float)fabs(aj[t])) & ~0x1FFu) | (uint32_t)(511 - r);
        if (r < n && !used[t]) key = max(key, kt);
      }
      key = wave_max_u32(key);
      const int pr = 511 - (int)(key & 0x1FFu), pl = pr & 63, pt = pr >> 6;
      double pmine = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) pmine = (t == pt) ? aj[t] : pmine;
      const double pj = lane_value(pmine, pl);
      const double ip = rcp_nr(pj);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (wave + 4 * q == j) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[q][t] = (lane + 64 * t == pr) ? ip : -aj[t] * ip;
        } else {
          // the pivot row's entry of this column, broadcast from its lane
          double mine = 0.0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) mine = (t == pt) ? a[q][t] : mine;
          const double wp = lane_value(mine, pl) * ip;
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[q][t] = (lane + 64 * t == pr) ? wp : fma(-aj[t], wp, a[q][t]);
        }
      }
#pragma unroll
      for (int t = 0; t < RPL; ++t)
        if (lane + 64 * t == pr) used[t] = true;
      if (tid == 0) {
        perm[p0 + j] = pr;
        pinv[pr] = p0 + j;
        pivot[p0 + j] = pj;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < RPL; ++t) store(wave + 4 * q, lane + 64 * t, a[q][t]);
}

// ---------------------------------------------------------------------------
// A <- A - V op(T) (V^T A) on rows [p0, n) and columns [c_begin, n),
// op(T) = T^T (transT) or T.  V: Vs[k][r] (r relative to p0, zero outside the
// panel's rows), T: Ts.  Each wave takes 16-column strips and holds a strip in
// registers as 16-row MFMA tiles: in the f64 16x16x4 layout the B operands of
// four consecutive 4-row chunks are exactly the C/D tile of those 16 rows.
// ---------------------------------------------------------------------------
template <int MX>
__device__ void apply_reflector(double* A, int n, int p0, int m, const double (*Vs)[VLD],
                                const double (*Ts)[NB + 1], int transT, int c_begin, double (*Sc)[NB + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nstrip = (n - c_begin + 15) / 16;
  const int ntile = (m + 15) / 16;
  for (int s = wave; s < nstrip; s += 4) {
    const int col = c_begin + 16 * s + li;
    d4 tile[Cap<MX>::tiles];
#pragma unroll
    for (int t = 0; t < Cap<MX>::tiles; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = p0 + 16 * t + frag_row<double>(lane, v);
        tile[t][v] = (t < ntile && row < n && col < n) ? A[(long)row * n + col] : 0.0;
      }
    }
    d4 w1 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < Cap<MX>::tiles; ++t)
      if (t < ntile) {
#pragma unroll
        for (int q = 0; q < 4; ++q) w1 = mfma16(Vs[li][16 * t + 4 * q + lk], tile[t][q], w1);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) Sc[frag_row<double>(lane, v)][li] = w1[v];
    wave_sync_lds();
    d4 w2 = {0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < NB; k0 += 4) {
      const double at = transT ? Ts[k0 + lk][li] : Ts[li][k0 + lk];
      w2 = mfma16(at, Sc[k0 + lk][li], w2);
    }
    wave_sync_lds();
#pragma unroll
    for (int v = 0; v < 4; ++v) Sc[frag_row<double>(lane, v)][li] = w2[v];
    wave_sync_lds();
    double wb[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) wb[q] = Sc[4 * q + lk][li];
#pragma unroll
    for (int t = 0; t < Cap<MX>::tiles; ++t)
      if (t < ntile) {
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) tile[t] = mfma16(-Vs[4 * q + lk][16 * t + li], wb[q], tile[t]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = p0 + 16 * t + frag_row<double>(lane, v);
          if (row < n && col < n) A[(long)row * n + col] = tile[t][v];
        }
      }
    wave_sync_lds();
  }
}

// The same update with buffer loads and stores: one resource for rows p0..n
// of A, so a tile element's address is a per-lane byte offset (four of them,
// one per fragment row, plus the tile's start) instead of a 64-bit pointer
// per element.  Rows past n fall outside the resource (loads give 0, stores
// are dropped); columns past n take an offset past it on purpose.

template <int MX>
__device__ __attribute__((always_inline)) void apply_reflector_buf(double* A, int n, int p0, int m, const double (*Vs)[VLD],
                                    const double (*Ts)[NB + 1], int transT, int c_begin, double (*Sc)[NB + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nstrip = (n - c_begin + 15) / 16;
  const int ntile = (m + 15) / 16;
  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc(A + (long)p0 * n, 0, (int)((long)m * n * 8), BUF_WORD3);
  const unsigned tstep = 16u * (unsigned)n * 8u;   // bytes per 16 rows
  constexpr int NTL = Cap<MX>::tiles;
  auto offsets = [&](int s, unsigned (&off)[4]) {
    const int col = c_begin + 16 * s + li;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      off[v] = (col < n) ? ((unsigned)(frag_row<double>(lane, v) * n + col) * 8u) : BUF_OUTSIDE;
  };
  auto load = [&](int s, d4 (&tile)[NTL]) {
    unsigned off[4];
    offsets(s, off);
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) tile[t][v] = (t < ntile) ? buf_load_f64(rsrc, off[v] + t * tstep) : 0.0;
  };
  auto update = [&](int s, d4 (&tile)[NTL]) {
    d4 w1 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < NTL; ++t)
      if (t < ntile) {
#pragma unroll
        for (int q = 0; q < 4; ++q) w1 = mfma16(Vs[li][16 * t + 4 * q + lk], tile[t][q], w1);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) Sc[frag_row<double>(lane, v)][li] = w1[v];
    wave_sync_lds();
    d4 w2 = {0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < NB; k0 += 4) {
      const double at = transT ? Ts[k0 + lk][li] : Ts[li][k0 + lk];
      w2 = mfma16(at, Sc[k0 + lk][li], w2);
    }
    wave_sync_lds();
#pragma unroll
    for (int v = 0; v < 4; ++v) Sc[frag_row<double>(lane, v)][li] = w2[v];
    wave_sync_lds();
    double wb[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) wb[q] = Sc[4 * q + lk][li];
    unsigned off[4];
    offsets(s, off);
#pragma unroll
    for (int t = 0; t < NTL; ++t)
      if (t < ntile) {
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) tile[t] = mfma16(-Vs[4 * q + lk][16 * t + li], wb[q], tile[t]);
#pragma unroll
        for (int v = 0; v < 4; ++v) buf_store_f64(tile[t][v], rsrc, off[v] + t * tstep);
      }
    wave_sync_lds();
  };
  // strips s = wave, wave + 4, ...; one register set, so that the caller
  // fits two workgroups per CU, whose strips' loads then run under each
  // other's products (at N = 256, 1024 matrices: 2.94 ms for the QR against
  // 3.68 ms with two register sets and one workgroup per CU)
  d4 ta[NTL];
  for (int s = wave; s < nstrip; s += 4) {
    load(s, ta);
    update(s, ta);
  }
}

// T (upper triangular; H_0 ... H_{nb-1} = I - V T V^T) from the Gram matrix
// V^T V, which comes from MFMA (both operands are the same V fragment, the
// four waves taking every fourth 4-row chunk).  T is built by recursive
// doubling, one element per thread (see below).
template <int LD>
__device__ void form_t(const double (*Vs)[LD], int m, int nbw, const double* tau, double (*Gm)[NB + 1],
                       double (*Ts)[NB + 1], double (*Sc)[NB][NB + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  d4 g = {0, 0, 0, 0};
  for (int r0 = 4 * wave; r0 < m; r0 += 16) {
    const double x = Vs[li][r0 + lk];      // rows past m are zero in Vs
    g = mfma16(x, x, g);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Sc[wave][frag_row<double>(lane, v)][li] = g[v];
  __syncthreads();
  // T by recursive doubling (one element per thread): with T_1, T_2 the
  // factors of two adjacent groups of b reflectors, the factor of the pair is
  // [[T_1, -T_1 (V_1^T V_2) T_2], [0, T_2]]; start from T_jj = tau_j
  const int a = tid >> 4, b = tid & 15;
  Gm[a][b] = (Sc[0][a][b] + Sc[1][a][b]) + (Sc[2][a][b] + Sc[3][a][b]);
  Ts[a][b] = (a == b && a < nbw) ? tau[a] : 0.0;
  __syncthreads();
  double (*X)[NB + 1] = Sc[0];             // V_1^T V_2 T_2, reusing the Gram partials' space
#pragma unroll
  for (int w = 1; w < NB; w *= 2) {
    const int o = a & ~(2 * w - 1);        // first row of this pair of groups
    const bool upper = (a - o) < w && (b & ~(2 * w - 1)) == o && (b - o) >= w;
    if (upper) {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < w; ++k) x += Gm[a][o + w + k] * Ts[o + w + k][b];
      X[a][b] = x;
    }
    __syncthreads();
    if (upper) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < w; ++k) t += Ts[a][o + k] * X[o + k][b];
      Ts[a][b] = -t;
    }
    __syncthreads();
  }
}

template <int MX>
__global__ __launch_bounds__(256, 2) void qr_blocked_kernel(double* __restrict__ Zg, double* __restrict__ Wg,
                                                            double* __restrict__ Qg, double* __restrict__ Dg,
                                                            double* __restrict__ Tg, int n) {
  __shared__ double Vs[NB][VLD];
  __shared__ double Ts[NB][NB + 1];
  __shared__ double Gm[NB][NB + 1];
  __shared__ double Sc[4][NB][NB + 1];
  __shared__ double norms[MAXN];
  __shared__ double tau[NB];
  __shared__ double Colj[2][MAXN];         // panel column j, alternating per column
  __shared__ int perm[MAXN];
  const int z = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6;
  double* Z = Zg + (long)z * n * n;
  double* W = Wg + (long)z * n * n;
  double* Q = Qg + (long)z * n * n;
  double* Tst = Tg + (long)z * NB * (n + NB);
  const int npan = (n + NB - 1) / NB;

  // pre-pivoting: columns of Z in order of decreasing norm (NaN last)
  if (tid < n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // 32 rows in flight per round trip; s[u] sums rows u, u + 8, u + 16, ... in order
    for (int r0 = 0; r0 < n; r0 += 32) {
      double v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = (r0 + u < n) ? Z[(long)(r0 + u) * n + tid] : 0.0;
#pragma unroll
      for (int u = 0; u < 32; ++u) s[u & 7] += v[u] * v[u];
    }
    const double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    norms[tid] = (t == t) ? t : -1.0;
  }
  __syncthreads();
  if (tid < n) {
    const double s = norms[tid];
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += (norms[k] > s || (norms[k] == s && k < tid)) ? 1 : 0;
    perm[rank] = tid;
  }
  __syncthreads();
  batched_copy<256, 16, double>(n * n, [&](int e) { const int r = e / n; return Z[(long)r * n + perm[e - r * n]]; },
                                [&](int e, double v) { W[e] = v; });
  __syncthreads();

  for (int pi = 0; pi < npan; ++pi) {
    const int p0 = pi * NB, nbw = min(NB, n - p0), m = n - p0;
    factor_panel<Cap<MX>::rpl>(
        nbw, m, Colj, tau, [&](int c, int r) { return W[(long)(p0 + r) * n + p0 + c]; },
        [&](int c, int r, double v) {
          // V to LDS (unit diagonal, zero above and below the panel rows); R and V back to W
          if (r < VLD) Vs[c][r] = (c < nbw && r < m) ? ((r == c) ? 1.0 : ((r > c) ? v : 0.0)) : 0.0;
          if (c < nbw && r < m) W[(long)(p0 + r) * n + p0 + c] = v;
        });
    Vs[tid >> 4][MAXN + (tid & 15)] = 0.0;
    __syncthreads();
    form_t(Vs, m, nbw, tau, Gm, Ts, Sc);
    Tst[(long)pi * NB * NB + tid] = Ts[tid >> 4][tid & 15];
    apply_reflector_buf<MX>(W, n, p0, m, Vs, Ts, 1, p0 + nbw, Sc[wave]);
    __syncthreads();
  }

  // D = |diag R|, Rt = D^-1 R P^T written over Z
  for (int r = tid; r < n; r += 256) norms[r] = fabs(W[(long)r * n + r]);
  __syncthreads();
  for (int r = tid; r < n; r += 256) Dg[(long)z * n + r] = norms[r];
  batched_copy<256, 16, double>(n * n, [&](int e) { return W[e]; },
                                [&](int e, double v) {
                                  const int r = e / n, c = e - r * n;
                                  Z[(long)r * n + perm[c]] = (r <= c) ? v / norms[r] : 0.0;
                                });
}

// ---------------------------------------------------------------------------
// The same QR with the matrix resident in registers (N <= 144): the four
// waves hold it as 16 x 16 MFMA tiles, wave w owning tile columns w, w + 4,
// w + 8.  A panel passes through LDS once to be factored by the four waves;
// the block reflector is applied to the tiles in place, so the trailing
// update touches no memory but the 16-column reflector.  V and T of every
// panel go to W and T in global memory, from which qr_formq_kernel forms Q
// (Q is not an input of the factorization's later panels, so its
// accumulation need not wait on the four waves of this workgroup).
// ---------------------------------------------------------------------------
template <int MX>
__global__ __launch_bounds__(256) void qr_regs_kernel(double* __restrict__ Zg, double* __restrict__ Wg,
                                                      double* __restrict__ Qg, double* __restrict__ Dg,
                                                      double* __restrict__ Tg, int n) {
  constexpr int NTT = (MX + 15) / 16;      // tile rows
  constexpr int CPW = (NTT + 3) / 4;       // tile columns per wave
  // panel rows and column j in LDS cover every row slot of factor_panel (64
  // per lane register).  Compact rows where the registers leave room for
  // three workgroups per CU (N <= 64: 35 KB of LDS instead of 90 KB); the
  // larger sizes run one workgroup per CU and keep the full row length, with
  // which the register allocation spills least
  constexpr int CJ = 64 * Cap<MX>::rpl;
  constexpr int LD = (MX <= 64) ? MX + 16 : VLD;   // panel row length (zero tail)
  __shared__ double Vs[NB][LD];
  __shared__ double Pn[NB][LD];            // the panel being factored, column-major
  __shared__ double Ts[NB][NB + 1];
  __shared__ double Gm[NB][NB + 1];
  __shared__ double Sc[4][NB][NB + 1];
  __shared__ double norms[MX];
  __shared__ double tau[NB];
  __shared__ double Colj[2][CJ];           // panel column j, alternating per column
  __shared__ int perm[MX];
  const int z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  double* Z = Zg + (long)z * n * n;
  double* W = Wg + (long)z * n * n;
  double* Q = Qg + (long)z * n * n;
  double* Tst = Tg + (long)z * NB * (n + NB);
  const int nt = (n + 15) / 16;
  const int npan = nt;

  // pre-pivoting: columns of Z in order of decreasing norm (NaN last)
  if (tid < n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // 16 rows in flight per round trip (32 make the N = 144 kernel spill more);
    // s[u] sums rows u, u + 8, u + 16, ... in order
    for (int r0 = 0; r0 < n; r0 += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = (r0 + u < n) ? Z[(long)(r0 + u) * n + tid] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) s[u & 7] += v[u] * v[u];
    }
    const double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    norms[tid] = (t == t) ? t : -1.0;
  }
  __syncthreads();
  if (tid < n) {
    const double s = norms[tid];
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += (norms[k] > s || (norms[k] == s && k < tid)) ? 1 : 0;
    perm[rank] = tid;
  }
  __syncthreads();

  d4 A[CPW][NTT];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    const int col = 16 * (wave + 4 * u) + li;
    const int pc = (col < n) ? perm[col] : 0;
#pragma unroll
    for (int t = 0; t < NTT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + frag_row<double>(lane, v);
        A[u][t][v] = (row < n && col < n) ? Z[(long)row * n + pc] : 0.0;
      }
  }

  // A <- (I - V op(T) V^T) A on rows >= p0 of tile column u (tiles t >= p)
  auto apply = [&](int u, int p, int transT) {
    double (*S)[NB + 1] = Sc[wave];
    d4 w1 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < NTT; ++t)
      if (t >= p && t < nt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) w1 = mfma16(Vs[li][16 * (t - p) + 4 * q + lk], A[u][t][q], w1);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) S[frag_row<double>(lane, v)][li] = w1[v];
    wave_sync_lds();
    d4 w2 = {0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < NB; k0 += 4) {
      const double at = transT ? Ts[k0 + lk][li] : Ts[li][k0 + lk];
      w2 = mfma16(at, S[k0 + lk][li], w2);
    }
    wave_sync_lds();
#pragma unroll
    for (int v = 0; v < 4; ++v) S[frag_row<double>(lane, v)][li] = w2[v];
    wave_sync_lds();
    double wb[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) wb[q] = S[4 * q + lk][li];
#pragma unroll
    for (int t = 0; t < NTT; ++t)
      if (t >= p && t < nt) {
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) A[u][t] = mfma16(-Vs[4 * q + lk][16 * (t - p) + li], wb[q], A[u][t]);
      }
    wave_sync_lds();
  };

  for (int p = 0; p < npan; ++p) {
    const int p0 = p * NB, nbw = min(NB, n - p0), m = n - p0;
    const int owner = p & 3, up = p >> 2;
    // the panel's tiles to LDS (rows relative to p0)
    if (wave == owner) {
#pragma unroll
      for (int u = 0; u < CPW; ++u)
        if (u == up) {
#pragma unroll
          for (int t = 0; t < NTT; ++t)
            if (t >= p && t < nt) {
#pragma unroll
              for (int v = 0; v < 4; ++v) Pn[li][16 * (t - p) + frag_row<double>(lane, v)] = A[u][t][v];
            }
        }
    }
    __syncthreads();
    // the panel is factored by all four waves
    factor_panel<Cap<MX>::rpl>(
        nbw, m, Colj, tau, [&](int c, int r) { return Pn[c][r]; },
        [&](int c, int r, double v) {
          // V (unit diagonal, zero above, zero past the panel) to Vs; R and V to Pn and to W
          if (r < LD) {
            Vs[c][r] = (c < nbw && r < m) ? ((r == c) ? 1.0 : ((r > c) ? v : 0.0)) : 0.0;
            Pn[c][r] = (c < nbw && r < m) ? v : 0.0;
          }
          if (c < nbw && r < m) W[(long)(p0 + r) * n + p0 + c] = v;
        });
    Vs[tid >> 4][MX + (tid & 15)] = 0.0;
    __syncthreads();
    form_t(Vs, m, nbw, tau, Gm, Ts, Sc);
    Tst[(long)p * NB * NB + tid] = Ts[tid >> 4][tid & 15];
    // the factored panel back into its tiles, then the trailing tile columns
    if (wave == owner) {
#pragma unroll
      for (int u = 0; u < CPW; ++u)
        if (u == up) {
#pragma unroll
          for (int t = 0; t < NTT; ++t)
            if (t >= p && t < nt) {
#pragma unroll
              for (int v = 0; v < 4; ++v) A[u][t][v] = Pn[li][16 * (t - p) + frag_row<double>(lane, v)];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < CPW; ++u) {
      const int cj = wave + 4 * u;
      if (cj > p && cj < nt) apply(u, p, 1);
    }
    __syncthreads();
  }

  // D = |diag R|; Rt = D^-1 R P^T written over Z
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    const int cj = wave + 4 * u;
#pragma unroll
    for (int t = 0; t < NTT; ++t)
      if (t == cj && cj < nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + frag_row<double>(lane, v), col = 16 * cj + li;
          if (row == col && row < n) norms[row] = fabs(A[u][t][v]);
        }
      }
  }
  __syncthreads();
  for (int r = tid; r < n; r += 256) Dg[(long)z * n + r] = norms[r];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    const int col = 16 * (wave + 4 * u) + li;
    if (col < n) {
      const int pc = perm[col];
#pragma unroll
      for (int t = 0; t < NTT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + frag_row<double>(lane, v);
          if (row < n) Z[(long)row * n + pc] = (row <= col) ? A[u][t][v] / norms[row] : 0.0;
        }
    }
  }

}

// ---------------------------------------------------------------------------
// Q = H_0 H_1 ... H_{np-1} of a QR left by qr_regs_kernel or
// qr_blocked_kernel (V of every panel below the diagonal of W, its T in T):
// one wave per 16-column tile of Q and matrix, four tiles (4g .. 4g + 3) per
// workgroup.  Tile cj starts as the identity's and takes the block
// reflectors I - V_p T_p V_p^T of panels p = cj, cj - 1, ..., 0 (those right
// of its columns leave it unchanged), backwards from the identity.  The
// tiles are independent, so they spread over the SIMDs instead of queueing
// on the four waves of the factorization's workgroup, and the four waves of
// a workgroup share each panel's V in LDS (up to 32 KB at N = 256).  Two
// workgroups per CU (register cap) hide each other's panel loads: 939 us for
// 256 QRs of 256 x 256 against 1008 us at one per CU with the next panel
// prefetched to registers; at 12 x 12, 128 matrices, the QR takes 246 us
// against 285 us with Q accumulated in the factorization's workgroup and 257
// us with one single-wave workgroup per tile.  A wave whose tile lies left
// of the panel only takes part in the staging.  The operations on a tile,
// and their order, are those of that former in-place accumulation, so Q is
// the same to the bit.
// ---------------------------------------------------------------------------
template <int MX>
__global__ __launch_bounds__(256, 2) void qr_formq_kernel(const double* __restrict__ Wg, const double* __restrict__ Tg,
                                                        double* __restrict__ Qg, int n) {
  constexpr int NTT = (MX + 15) / 16;
  constexpr int LD = 16 * NTT + 1;         // V row length (odd: column reads spread over the banks)
  constexpr int RL = NTT;                  // V values per thread and panel: 16 x 16 NTT / 256
  __shared__ double Vs[NB][LD];
  __shared__ double Ts[NB][NB + 1];
  __shared__ double Sc[4][NB][NB + 1];
  const int z = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (n + 15) / 16;
  const int cj = 4 * blockIdx.x + wave;    // this wave's tile column (none when >= nt)
  const int pmax = min(4 * (int)blockIdx.x + 3, nt - 1);
  const double* W = Wg + (long)z * n * n;
  const double* Tst = Tg + (long)z * NB * (n + NB);
  double* Q = Qg + (long)z * n * n;
  double (*S)[NB + 1] = Sc[wave];

  // thread's share of panel p: column tid % 16, rows tid / 16 + 16 i of the
  // panel (below the diagonal only; the unit diagonal is set when staged)
  const int sc = tid & 15, sr = tid >> 4;
  double vn[RL], tn;
  auto fetch = [&](int p) {
    const int p0 = 16 * p, nbw = min(NB, n - p0), m = n - p0;
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      const int r = sr + 16 * i;
      vn[i] = (sc < nbw && r < m && r > sc) ? W[(long)(p0 + r) * n + p0 + sc] : 0.0;
    }
    tn = Tst[(long)p * NB * NB + tid];
  };

  d4 A[NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + frag_row<double>(lane, v), col = 16 * cj + li;
      A[t][v] = (row == col && row < n) ? 1.0 : 0.0;
    }
  for (int p = pmax; p >= 0; --p) {
    const int p0 = 16 * p, nbw = min(NB, n - p0), m = n - p0;
    fetch(p);
    __syncthreads();                       // the previous panel's V and T are no longer read
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      const int r = sr + 16 * i;
      Vs[sc][r] = (r == sc && sc < nbw && r < m) ? 1.0 : vn[i];
    }
    Ts[tid >> 4][tid & 15] = tn;
    __syncthreads();
    if (cj >= p && cj < nt) {
      // A <- (I - V T V^T) A on the tiles t >= p
      d4 w1 = {0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < NTT; ++t)
        if (t >= p && t < nt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) w1 = mfma16(Vs[li][16 * (t - p) + 4 * q + lk], A[t][q], w1);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) S[frag_row<double>(lane, v)][li] = w1[v];
      wave_sync_lds();
      d4 w2 = {0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < NB; k0 += 4) w2 = mfma16(Ts[li][k0 + lk], S[k0 + lk][li], w2);
      wave_sync_lds();
#pragma unroll
      for (int v = 0; v < 4; ++v) S[frag_row<double>(lane, v)][li] = w2[v];
      wave_sync_lds();
      double wb[NB / 4];
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) wb[q] = S[4 * q + lk][li];
#pragma unroll
      for (int t = 0; t < NTT; ++t)
        if (t >= p && t < nt) {
#pragma unroll
          for (int q = 0; q < NB / 4; ++q) A[t] = mfma16(-Vs[4 * q + lk][16 * (t - p) + li], wb[q], A[t]);
        }
    }
  }
  if (cj < nt) {
    const int col = 16 * cj + li;
#pragma unroll
    for (int t = 0; t < NTT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + frag_row<double>(lane, v);
        if (row < n && col < n) Q[(long)row * n + col] = A[t][v];
      }
  }
}

// ---------------------------------------------------------------------------
// blocked Gauss-Jordan inversion in place
// ---------------------------------------------------------------------------
template <int MX>
__global__ __launch_bounds__(256) void inv_blocked_kernel(double* __restrict__ Mg, double* __restrict__ Wg,
                                                          const double* __restrict__ rsg,
                                                          const double* __restrict__ csg,
                                                          const double* __restrict__ base,
                                                          double* __restrict__ logdet, int n) {
  __shared__ double Fs[NB][VLD];          // eliminated panel, column-major, zero tail
  __shared__ double Sc[4][NB][NB + 1];
  __shared__ int perm[MAXN];              // perm[j]: pivot row of column j
  __shared__ int pinv[MAXN];
  __shared__ int panel_of[MAXN];          // panel in which a row became a pivot row
  __shared__ double pivot[MAXN];           // pivot value of column j
  __shared__ double Colj[2][MAXN];         // panel column j, alternating per column
  __shared__ double part[4];
  const int z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double* M = Mg + (long)z * n * n;
  double* W = Wg + (long)z * n * n;
  batched_copy<256, 16, double>(n * n, [&](int e) { return M[e]; }, [&](int e, double v) { W[e] = v; });
  panel_of[tid] = -1;
  __syncthreads();
  const int npan = (n + NB - 1) / NB;
  bool used[Cap<MX>::rpl];                         // rows of this lane already pivoted (same in every wave)
#pragma unroll
  for (int t = 0; t < Cap<MX>::rpl; ++t) used[t] = false;

  for (int pi = 0; pi < npan; ++pi) {
    const int p0 = pi * NB, nbw = min(NB, n - p0);
    eliminate_panel<Cap<MX>::rpl>(
        p0, nbw, n, Colj, used, perm, pinv, pivot, [&](int c, int r) { return W[(long)r * n + p0 + c]; },
        [&](int c, int r, double v) {
          if (r < VLD - NB) Fs[c][r] = (c < nbw && r < n) ? v : 0.0;
          if (c < nbw && r < n) W[(long)r * n + p0 + c] = v;
        });
    __syncthreads();
    for (int j = tid; j < nbw; j += 256) panel_of[perm[p0 + j]] = pi;
    Fs[tid >> 4][MAXN + (tid & 15)] = 0.0;
    __syncthreads();
    // rank-NB update of every column outside the panel, all rows (tiles through
    // buffer loads and stores, as in the QR's reflector updates)
    const int nstrip = (n + 15) / 16;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(W, 0, (int)((long)n * n * 8), BUF_WORD3);
    const unsigned tstep = 16u * (unsigned)n * 8u;
    const int ntile = (n + 15) / 16;
    constexpr int NTL = Cap<MX>::tiles;
    auto outside = [&](int c) { return c >= n || (c >= p0 && c < p0 + nbw); };   // columns this panel leaves alone
    // strip s: its tiles (rows of this panel's pivots as 0) and its old pivot rows
    auto load = [&](int s, d4 (&tile)[NTL], double (&pv)[4]) {
      const int col = 16 * s + li;
      unsigned off[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) off[v] = outside(col) ? BUF_OUTSIDE : ((unsigned)(frag_row<double>(lane, v) * n + col) * 8u);
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + frag_row<double>(lane, v);   // rows past n: outside the resource
          tile[t][v] = (t < ntile && panel_of[row] != pi) ? buf_load_f64(rsrc, off[v] + t * tstep) : 0.0;
        }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = lane + 64 * i, k = e >> 4, cg = 16 * s + (e & 15);
        pv[i] = (k < nbw && !outside(cg)) ? W[(long)perm[p0 + k] * n + cg] : 0.0;
      }
    };
    auto update = [&](int s, d4 (&tile)[NTL], const double (&pv)[4]) {
      const int col = 16 * s + li;
      unsigned off[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) off[v] = outside(col) ? BUF_OUTSIDE : ((unsigned)(frag_row<double>(lane, v) * n + col) * 8u);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = lane + 64 * i;
        Sc[wave][e >> 4][e & 15] = pv[i];
      }
      wave_sync_lds();
      double tb[NB / 4];
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) tb[q] = Sc[wave][4 * q + lk][li];
#pragma unroll
      for (int t = 0; t < NTL; ++t)
        if (t < ntile) {
#pragma unroll
          for (int q = 0; q < NB / 4; ++q) tile[t] = mfma16(Fs[4 * q + lk][16 * t + li], tb[q], tile[t]);
#pragma unroll
          for (int v = 0; v < 4; ++v) buf_store_f64(tile[t][v], rsrc, off[v] + t * tstep);
        }
      wave_sync_lds();
    };
    // strips s = wave, wave + 4, ...; the next strip loads while the current one is updated
    d4 ta[NTL], tb2[NTL];
    double pa[4], pb[4];
    if (wave < nstrip) load(wave, ta, pa);
    for (int s = wave; s < nstrip; s += 8) {
      if (s + 4 < nstrip) load(s + 4, tb2, pb);
      update(s, ta, pa);
      if (s + 4 >= nstrip) break;
      if (s + 8 < nstrip) load(s + 8, ta, pa);
      update(s + 4, tb2, pb);
    }
    __syncthreads();
  }

  // M^-1[j][perm[k]] = W[perm[j]][k]; written scaled over M
  const double* rs = rsg + (long)z * n;
  const double* cs = csg + (long)z * n;
  batched_copy<256, 16, double>(n * n, [&](int e) { return W[e]; },
                                [&](int e, double v) {
                                  const int r = e / n, k = e - r * n;
                                  const int j = pinv[r], pk = perm[k];
                                  M[(long)j * n + pk] = rs[j] * v * cs[pk];
                                });
  // log|det M| = sum of log|pivot|
  double lg = 0.0;
  for (int i = tid; i < n; i += 256) lg += log(fabs(pivot[i]));
  lg = wave_total(lg);
  if (lane == 0) part[wave] = lg;
  __syncthreads();
  if (tid == 0) logdet[z] = base[z] + ((part[0] + part[1]) + (part[2] + part[3]));
}

// ---------------------------------------------------------------------------
// Gauss-Jordan inversion with the matrix held in registers (N <= MX <= 144):
// the same elimination as inv_blocked_kernel, panel by panel, but every
// column tile lives in the accumulators of the wave that owns it (tile column
// c belongs to wave c % 4), so the trailing rank-16 update of a panel never
// leaves the CU.  Per panel: the owner hands the panel to the four waves
// through LDS, they eliminate its 16 columns, and each wave fetches the
// panel's pivot rows of its own columns through a per-wave LDS copy of the
// tile column.
// ---------------------------------------------------------------------------
template <int MX>
__global__ __launch_bounds__(256) void gj_regs_kernel(double* __restrict__ Mg, double* __restrict__ Wg,
                                                      const double* __restrict__ rsg,
                                                      const double* __restrict__ csg,
                                                      const double* __restrict__ base,
                                                      double* __restrict__ logdet, int n) {
  constexpr int NTT = (MX + 15) / 16;      // tile rows (and tile columns)
  constexpr int CPW = (NTT + 3) / 4;       // tile columns per wave
  constexpr int RPL = Cap<MX>::rpl;
  static_assert(4 * NTT <= 64, "pivot-row flags hold 64 rows per lane");
  __shared__ double Pn[NB][MX];            // the panel, column-major; after elimination its F
  __shared__ double Cs[4][NTT * 16][NB + 1];   // per-wave copy of one tile column
  __shared__ int perm[MX];                 // perm[j]: pivot row of column j
  __shared__ int pinv[MX];
  __shared__ double pivot[MX];             // pivot value of column j
  __shared__ double Colj[2][64 * RPL];     // panel column j, alternating per column
  __shared__ double rsl[MX], csl[MX];
  __shared__ double part[4];
  const int z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  double* M = Mg + (long)z * n * n;
  double* W = Wg + (long)z * n * n;
  const int nt = (n + 15) / 16;
  for (int i = tid; i < n; i += 256) {
    rsl[i] = rsg[(long)z * n + i];
    csl[i] = csg[(long)z * n + i];
  }

  d4 A[CPW][NTT];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    const int col = 16 * (wave + 4 * u) + li;
#pragma unroll
    for (int t = 0; t < NTT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + frag_row<double>(lane, v);
        A[u][t][v] = (row < n && col < n) ? M[(long)row * n + col] : 0.0;
      }
  }
  bool used[RPL];                          // rows of this lane already pivoted (same in every wave)
#pragma unroll
  for (int t = 0; t < RPL; ++t) used[t] = false;

  for (int p = 0; p < nt; ++p) {
    const int p0 = p * NB, nbw = min(NB, n - p0);
    const int owner = p & 3, up = p >> 2;
    if (wave == owner) {
#pragma unroll
      for (int u = 0; u < CPW; ++u)
        if (u == up) {
#pragma unroll
          for (int t = 0; t < NTT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) Pn[li][16 * t + frag_row<double>(lane, v)] = A[u][t][v];
        }
    }
    __syncthreads();
    // the panel is eliminated by all four waves
    eliminate_panel<RPL>(
        p0, nbw, n, Colj, used, perm, pinv, pivot, [&](int c, int r) { return Pn[c][r]; },
        [&](int c, int r, double v) {
          if (r < 16 * NTT) Pn[c][r] = (c < nbw) ? v : 0.0;
        });
    __syncthreads();
    // rows of this lane (bit 4t + v for row 16t + frag_row(lane, v)) that became pivots in this panel
    uint64_t pm = 0;
    for (int k = 0; k < nbw; ++k) {
      const int r = perm[p0 + k];
      if ((r & 3) == lk) pm |= 1ull << (4 * (r >> 4) + ((r & 15) >> 2));
    }
    if (wave == owner) {
#pragma unroll
      for (int u = 0; u < CPW; ++u)
        if (u == up) {
#pragma unroll
          for (int t = 0; t < NTT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) A[u][t][v] = Pn[li][16 * t + frag_row<double>(lane, v)];
        }
    }
    // every other column: rows outside the panel's pivots keep their value,
    // then all rows gain F * (old pivot rows)
#pragma unroll
    for (int u = 0; u < CPW; ++u) {
      const int cj = wave + 4 * u;
      if (cj != p && cj < nt) {
#pragma unroll
        for (int t = 0; t < NTT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) Cs[wave][16 * t + frag_row<double>(lane, v)][li] = A[u][t][v];
        wave_sync_lds();
        double b[NB / 4];
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) b[q] = (4 * q + lk < nbw) ? Cs[wave][perm[p0 + 4 * q + lk]][li] : 0.0;
#pragma unroll
        for (int t = 0; t < NTT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if ((pm >> (4 * t + v)) & 1) A[u][t][v] = 0.0;
#pragma unroll
        for (int t = 0; t < NTT; ++t)
          if (t < nt) {
#pragma unroll
            for (int q = 0; q < NB / 4; ++q) A[u][t] = mfma16(Pn[4 * q + lk][16 * t + li], b[q], A[u][t]);
          }
        wave_sync_lds();                    // Cs is rewritten by the next tile column
      }
    }
    __syncthreads();                        // Pn is rewritten by the next panel
  }

  // M^-1[j][perm[k]] = W[perm[j]][k]: each element straight from its
  // register to its permuted place, scaled, over M
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    const int col = 16 * (wave + 4 * u) + li;
    if (col < n) {
      const int pk = perm[col];
      const double cv = csl[pk];
#pragma unroll
      for (int t = 0; t < NTT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + frag_row<double>(lane, v);
          if (row < n) {
            const int j = pinv[row];
            M[(long)j * n + pk] = rsl[j] * A[u][t][v] * cv;
          }
        }
    }
  }
  // log|det M| = sum of log|pivot|
  double lg = 0.0;
  for (int i = tid; i < n; i += 256) lg += log(fabs(pivot[i]));
  lg = wave_total(lg);
  if (lane == 0) part[wave] = lg;
  __syncthreads();
  if (tid == 0) logdet[z] = base[z] + ((part[0] + part[1]) + (part[2] + part[3]));
  (void)W;
}

// ===========================================================================
// Wide forms for a few large matrices (N > 144 with a batch small enough that
// one workgroup per matrix would leave most CUs idle): S workgroups per
// matrix and one launch per panel.  Every wave holds the whole 16-column
// panel in its registers and factors (or eliminates) it alone, so a column
// step needs no barrier and no LDS round trip; the S x 4 waves of a matrix
// then share the panel's independent work items, strips of 16 columns.
// All waves reach the same reflectors and pivots (same data, same
// instruction order), so no workgroup waits for another inside a launch:
// the launch boundary orders the panels.  Workgroup w of matrix z is block
// w * batch + z, which keeps a matrix's workgroups on one XCD (one L2) when
// the batch is a multiple of 8.
// ===========================================================================

// totals over the 64 lanes of NV values (NV = 16, 8, 4, 2, 1), returned
// wave-uniform.  The halving butterfly leaves value k in lane (64 / NV) k.
template <int NV>
__device__ inline void wave_totals_n(const double (&v)[NV], double (&t)[NV]) {
  const int lane = threadIdx.x & 63;
  if constexpr (NV == 16) {
    double a8[8], a4[4], a2[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) a8[i] = swap_sum32(v[i], v[8 + i]);     // lane bit 5 picks the upper half
#pragma unroll
    for (int i = 0; i < 4; ++i) a4[i] = swap_sum16(a8[i], a8[4 + i]);   // bit 4
    const bool h3 = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) a2[i] = (h3 ? a4[2 + i] : a4[i]) + dpp_move<0x128>(h3 ? a4[i] : a4[2 + i]);
    const bool h2 = (lane & 4) != 0;
    double a1 = (h2 ? a2[1] : a2[0]) + dpp_move<0x141>(h2 ? a2[0] : a2[1]);   // lane ^ 7 flips bit 2
    a1 += dpp_move<0xB1>(a1);
    a1 += dpp_move<0x4E>(a1);
#pragma unroll
    for (int c = 0; c < 16; ++c) t[c] = lane_value(a1, 4 * c);
  } else if constexpr (NV == 8) {
    wave_totals8(v, t);
  } else if constexpr (NV == 4) {
    double a2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a2[i] = swap_sum32(v[i], v[2 + i]);
    double a1 = swap_sum16(a2[0], a2[1]);
    a1 += dpp_move<0xB1>(a1);
    a1 += dpp_move<0x4E>(a1);
    a1 += dpp_move<0x141>(a1);
    a1 += dpp_move<0x140>(a1);
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] = lane_value(a1, 16 * c);
  } else if constexpr (NV == 2) {
    double a1 = swap_sum32(v[0], v[1]);
    a1 = swap_sum16(a1, a1);                                             // rows 2i and 2i + 1
    a1 += dpp_move<0xB1>(a1);
    a1 += dpp_move<0x4E>(a1);
    a1 += dpp_move<0x141>(a1);
    a1 += dpp_move<0x140>(a1);
    t[0] = lane_value(a1, 0);
    t[1] = lane_value(a1, 32);
  } else {
    t[0] = wave_total(v[0]);
  }
}

// Column j of a panel held whole by the calling wave (a[c][t]: column c, row
// lane + 64 t, rows relative to the panel's diagonal block, m of them).  One
// butterfly gives the squared norm of the column's tail below the diagonal
// (slot 0) and the tail's dots with the columns right of j (slot k: column
// j + k); the reflector H = I - tau v v^T with v = e_j + tail / (al - be)
// maps the column to be e_j and is applied to those columns.  NV >= 16 - j.
template <int NV, int RPL>
__device__ inline void qr_column(int j, int m, double (&a)[NB][RPL], double* tau) {
  const int lane = threadIdx.x & 63;
  double tail[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + 64 * t;
    tail[t] = (r > j && r < m) ? a[j][t] : 0.0;
  }
  double part[NV];
  part[0] = 0.0;
#pragma unroll
  for (int t = 0; t < RPL; ++t) part[0] += tail[t] * tail[t];
#pragma unroll
  for (int k = 1; k < NV; ++k) {
    part[k] = 0.0;
    if (j + k < NB) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) part[k] += tail[t] * a[j + k][t];
    }
  }
  double tot[NV];
  wave_totals_n<NV>(part, tot);
  const double sg = tot[0];
  const double al = lane_value(a[j][0], j);          // row j < 16 lives in slot 0 of lane j
  double be = al, tj = 0.0, scl = 0.0;
  if (sg > 0.0) {
    const double nrm = sqrt(al * al + sg);
    be = (al >= 0.0) ? -nrm : nrm;
    tj = (be - al) * rcp_nr(be);
    scl = rcp_nr(al - be);                           // |al - be| = |al| + nrm > 0
  }
  double vr[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) vr[t] = (lane + 64 * t == j) ? 1.0 : tail[t] * scl;
#pragma unroll
  for (int k = 1; k < NV; ++k)
    if (j + k < NB) {
      const double w = tj * (lane_value(a[j + k][0], j) + scl * tot[k]);   // v^T a_c = a_c[j] + scl (tail . a_c)
#pragma unroll
      for (int t = 0; t < RPL; ++t) a[j + k][t] -= vr[t] * w;
    }
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + 64 * t;
    if (r >= j) a[j][t] = (r == j) ? be : vr[t];
  }
  if (threadIdx.x == 0) tau[j] = tj;
}

// the nbw columns of a panel, in order; on return a holds R on and above the
// diagonal and the reflectors' tails below it, tau (LDS, written by thread 0)
// their scales, zero past nbw
template <int RPL>
__device__ inline void qr_panel_wave(int nbw, int m, double (&a)[NB][RPL], double* tau) {
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nbw) {
      if (j < 8) qr_column<16>(j, m, a, tau);
      else if (j < 12) qr_column<8>(j, m, a, tau);
      else if (j < 14) qr_column<4>(j, m, a, tau);
      else if (j < 15) qr_column<2>(j, m, a, tau);
      else qr_column<1>(j, m, a, tau);
    } else if (threadIdx.x == 0) {
      tau[j] = 0.0;
    }
  }
}

// Gauss-Jordan elimination of a panel held whole by the calling wave (all n
// rows; a[c][t]: column c, row lane + 64 t).  Column j: the pivot is the
// unused row of largest |a| (the FP32 key of eliminate_panel: near-equal
// magnitudes go to the lower row); its row across the panel is read from its
// lane; rows other than the pivot row lose a multiple of it, the pivot row is
// divided by the pivot, and column j becomes -a / pivot with 1 / pivot on the
// pivot row.  prow[j] and pval[j] (LDS, written by thread 0) record the pivots.
template <int RPL>
__device__ inline void gj_panel_wave(int nbw, int n, double (&a)[NB][RPL], bool (&used)[RPL], int* prow,
                                     double* pval) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nbw) {
      uint32_t key = 0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        const uint32_t kt = (__float_as_uint((float)fabs(a[j][t])) & ~0x1FFu) | (uint32_t)(511 - r);
        if (r < n && !used[t]) key = max(key, kt);
      }
      key = wave_max_u32(key);
      const int pr = 511 - (int)(key & 0x1FFu), pl = pr & 63, pt = pr >> 6;
      double pv[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) pv[c] = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t)
        if (pt == t) {                                  // uniform: the pivot row's register slot
#pragma unroll
          for (int c = 0; c < NB; ++c) pv[c] = lane_value(a[c][t], pl);
        }
      const double pj = pv[j];
      const double ip = rcp_nr(pj);
      double aj[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) aj[t] = a[j][t];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c == j) continue;
        const double wp = pv[c] * ip;
#pragma unroll
        for (int t = 0; t < RPL; ++t) a[c][t] = fma(-aj[t], wp, a[c][t]);
      }
#pragma unroll
      for (int t = 0; t < RPL; ++t) a[j][t] = -aj[t] * ip;
      const bool me = lane == pl;
#pragma unroll
      for (int t = 0; t < RPL; ++t)
        if (pt == t) {
#pragma unroll
          for (int c = 0; c < NB; ++c) a[c][t] = me ? ((c == j) ? ip : pv[c] * ip) : a[c][t];
          used[t] = used[t] || me;
        }
      if (threadIdx.x == 0) {
        prow[j] = pr;
        pval[j] = pj;
      }
    }
  }
}

// One strip of 16 columns as 16-row MFMA tiles (rows from the panel's top,
// m of them): lane l, element v of tile t holds row 16 t + frag_row(l, v),
// column l % 16.  ld(rr, c) gives row rr and strip column c; it returns 0
// outside the matrix by a buffer load whose offset, not whose value, is
// masked, so that nothing sinks the loads into branches: they issue back to
// back, and a caller can issue them before work that does not need them.
template <int MX, typename Load>
__device__ inline void strip_load(int m, d4 (&tile)[Cap<MX>::tiles], Load ld) {
  const int lane = threadIdx.x & 63, li = lane & 15;
  const int ntile = (m + 15) / 16;
#pragma unroll
  for (int t = 0; t < Cap<MX>::tiles; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) tile[t][v] = (t < ntile) ? ld(16 * t + frag_row<double>(lane, v), li) : 0.0;
}

// One wave applies I - V op(T) V^T (op(T) = T^T: the transposed block
// reflector, Q^T from the left) to a strip loaded by strip_load: w1 = V^T X,
// w2 = op(T) w1, X -= V w2; store(rr, c, v) receives the result (and drops
// elements outside the matrix).
template <int MX, typename Store>
__device__ inline void strip_apply(int m, d4 (&tile)[Cap<MX>::tiles], const double (*Vs)[VLD],
                                   const double (*Ts)[NB + 1], double (*S)[NB + 1], Store store) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  constexpr int NTL = Cap<MX>::tiles;
  const int ntile = (m + 15) / 16;
  d4 w1 = {0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < NTL; ++t)
    if (t < ntile) {
#pragma unroll
      for (int q = 0; q < 4; ++q) w1 = mfma16(Vs[li][16 * t + 4 * q + lk], tile[t][q], w1);
    }
#pragma unroll
  for (int v = 0; v < 4; ++v) S[frag_row<double>(lane, v)][li] = w1[v];
  wave_sync_lds();
  d4 w2 = {0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4) w2 = mfma16(Ts[k0 + lk][li], S[k0 + lk][li], w2);
  wave_sync_lds();
#pragma unroll
  for (int v = 0; v < 4; ++v) S[frag_row<double>(lane, v)][li] = w2[v];
  wave_sync_lds();
  double wb[NB / 4];
#pragma unroll
  for (int q = 0; q < NB / 4; ++q) wb[q] = S[4 * q + lk][li];
  wave_sync_lds();                                    // S is rewritten by the next strip
#pragma unroll
  for (int t = 0; t < NTL; ++t)
    if (t < ntile) {
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) tile[t] = mfma16(-Vs[4 * q + lk][16 * t + li], wb[q], tile[t]);
#pragma unroll
      for (int v = 0; v < 4; ++v) store(16 * t + frag_row<double>(lane, v), li, tile[t][v]);
    }
}

// wide-form scratch per matrix: Q^T and the factored panels (n x n each) and
// S partial column norms (QR); the second work matrix, pivot rows and pivot
// values (Gauss-Jordan) share the same space
constexpr int WIDE_MAX_SPLIT = 8;
__host__ __device__ inline long wide_stride(int n) { return 2L * n * n + (long)WIDE_MAX_SPLIT * n; }
size_t wide_scratch_doubles(int n) { return (size_t)wide_stride(n); }

// Workgroups per matrix of the wide forms: as many as leave every CU one (at
// most 8), for N > 144 only, and only from four on.  Up to 144 the
// register-resident forms are faster: at 12x12 with 128 chains the wide QR
// over two workgroups per matrix took 358 us per batch against 278 us (nine
// launches, each paying a memory round trip, against one).  At N = 256 two
// workgroups do not pay either: 128 QRs took 1.36 ms spread over two each,
// while 256 QRs took 1.13 ms at one workgroup each; four per matrix (64
// QRs) took 0.90 ms.
int wide_split(int n, int batch) {
  if (n <= 144 || batch < 1) return 1;
  const int s = std::min(WIDE_MAX_SPLIT, 256 / batch);
  return s >= 4 ? s : 1;
}
static int qr_wide_split(int n, int batch) { return wide_split(n, batch); }
static int gj_wide_split(int n, int batch) { return wide_split(n, batch); }

// partial squared column norms of Z over row block w of S
__global__ __launch_bounds__(256) void qr_wide_norms_kernel(const double* __restrict__ Zg, double* __restrict__ Xg,
                                                            int n, int batch, int S) {
  const int z = blockIdx.x % batch, w = blockIdx.x / batch;
  const int c = threadIdx.x;
  if (c >= n) return;
  const double* Z = Zg + (long)z * n * n;
  const int r0 = (int)((long)w * n / S), r1 = (int)((long)(w + 1) * n / S);
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = r0; r < r1; r += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (r + u < r1) ? Z[(long)(r + u) * n + c] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += v[u] * v[u];
  }
  Xg[(long)z * wide_stride(n) + 2L * n * n + (long)w * n + c] =
      ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// the pre-pivoting order from the partial norms (decreasing norm, NaN last,
// ties to the lower column), into perm (LDS), by every workgroup alike
__device__ inline void wide_perm(const double* part, int n, int S, double* norms, int* perm) {
  const int tid = threadIdx.x;
  if (tid < n) {
    double t = 0.0;
    for (int w = 0; w < S; ++w) t += part[(long)w * n + tid];
    norms[tid] = (t == t) ? t : -1.0;
  }
  __syncthreads();
  if (tid < n) {
    const double s = norms[tid];
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += (norms[k] > s || (norms[k] == s && k < tid)) ? 1 : 0;
    perm[rank] = tid;
  }
  __syncthreads();
}

// The tiles of work item it of panel p of the wide QR: the trailing strips
// right of the panel (it < ntr), then every strip of Q^T, rows from the
// panel's top; at p = 0 the trailing strips come from the input in
// pre-pivoted column order (perm) and Q^T starts as the identity.
template <int MX>
__device__ __attribute__((always_inline)) inline void qr_item_load(d4 (&tile)[Cap<MX>::tiles], int it, int ntr, int p,
                                                                   int m, int n, const double* Z, const double* W,
                                                                   const double* QT, const int* perm, unsigned bytes) {
  const int li = threadIdx.x & 15;
  const bool first = (p == 0), trailing = it < ntr;
  const int p0 = p * NB, c0 = trailing ? 16 * (p + 1 + it) : 16 * (it - ntr);
  const bool ident = first && !trailing;
  const __amdgpu_buffer_rsrc_t rs = uniform_rsrc((first && trailing) ? Z : (trailing ? W : QT), bytes);
  const int colsrc = (first && trailing) ? perm[min(c0 + li, n - 1)] : c0 + li;
  const bool live = (c0 + li < n) && !ident;
  strip_load<MX>(m, tile, [&](int rr, int c) -> double {
    const int r = p0 + rr, col = c0 + c;
    const unsigned off = (live && r < n) ? (unsigned)((r * n + colsrc) * 8) : BUF_OUTSIDE;
    return buf_load_f64(rs, off) + ((ident && r == col && r < n) ? 1.0 : 0.0);
  });
}

// Panel p of the wide QR.  Z (input, read through the column order at p = 0),
// W (R rows and trailing columns), X: Q^T, the factored panels Pf, partial
// norms.  Work items: the trailing strips right of the panel, then every
// strip of Q^T (rows from the panel's top), Q^T accumulated forwards as
// H_p^T ... H_0^T.
template <int MX>
__global__ __launch_bounds__(256) void qr_wide_step_kernel(const double* __restrict__ Zg, double* __restrict__ Wg,
                                                           double* __restrict__ Xg, int n, int batch, int S, int p) {
  constexpr int RPL = Cap<MX>::rpl;
  __shared__ double Vs[NB][VLD];
  __shared__ double Ts[NB][NB + 1];
  __shared__ double Gm[NB][NB + 1];
  __shared__ double Sc[4][NB][NB + 1];
  __shared__ double tau_s[NB];
  __shared__ double norms[MAXN];
  __shared__ int perm[MAXN];
  const int z = blockIdx.x % batch, w = blockIdx.x / batch;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const long nn = (long)n * n;
  const double* Z = Zg + z * nn;
  double* W = Wg + z * nn;
  double* QT = Xg + (long)z * wide_stride(n);
  double* Pf = QT + nn;
  const int p0 = p * NB, nbw = min(NB, n - p0), m = n - p0;
  const bool first = (p == 0);
  if (first) wide_perm(QT + 2 * nn, n, S, norms, perm);

  // the panel through buffer loads (masked elements read 0 from outside the
  // resource), then this wave's first work item, whose loads do not depend on
  // the panel and so run under its factorization
  const unsigned bytes = (unsigned)(nn * 8);
  double a[NB][RPL];
  {
    const __amdgpu_buffer_rsrc_t rp = uniform_rsrc(first ? (const double*)Z : W, bytes);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int col = first ? perm[min(c, n - 1)] : p0 + c;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        const unsigned off = (c < nbw && r < m) ? (unsigned)(((p0 + r) * n + col) * 8) : BUF_OUTSIDE;
        a[c][t] = buf_load_f64(rp, off);
      }
    }
  }
  // work items (qr_item_load)
  const int nst = (n + 15) / 16, ntr = nst - p - 1;
  const int nitems = ntr + nst, units = 4 * S;
  const int it0 = w * 4 + wave;
  d4 tile[Cap<MX>::tiles];
  if (it0 < nitems) qr_item_load<MX>(tile, it0, ntr, p, m, n, Z, W, QT, perm, bytes);

  qr_panel_wave<RPL>(nbw, m, a, tau_s);
  // V to LDS (unit diagonal, zero above and below the panel's rows), wave w
  // writing columns w, w + 4, ...; the factored panel to Pf from workgroup 0
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if ((c & 3) == wave) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        if (r < VLD) Vs[c][r] = (c < nbw && r < m) ? ((r == c) ? 1.0 : ((r > c) ? a[c][t] : 0.0)) : 0.0;
        if (w == 0 && c < nbw && r < m) Pf[(long)(p0 + r) * n + p0 + c] = a[c][t];
      }
    }
  if (64 * RPL < VLD) Vs[tid >> 4][64 * RPL + (tid & 15)] = 0.0;
  __syncthreads();
  form_t(Vs, m, nbw, tau_s, Gm, Ts, Sc);

  for (int it = it0; it < nitems; it += units) {
    if (it != it0) qr_item_load<MX>(tile, it, ntr, p, m, n, Z, W, QT, perm, bytes);
    const bool trailing = it < ntr;
    const int c0 = trailing ? 16 * (p + 1 + it) : 16 * (it - ntr);
    double* dst = trailing ? W : QT;
    strip_apply<MX>(m, tile, Vs, Ts, Sc[wave], [&](int rr, int c, double v) {
      const int r = p0 + rr, col = c0 + c;
      if (r < n && col < n) dst[(long)r * n + col] = v;
    });
  }
}

// D = |diag R|, Rt = D^-1 R P^T over Z and Q = (Q^T)^T, rows w n / S ...
// (w + 1) n / S of each; R is Pf on the panels' diagonal blocks and W right
// of them.  Thread c takes column c of those rows, eight rows' loads in
// flight at a time (clamped addresses, so none waits behind a branch).
__global__ __launch_bounds__(256) void qr_wide_final_kernel(double* __restrict__ Zg, const double* __restrict__ Wg,
                                                            double* __restrict__ Qg, double* __restrict__ Dg,
                                                            const double* __restrict__ Xg, int n, int batch, int S) {
  __shared__ double norms[MAXN];
  __shared__ int perm[MAXN];
  const int z = blockIdx.x % batch, w = blockIdx.x / batch;
  const int c = threadIdx.x, cc = min(c, n - 1);
  const long nn = (long)n * n;
  double* Z = Zg + z * nn;
  const double* W = Wg + z * nn;
  double* Q = Qg + z * nn;
  const double* QT = Xg + (long)z * wide_stride(n);
  const double* Pf = QT + nn;
  wide_perm(QT + 2 * nn, n, S, norms, perm);
  const int r0 = (int)((long)w * n / S), r1 = (int)((long)(w + 1) * n / S);
  const int pc = perm[cc];
  constexpr int U = 8;
  for (int b = r0; b < r1; b += U) {
    double pf[U], wv[U], dg[U], qt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = min(b + u, r1 - 1);
      pf[u] = Pf[(long)r * n + cc];
      wv[u] = W[(long)r * n + cc];
      dg[u] = Pf[(long)r * n + r];
      qt[u] = QT[(long)cc * n + r];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = b + u;
      if (r < r1 && c < n) {
        const int pe = min(n, (r / NB + 1) * NB);        // end of the panel holding row r's diagonal
        const double d = fabs(dg[u]);
        Z[(long)r * n + pc] = (c < r) ? 0.0 : ((c < pe) ? pf[u] : wv[u]) / d;
        Q[(long)r * n + c] = qt[u];
        if (c == 0) Dg[(long)z * n + r] = d;
      }
    }
  }
}

// Panel p of the wide Gauss-Jordan inversion.  The matrix alternates between
// two work copies (W at even p, the scratch copy at odd p; step 0 reads M);
// the pivot rows and values of earlier panels are read from the scratch.
// Work items: every strip outside the panel, updated as
//   A[r][C] = [r not a pivot row of the panel] A[r][C] + F[r][:] A_old[P][C]
// (F: the eliminated panel, P: its pivot rows).  A wave's first strip is
// loaded before the elimination; its old pivot rows are taken from those
// registers afterwards.
template <int MX>
__global__ __launch_bounds__(256) void gj_wide_step_kernel(const double* __restrict__ Mg, double* __restrict__ Wg,
                                                           double* __restrict__ Xg, int n, int batch, int S, int p) {
  constexpr int RPL = Cap<MX>::rpl;
  constexpr int NTL = Cap<MX>::tiles;
  __shared__ double Fs[NB][VLD];           // the eliminated panel, column-major, zero tail
  __shared__ double Sc[4][NB + 1][NB + 1];   // per wave: the strip's old pivot rows (+ a row for the rest)
  __shared__ int usedf[MAXN];              // rows pivoted in earlier panels
  __shared__ int kmap[MAXN];               // row -> its pivot index in this panel, or -1
  __shared__ int prs[NB];                  // this panel's pivot rows and values
  __shared__ double pvs[NB];
  const int z = blockIdx.x % batch, w = blockIdx.x / batch;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const long nn = (long)n * n;
  double* X = Xg + (long)z * wide_stride(n);
  double* X2 = X;                          // second work copy
  int* perm_g = (int*)(X + nn);            // pivot row of column j
  double* pivot_g = X + nn + n;            // pivot value of column j (n doubles after n ints)
  const double* src = (p == 0) ? Mg + z * nn : ((p & 1) ? Wg + z * nn : X2);
  double* dst = (p & 1) ? X2 : Wg + z * nn;
  const int p0 = p * NB, nbw = min(NB, n - p0);
  const int nst = (n + 15) / 16;
  // the earlier pivots first (their loads retire first), then the panel, then
  // this wave's first strip; loads through a buffer resource, masked elements
  // reading 0 from outside it
  const int prev = (tid < p0) ? perm_g[tid] : -1;
  const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(src, (unsigned)(nn * 8));
  double a[NB][RPL];
#pragma unroll
  for (int c = 0; c < NB; ++c)
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + 64 * t;
      a[c][t] = buf_load_f64(rs, (c < nbw && r < n) ? (unsigned)((r * n + p0 + c) * 8) : BUF_OUTSIDE);
    }
  auto load_strip = [&](int it, d4 (&tile)[NTL]) __attribute__((always_inline)) {
    const int s = (it < p) ? it : it + 1;
    const int col = 16 * s + li;
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + frag_row<double>(lane, v);
        tile[t][v] = buf_load_f64(rs, (row < n && col < n) ? (unsigned)((row * n + col) * 8) : BUF_OUTSIDE);
      }
  };
  const int it0 = w * 4 + wave;
  d4 tile[NTL];
  if (it0 < nst - 1) load_strip(it0, tile);

  if (tid < MAXN) {
    usedf[tid] = 0;
    kmap[tid] = -1;
  }
  __syncthreads();
  if (prev >= 0) usedf[prev] = 1;
  __syncthreads();
  bool used[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + 64 * t;
    used[t] = (r < n) ? usedf[r] != 0 : true;
  }
  gj_panel_wave<RPL>(nbw, n, a, used, prs, pvs);
  __syncthreads();
  if (tid < nbw) {
    kmap[prs[tid]] = tid;
    if (w == 0) {
      perm_g[p0 + tid] = prs[tid];
      pivot_g[p0 + tid] = pvs[tid];
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if ((c & 3) == wave) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        if (r < VLD) Fs[c][r] = (c < nbw && r < n) ? a[c][t] : 0.0;
        if (w == 0 && c < nbw && r < n) dst[(long)r * n + p0 + c] = a[c][t];
      }
    }
  if (64 * RPL < VLD) Fs[tid >> 4][64 * RPL + (tid & 15)] = 0.0;
  __syncthreads();

  for (int it = it0; it < nst - 1; it += 4 * S) {
    if (it != it0) load_strip(it, tile);
    const int s = (it < p) ? it : it + 1;
    const int col = 16 * s + li;
    // the strip's old pivot rows (k, column) to LDS from the registers that
    // hold them, and those rows as 0 in the tiles; every element is written,
    // the rows that are no pivot of this panel to the spare row NB, so that
    // no LDS access sits behind a branch
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = lane + 64 * i;
      Sc[wave][e >> 4][e & 15] = 0.0;
    }
    wave_sync_lds();
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + frag_row<double>(lane, v);
        const int k = (row < n) ? kmap[row] : -1;
        Sc[wave][(k >= 0) ? k : NB][li] = tile[t][v];
        tile[t][v] = (k >= 0) ? 0.0 : tile[t][v];
      }
    wave_sync_lds();
    double tb[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) tb[q] = Sc[wave][4 * q + lk][li];
    wave_sync_lds();
#pragma unroll
    for (int t = 0; t < NTL; ++t)
      if (16 * t < n) {
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) tile[t] = mfma16(Fs[4 * q + lk][16 * t + li], tb[q], tile[t]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + frag_row<double>(lane, v);
          if (row < n && col < n) dst[(long)row * n + col] = tile[t][v];
        }
      }
  }
}

// M^-1[j][perm[k]] = A[perm[j]][k] scaled, over M (rows w n / S ... of A;
// thread k takes column k, eight rows' loads in flight at a time); workgroup
// 0 also forms logdet = base + sum log|pivot|
__global__ __launch_bounds__(256) void gj_wide_final_kernel(double* __restrict__ Mg, const double* __restrict__ Wg,
                                                            const double* __restrict__ Xg,
                                                            const double* __restrict__ rsg,
                                                            const double* __restrict__ csg,
                                                            const double* __restrict__ base,
                                                            double* __restrict__ logdet, int n, int batch, int S,
                                                            int npan) {
  __shared__ int perm[MAXN];
  __shared__ int pinv[MAXN];
  __shared__ double part[4];
  const int z = blockIdx.x % batch, w = blockIdx.x / batch;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long nn = (long)n * n;
  const double* X = Xg + (long)z * wide_stride(n);
  const int* perm_g = (const int*)(X + nn);
  const double* pivot_g = X + nn + n;
  const double* A = ((npan - 1) & 1) ? X : Wg + z * nn;   // the last step's output
  double* M = Mg + z * nn;
  const double* rs = rsg + (long)z * n;
  const double* cs = csg + (long)z * n;
  for (int j = tid; j < n; j += 256) {
    const int r = perm_g[j];
    perm[j] = r;
    pinv[r] = j;
  }
  __syncthreads();
  const int r0 = (int)((long)w * n / S), r1 = (int)((long)(w + 1) * n / S);
  const int k = tid, kc = min(k, n - 1);
  const int pk = perm[kc];
  const double ck = cs[pk];
  constexpr int U = 8;
  for (int b = r0; b < r1; b += U) {
    double av[U], rj[U];
    int jr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = min(b + u, r1 - 1);
      jr[u] = pinv[r];
      av[u] = A[(long)r * n + kc];
      rj[u] = rs[jr[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (b + u < r1 && k < n) M[(long)jr[u] * n + pk] = rj[u] * av[u] * ck;
  }
  if (w == 0) {
    double lg = 0.0;
    for (int i = tid; i < n; i += 256) lg += log(fabs(pivot_g[i]));
    lg = wave_total(lg);
    if (lane == 0) part[wave] = lg;
    __syncthreads();
    if (tid == 0) logdet[z] = base[z] + ((part[0] + part[1]) + (part[2] + part[3]));
  }
}

bool qr_supported(int n) { return n >= 1 && n <= MAXN; }
bool gj_supported(int n) { return n >= 1 && n <= MAXN; }
size_t qr_t_doubles(int n) { return (size_t)NB * (n + NB); }

hipError_t launch_qr(double* Z, double* W, double* Q, double* D, double* T, int n, int batch, hipStream_t s,
                     double* X) {
  if (!qr_supported(n)) return hipErrorInvalidValue;
  const int S = X ? qr_wide_split(n, batch) : 1;
  if (S > 1) {
    const dim3 grid(batch * S);
    hipLaunchKernelGGL(qr_wide_norms_kernel, grid, dim3(256), 0, s, Z, X, n, batch, S);
    for (int p = 0; p < (n + NB - 1) / NB; ++p)
      hipLaunchKernelGGL(qr_wide_step_kernel<256>, grid, dim3(256), 0, s, Z, W, X, n, batch, S, p);
    hipLaunchKernelGGL(qr_wide_final_kernel, grid, dim3(256), 0, s, Z, W, Q, D, X, n, batch, S);
    return hipGetLastError();
  }
  // R, D and Rt (in registers up to N = 144, else through L2), then Q in a
  // launch of its own
  const dim3 qgrid((n + 63) / 64, batch);
  if (n <= 64) {
    hipLaunchKernelGGL(qr_regs_kernel<64>, dim3(batch), dim3(256), 0, s, Z, W, Q, D, T, n);
    hipLaunchKernelGGL(qr_formq_kernel<64>, qgrid, dim3(256), 0, s, W, T, Q, n);
  } else if (n <= 112) {
    hipLaunchKernelGGL(qr_regs_kernel<112>, dim3(batch), dim3(256), 0, s, Z, W, Q, D, T, n);
    hipLaunchKernelGGL(qr_formq_kernel<112>, qgrid, dim3(256), 0, s, W, T, Q, n);
  } else if (n <= 144) {
    hipLaunchKernelGGL(qr_regs_kernel<144>, dim3(batch), dim3(256), 0, s, Z, W, Q, D, T, n);
    hipLaunchKernelGGL(qr_formq_kernel<144>, qgrid, dim3(256), 0, s, W, T, Q, n);
  } else {
    hipLaunchKernelGGL(qr_blocked_kernel<256>, dim3(batch), dim3(256), 0, s, Z, W, Q, D, T, n);
    hipLaunchKernelGGL(qr_formq_kernel<256>, qgrid, dim3(256), 0, s, W, T, Q, n);
  }
  return hipGetLastError();
}

hipError_t launch_gj(double* M, double* W, const double* rs, const double* cs, const double* base, double* logdet,
                     int n, int batch, hipStream_t s, double* X) {
  if (!gj_supported(n)) return hipErrorInvalidValue;
  const int S = X ? gj_wide_split(n, batch) : 1;
  if (S > 1) {
    const dim3 grid(batch * S);
    const int npan = (n + NB - 1) / NB;
    for (int p = 0; p < npan; ++p)
      hipLaunchKernelGGL(gj_wide_step_kernel<256>, grid, dim3(256), 0, s, M, W, X, n, batch, S, p);
    hipLaunchKernelGGL(gj_wide_final_kernel, grid, dim3(256), 0, s, M, W, X, rs, cs, base, logdet, n, batch, S, npan);
    return hipGetLastError();
  }
  if (n <= 64)
    hipLaunchKernelGGL(gj_regs_kernel<64>, dim3(batch), dim3(256), 0, s, M, W, rs, cs, base, logdet, n);
  else if (n <= 112)
    hipLaunchKernelGGL(gj_regs_kernel<112>, dim3(batch), dim3(256), 0, s, M, W, rs, cs, base, logdet, n);
  else if (n <= 144)
    hipLaunchKernelGGL(gj_regs_kernel<144>, dim3(batch), dim3(256), 0, s, M, W, rs, cs, base, logdet, n);
  else
    hipLaunchKernelGGL(inv_blocked_kernel<256>, dim3(batch), dim3(256), 0, s, M, W, rs, cs, base, logdet, n);
  return hipGetLastError();
}

}  // namespace hq
