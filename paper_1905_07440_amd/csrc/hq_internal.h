// Internal interfaces between the host layer (hq_api.hip) and the kernel
// translation units of libhq.  Every launcher enqueues on the given stream
// and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hq {

// Diagonal scaling used by the GEMM epilogue and the Kronecker products:
//   value(z, i) = v[outer*so + inner*si + off + i]            (plain)
//   value(z, i) = exp(cmul * coef[outer] * v[...])             (coef != null)
// with outer = z / inner_count, inner = z % inner_count for batch entry z.
// A null v means value 1.  invert = 1 takes the reciprocal.
struct Scale {
  const double* v = nullptr;
  long off = 0, so = 0, si = 0;
  const double* coef = nullptr;
  double cmul = 0.0;
  int invert = 0;
};

// C[z] = alpha * diag(rs) * op(A[z]) * diag(ks) * op(B[z]) * diag(cs) + beta * C[z]
// for z in [0, batch); matrices row-major.  op = transpose when trans != 0.
// Matrix pointers advance by the stride per batch entry (stride 0 = shared);
// with split > 0 the batch is read as groups of split entries: entry z sits
// at (z / split) * sXo + (z % split) * sX.
template <typename T>
struct GemmArgs {
  int M = 0, N = 0, K = 0;
  const T* A = nullptr; long lda = 0, sA = 0; int tA = 0;
  const T* B = nullptr; long ldb = 0, sB = 0; int tB = 0;
  T* C = nullptr; long ldc = 0, sC = 0;
  int split = 0; long sAo = 0, sBo = 0, sCo = 0;
  double alpha = 1.0, beta = 0.0;
  Scale rs, cs, ks;                        // ks: on the inner index, K <= 256
  int batch = 1, inner_count = 1;
};

// Workgroups are dealt to the eight XCDs in turn (workgroup g runs on XCD
// g mod 8), each XCD with its own L2.  The grid is one-dimensional and is
// read so that all tiles of one batch entry land on the same XCD: XCD x
// takes entries x, x + 8, ..., tile by tile, and the entry's operands are
// fetched into that L2 once.  Returns false for the padding workgroups of a
// batch that is not a multiple of 8.
constexpr int N_XCD = 8;
__device__ inline bool xcd_tile(int tiles, int batch, int& z, int& tile) {
  const int g = blockIdx.x, x = g % N_XCD, k = g / N_XCD;
  z = N_XCD * (k / tiles) + x;
  tile = k % tiles;
  return z < batch;
}
inline unsigned xcd_grid(int tiles, int batch) { return (unsigned)(N_XCD * ((batch + N_XCD - 1) / N_XCD) * tiles); }

// offset of batch entry z: z * s, or, with split > 0 entries per group,
// (z / split) * so + (z % split) * s
__device__ inline long batch_offset(int z, int split, long s, long so) {
  if (split <= 0) return (long)z * s;
  const int o = z / split;
  return (long)o * so + (long)(z - o * split) * s;
}

__device__ inline double scale_value(const Scale& s, int z, int inner_count, int i) {
  if (!s.v) return 1.0;
  const int outer = z / inner_count, inner = z - outer * inner_count;
  double v = s.v[(long)outer * s.so + (long)inner * s.si + s.off + i];
  if (s.coef) v = exp(s.cmul * s.coef[outer] * v);
  if (s.invert) v = 1.0 / v;
  return v;
}

// GEMM tile configurations (see gemm.hip); the autotuner picks one per shape.
// TILE_FK_*: the whole K extent staged at once (needs K small enough for LDS).
// TILE_PF_*: each thread prefetches its whole share of K into registers.
// TILE_DX_*: every wave loads its own operands into registers, no LDS staging.
enum GemmTile { TILE_64x64 = 0, TILE_32x32 = 1, TILE_48x48 = 2, TILE_16x64 = 3, TILE_FK_32x32 = 4, TILE_FK_48x48 = 5,
                TILE_FK_64x64 = 6, TILE_FK_32x64 = 7, TILE_PF_48x48 = 8, TILE_PF_64x64 = 9, TILE_PF_32x32 = 10,
                TILE_DX_48x48 = 11, TILE_DX_32x32 = 12, TILE_DX_64x64 = 13, N_GEMM_TILES = 14 };

// Both products of a wrap for every chain in one launch (gemm.hip):
//   Gout[z] = diag(rs2) (A1 diag(ks1) Gin[z] diag(cs1)) A2 diag(cs2)
// A1, A2 shared by the batch (n x n, row-major); Gout must not overlap Gin.
template <typename T>
struct WrapArgs {
  int n = 0, batch = 0;
  const T* A1 = nullptr;
  const T* A2 = nullptr;
  const T* Gin = nullptr;
  T* Gout = nullptr;
  long sG = 0;
  Scale ks1, cs1, rs2, cs2;
};
bool wrap_fused_supported(int n, bool fp32);
hipError_t launch_wrap_fused(const WrapArgs<double>& w, hipStream_t s);
hipError_t launch_wrap_fused(const WrapArgs<float>& w, hipStream_t s);

// Products with A (x) A for an nx x nx factor A (kron.hip), the form that
// exp(s dtau K) takes on the periodic square lattice; site i = ix + nx iy.
//   side 0: Y[z] = diag(r_{S-1}) (A (x) A) ... diag(r_0) (A (x) A) diag(ks) X[z] diag(cs)
//           for S = steps, r_t = rs read at rs.off + t * rstep (rstep may be
//           negative); with pre = 1 each scale comes before its product:
//           Y[z] = (A (x) A) diag(r_{S-1}) ... (A (x) A) diag(r_0) diag(ks) X[z] diag(cs)
//   side 1: Y[z] = diag(rs) X[z] diag(ks) (A (x) A) diag(cs)     (steps = 1)
// X, Y n x n row-major (n = nx^2 <= 256), advancing by sX, sY per batch
// entry (sX = 0: one X for the whole batch); Y must not overlap X.  A shared
// by the batch.  steps * n <= KRON_MAX_SCALES.
constexpr int KRON_MAX_SCALES = 2048;
template <typename T>
struct KronArgs {
  int nx = 0, n = 0, batch = 0, inner_count = 1;
  const T* A = nullptr;
  const T* X = nullptr; long sX = 0;
  T* Y = nullptr; long sY = 0;
  Scale rs, ks, cs;
  int steps = 1; long rstep = 0;
  int pre = 0;
};
// A whole wrap Y = diag(rs2) (A1 (x) A1) diag(ks1) X diag(cs1) (A2 (x) A2)
// diag(cs2) in one launch, X resident in LDS (kron.hip): nx <= 12 in FP32,
// nx <= 10 in FP64.  Y must not overlap X.
template <typename T>
struct KronWrapArgs {
  int nx = 0, batch = 0;
  const T* A1 = nullptr;
  const T* A2 = nullptr;
  const T* X = nullptr; long sX = 0;
  T* Y = nullptr; long sY = 0;
  Scale ks1, cs1, rs2, cs2;
};
bool kron_wrap_lds_supported(int nx, bool fp32);
hipError_t launch_kron_wrap_lds(const KronWrapArgs<double>& w, hipStream_t s);
hipError_t launch_kron_wrap_lds(const KronWrapArgs<float>& w, hipStream_t s);
hipError_t launch_kron(const KronArgs<double>& a, int side, hipStream_t s);
hipError_t launch_kron(const KronArgs<float>& a, int side, hipStream_t s);

hipError_t launch_gemm(const GemmArgs<double>& a, int tile, hipStream_t s);
hipError_t launch_gemm(const GemmArgs<float>& a, int tile, hipStream_t s);
// two products of one M x N shape in one launch (one after the other where the tile cannot pair them)
hipError_t launch_gemm_pair(const GemmArgs<double>& a, const GemmArgs<double>& b, int tile, hipStream_t s);
bool gemm_tile_fits(int tile, int K, int precision);
hipError_t prepare_gemm();

// ---------------------------------------------------------------------------
// local moves of one slice: one workgroup per chain, sites in blocks of kd
// (local.hip)
// ---------------------------------------------------------------------------
struct LocalArgs {
  int n = 0, L = 0, slice = 0;
  void* G = nullptr;            // [C][n][n], double or float
  double* x = nullptr;          // [C][L][n]
  const double* g = nullptr;    // [C]
  double dtau = 0, mass = 0, omega = 0, width = 0;
  uint64_t seed = 0;
  int chain0 = 0;               // global index of chain 0 of this group
  const int64_t* sweep = nullptr;   // device sweep counter
  double* logdet = nullptr;     // [C]
  int64_t* counters = nullptr;  // [C][8]: proposals, accepts per kind
  float* log_margin = nullptr;  // [C][L*n] or null
  uint8_t* log_accept = nullptr;
  const uint8_t* replay = nullptr;  // [C][L*n] (255 = none) or null
  double band = 0;
  int64_t* replay_counts = nullptr; // [C][2]
};
hipError_t launch_local(const LocalArgs& a, int precision, int nt, int kd, int chains, hipStream_t s);
size_t local_lds_bytes(int n, int precision, int nt, int kd);
bool local_supported(int n, int precision, int nt, int kd);
// whether the slice keeps G in LDS (else it is streamed from global memory)
bool local_g_in_lds(int n, int precision, int kd);
hipError_t prepare_local();

// ---------------------------------------------------------------------------
// dense FP64 factorizations: one workgroup per matrix (factor.hip)
// ---------------------------------------------------------------------------
// Householder QR of Z[z] (n x n, n <= 256) with columns pre-sorted by
// decreasing norm, Z P = Q R.  Outputs Q (explicit), D = |diag R| and, over Z,
// Rt = D^-1 R P^T.  W: n x n work per matrix; T: qr_t_doubles(n) per matrix.
// X (optional): wide_scratch_doubles(n) per matrix; given, and with
// wide_split(n, batch) > 1, the factorization of each matrix is spread over
// that many workgroups (one launch per panel).
hipError_t launch_qr(double* Z, double* W, double* Q, double* D, double* T, int n, int batch, hipStream_t s,
                     double* X = nullptr);
bool qr_supported(int n);
size_t qr_t_doubles(int n);
size_t wide_scratch_doubles(int n);
int wide_split(int n, int batch);

// Gauss-Jordan inversion with partial pivoting: over M, diag(rs) M^-1 diag(cs)
// (rs, cs: [batch][n]); logdet[z] = base[z] + log|det M|.  W: n x n work.
// X (optional): as for launch_qr.
hipError_t launch_gj(double* M, double* W, const double* rs, const double* cs, const double* base,
                     double* logdet, int n, int batch, hipStream_t s, double* X = nullptr);
bool gj_supported(int n);

// ---------------------------------------------------------------------------
// small kernels (misc.hip)
// ---------------------------------------------------------------------------
hipError_t launch_identity(double* U, double* D, double* T, int n, int batch, hipStream_t s);
// dbinv = 1/max(D,1), ds = min(D,1), sumlog[z] (+)= sum log max(D,1)
hipError_t launch_dsplit2(const double* DL, double* lbinv, double* ls, const double* DR, double* rbinv, double* rs,
                          double* sumlog, int n, int batch, hipStream_t s);
hipError_t launch_dsplit(const double* D, double* dbinv, double* ds, double* sumlog, int accumulate,
                         int n, int batch, hipStream_t s);
// M = diag(dbinv) U^T + diag(ds) T per chain ([batch] n x n, U and T with chain strides sU, sT)
hipError_t launch_merge_identity(const double* U, long sU, const double* T, long sT, const double* dbinv,
                                 const double* ds, double* M, int n, int batch, hipStream_t s);
// drift of the tracked state against the recomputed one, then replace it;
// part: stab_part_doubles(batch) of scratch.  saved / saved_logdet (may be
// null): the tracked G (as FP64) and log det just before the replacement
size_t stab_part_doubles(int batch);
hipError_t launch_stab_finish(void* G, int precision, const double* Gnew, double* logdet,
                              const double* logdet_new, double* drift, double* part, int n, int batch,
                              int record_drift, hipStream_t s, double* saved = nullptr,
                              double* saved_logdet = nullptr);
hipError_t launch_copy_f64_to_f32(float* dst, const double* src, long count, hipStream_t s);
hipError_t launch_copy_f32_to_f64(double* dst, const float* src, long count, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t v, long count, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, long count, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, long count, hipStream_t s);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s);

struct GlobalArgs {
  int n = 0, L = 0, nb = 0, site = 0;
  double* x = nullptr;          // [C][L][n]
  double* xp = nullptr;         // [C][L][n] proposal fields
  const double* g = nullptr;
  double dtau = 0, mass = 0, omega = 0, width = 0;
  uint64_t seed = 0;
  int chain0 = 0;
  const int64_t* sweep = nullptr;
  double* shift = nullptr;      // [C] proposed shift
  double* logdet = nullptr;
  const double* logdet_new = nullptr;
  void* G = nullptr; int precision = 0;
  const double* Gnew = nullptr;
  int64_t* counters = nullptr;
  float* log_margin = nullptr; uint8_t* log_accept = nullptr;
  const uint8_t* replay = nullptr; double band = 0; int64_t* replay_counts = nullptr;
};
hipError_t launch_global_propose(const GlobalArgs& a, int chains, hipStream_t s);
hipError_t launch_global_accept(const GlobalArgs& a, int chains, hipStream_t s);

struct ObsArgs {
  int n = 0, L = 0, nx = 0;
  const void* G = nullptr; int precision = 0;
  const double* x = nullptr;
  double* out = nullptr;        // [C][5]: density, double occ, S_cdw, <x>, <x^2>
  int* flags = nullptr;         // [C]
  const double* logdet = nullptr;
};
hipError_t launch_observables(const ObsArgs& a, int chains, hipStream_t s);

// ---------------------------------------------------------------------------
// network proposals (network.hip)
// ---------------------------------------------------------------------------
struct NetArgs {
  int nx = 0, n = 0, L = 0, colour = 0;
  int inner = 0, nu = 1;        // inner sweep u of n_u: draws and log slots at u*L*n + l*n + i
  double* xp = nullptr;         // [C][L][n] proposal fields (updated in place)
  const double* g = nullptr;
  double dtau = 0, mass = 0, omega = 0, width = 0;
  uint64_t seed = 0;
  int chain0 = 0;
  const int64_t* sweep = nullptr;
  const float* w = nullptr;     // 7169 weights
  int activation = 0;
  int chains = 0;
  double* sum_y = nullptr;      // [C][L*n]: network outputs of the accepted proposals, summed over inner sweeps
  uint8_t* accepted = nullptr;  // [C][L*n]: accepted proposals, counted over inner sweeps
  int64_t* counters = nullptr;
  float* log_margin = nullptr; uint8_t* log_accept = nullptr;
  const uint8_t* replay = nullptr; double band = 0; int64_t* replay_counts = nullptr;
};
hipError_t launch_network_colour(const NetArgs& a, int chains, hipStream_t s);
// network block moves of one colour class (iy mod 2, ix mod 2) of inner sweep
// u: one thread per site, the convolutional network's weights in LDS
struct CnnArgs {
  int nx = 0, n = 0, L = 0, colour = 0, inner = 0, nu = 1;   // draws and log slots at u*n + i
  double* xp = nullptr;         // [C][L][n] proposal fields (columns shifted in place)
  const double* g = nullptr;
  double dtau = 0, mass = 0, omega = 0, width = 0;
  uint64_t seed = 0;
  int chain0 = 0;
  const int64_t* sweep = nullptr;
  const float* w = nullptr;     // 64 L + 117 weights
  int chains = 0;
  double* sum_y = nullptr;      // [C][n]: outputs of the accepted moves, summed over inner sweeps
  uint8_t* accepted = nullptr;  // [C][n]: accepted moves, counted over inner sweeps
  float* log_margin = nullptr; uint8_t* log_accept = nullptr;
  const uint8_t* replay = nullptr; double band = 0; int64_t* replay_counts = nullptr;
};
hipError_t launch_cnn_colour(const CnnArgs& a, int chains, hipStream_t s);
size_t cnn_lds_bytes(int L);
struct CumulativeArgs {
  int n = 0, L = 0, nb = 0;
  double* x = nullptr; const double* xp = nullptr;
  double* logdet = nullptr; const double* logdet_new = nullptr;
  void* G = nullptr; int precision = 0; const double* Gnew = nullptr;
  const double* sum_y = nullptr; const uint8_t* accepted = nullptr;
  const double* sum_yb = nullptr; const uint8_t* accepted_b = nullptr;   // block moves, [C][n], or null
  int inner = 1;                // n_u: proposals per slot of each kind
  uint64_t seed = 0; int chain0 = 0; const int64_t* sweep = nullptr;
  int64_t* counters = nullptr;
  float* log_margin = nullptr; uint8_t* log_accept = nullptr;
  const uint8_t* replay = nullptr; double band = 0; int64_t* replay_counts = nullptr;
  double* last_log_pc = nullptr;
};
hipError_t launch_cumulative(const CumulativeArgs& a, int chains, hipStream_t s);
hipError_t launch_copy_f64(double* dst, const double* src, long count, hipStream_t s);
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, long count, hipStream_t s);
// up to four copies dst[o dso + i dsi + e] = src[o sso + i ssi + e] (e < len,
// o < outer, i < inner) in one launch; copies of nonpositive size are skipped
struct BlockCopy {
  double* dst = nullptr;
  const double* src = nullptr;
  long dso = 0, dsi = 0, sso = 0, ssi = 0, len = 0;
  int outer = 0, inner = 0;
};
struct BlockCopies {
  BlockCopy c[4];
  int k = 0;
};
hipError_t launch_copy_blocks_multi(const BlockCopies& c, hipStream_t s);

// counters layout per chain
enum { CNT_LOCAL_P = 0, CNT_LOCAL_A, CNT_GLOBAL_P, CNT_GLOBAL_A, CNT_NN_P, CNT_NN_A, CNT_CUM_P,
       CNT_CUM_A, N_COUNTERS };

}  // namespace hq
