// Host layer of libhq: validation, workspace layout, model set-up, the sweep
// schedule (captured once into a HIP graph and replayed), and the C ABI of
// include/hq.h.
//
// Sweep schedule of one group (paper, section "Determinant quantum Monte
// Carlo"; stabilisation as in the DQMC literature the paper cites):
//   right stack R_b = C_{nb-1} ... C_{b+1} (as UDT of its transpose) from the
//     cached block products C_b = B_{(b+1)ns-1} ... B_{b ns}, which are valid
//     because no field has changed since they were formed;
//   for each block b: for its n_stab slices: wrap, local moves; then form C_b
//     with the new fields, fold it into the left UDT L_b = C_b L_{b-1}, and
//     merge G = (I + L_b R_b)^-1 and log|det M| (FP64);
//   then the block moves (if enabled), each with a from-scratch determinant;
//   network groups instead run the colour classes of network proposals, a
//     from-scratch determinant of the proposal, and the cumulative accept.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hq.h"
#include "hq_device.h"
#include "hq_internal.h"

using namespace hq;

namespace {

const int N_KIND_SLOTS = 7;   // indexed by HQ_KIND_* (0, 1, 3, 4, 6 used)
const int KINDS[] = {HQ_KIND_LOCAL, HQ_KIND_GLOBAL, HQ_KIND_NN, HQ_KIND_CUMULATIVE, HQ_KIND_NN_GLOBAL};

// a wrap G <- B G B^-1 as two tiled dense products, as one fused launch of
// both dense products, as two Kronecker launches (left, then right), or as
// one Kronecker launch with G held in LDS
enum { WRAP_TWO = HQ_WRAP_TWO, WRAP_FUSED = HQ_WRAP_FUSED, WRAP_KRON = HQ_WRAP_KRON, WRAP_KRON_LDS = HQ_WRAP_KRON_LDS };

struct Group {
  hq_group p{};
  int nx = 0, n = 0, L = 0, ns = 0, nb = 0, C = 0, chain0 = 0;
  int nt = 256, kd = 16, tile = TILE_64x64, tile32 = TILE_64x64;
  int tile_wide = TILE_64x64;              // FP64 products over all blocks of all chains
  double tile_us = 0.0, tile32_us = 0.0;   // autotuner timings
  double local_us = 0.0;                   // timed local slice at the chosen block size (0: not timed)
  int64_t* tune_cnt = nullptr;             // counters of the timed local slices (thrown away)
  int wrap_kind = WRAP_TWO;                // how a wrap is computed (autotuner's choice)
  double wrap_us = 0.0;                    // measured time of one wrap as chosen
  bool global = false, network = false;
  // fields, couplings, model matrices
  double *x = nullptr, *xp = nullptr, *g = nullptr;
  double *expk = nullptr, *expkinv = nullptr, *ident = nullptr, *ones = nullptr;
  float *expk32 = nullptr, *expkinv32 = nullptr;
  // nx x nx factors E1 of expK = E1 (x) E1 and of expK^-1
  double *ek1 = nullptr, *ek1inv = nullptr;
  float *ek1_32 = nullptr, *ek1inv_32 = nullptr;
  // Green's functions
  void* G = nullptr;             // [C][n][n], precision of the context
  void* Wt = nullptr;            // wrap temporary, same precision
  // A one-launch wrap (fused dense, or Kronecker with G in LDS) writes G'
  // into Wt and the two buffers trade places; G0 is where G lives between
  // sweeps
  void* G0 = nullptr;
  double* Gnew = nullptr;        // [C][n][n]
  // block products and UDT stacks
  double *blk = nullptr, *blkp = nullptr, *blks = nullptr;     // [C][nb][n][n]
  double *RU = nullptr, *RD = nullptr, *RT = nullptr;          // [C][nb][n][n], [C][nb][n]
  double *LU = nullptr, *LD = nullptr, *LT[2] = {nullptr, nullptr};
  double *SU = nullptr, *SD = nullptr, *ST = nullptr;          // left stack [nb][C][n][n], [nb][C][n]
  // from-scratch products by pairwise UDT merges (groups with block moves or
  // the network): UDT pairs [C][nb] (ping-pong), the merged middle factors
  // [C][nb/2], and the QR's scratch for a batch of C * nb
  bool tree = false;
  double *tU[2] = {nullptr, nullptr}, *tT[2] = {nullptr, nullptr}, *tD[2] = {nullptr, nullptr};
  double *tX = nullptr, *tUp = nullptr, *tDp = nullptr, *tQW = nullptr, *tQT = nullptr;
  bool alternate = false;        // sweeps alternate upward / downward (local moves only)
  double *Z = nullptr, *Rt = nullptr, *M = nullptr, *Minv = nullptr, *Xm = nullptr, *Tq = nullptr;
  double* Xw = nullptr;                        // wide-factorization scratch (large N, few matrices)
  double *dLbinv = nullptr, *dLs = nullptr, *dRbinv = nullptr, *dRs = nullptr, *sumlog = nullptr;
  double *logdet = nullptr, *logdet_new = nullptr, *shift = nullptr;
  int64_t* counters = nullptr;
  double *drift = nullptr, *dpart = nullptr, *obs = nullptr, *lastpc = nullptr;
  int* flags = nullptr;
  int64_t* replay_counts = nullptr;
  float* log_margin[N_KIND_SLOTS] = {};
  double* Gtrk = nullptr;                  // record: tracked G and log det before the last replacement
  double* ldtrk = nullptr;
  uint8_t* log_accept[N_KIND_SLOTS] = {};
  uint8_t* replay[N_KIND_SLOTS] = {};
  double band[N_KIND_SLOTS] = {};
  double* sum_y = nullptr;
  uint8_t* nn_acc = nullptr;
  // network block moves (network groups with global_width > 0): n_u inner
  // sweeps of each kind per cumulative accept
  int nu = 1;
  bool cnn = false;
  double* sum_yb = nullptr;      // [C][n]
  uint8_t* acc_b = nullptr;      // [C][n]
  long kind_slots(int kind) const {
    if (kind == HQ_KIND_LOCAL) return (long)L * n;
    if (kind == HQ_KIND_NN) return (long)nu * L * n;
    if (kind == HQ_KIND_NN_GLOBAL) return (long)nu * n;
    if (kind == HQ_KIND_GLOBAL) return n;
    return 1;
  }
};

// bump allocator over the caller's workspace (a null base only measures)
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct hq_ctx {
  std::vector<Group> groups;
  hq_options opt{};
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t* sweep_counter = nullptr;
  float* net = nullptr;
  bool net_loaded = false;
  float* cnn = nullptr;          // block-move network weights, 64 L + 117 floats
  int cnn_max_L = 0;             // room for the largest L of a group with block-move networks
  int cnn_L = 0;                 // L the loaded weights are for (0: none)
  int n_chains = 0;
  bool broken = false;
  std::string err;
  // one captured graph per (direction, stack rebuild) and the host's view of
  // the sweep state: the next sweep's index and which UDT stack is current
  // [direction][stack rebuild][network scan reversed]
  hipGraph_t graph[2][2][2] = {};
  hipGraphExec_t exec[2][2][2] = {};
  int scan = 0;                  // the sweep being enqueued visits the network schedule in reverse
  bool any_network = false;
  int64_t sweep_index = 0;
  bool left_valid = false, right_valid = false;
  bool profiling = false;
  // per-phase event timing (profiling mode runs the schedule eagerly)
  struct Phase { const char* name; double ms; int64_t launches; };
  std::vector<Phase> phases;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<int> pending_phase;
  std::vector<hipEvent_t> event_pool;
  // groups of different lattices run as concurrent branches of the sweep
  // graph: one side stream per group, forked from and joined to `stream`
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  int static_device = -1;        // >= 0: the workspace is that device's static array
};

namespace {

hq_status fail(hq_ctx* c, hq_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) {
    c->err = buf;
    if (st == HQ_EDEVICE) c->broken = true;
  }
  return st;
}

#define HQ_TRY(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(ctx, HQ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool valid_group(const hq_group& p, const hq_options& o, std::string& why) {
  char b[256];
  if (p.nx < 1 || p.nx * p.nx > 256) { why = "nx must give 1 <= N <= 256"; return false; }
  if (p.n_chains < 1) { why = "n_chains must be >= 1"; return false; }
  if (!(p.dtau > 0) || !(p.beta > 0) || !std::isfinite(p.beta / p.dtau)) { why = "beta, dtau must be > 0"; return false; }
  const long L = lround(p.beta / p.dtau);
  if (L < 2 || std::fabs(L * p.dtau - p.beta) > 1e-9) { why = "beta/dtau must be an integer >= 2"; return false; }
  if (p.n_stab < 1 || L % p.n_stab) { why = "n_stab must divide L"; return false; }
  if (!(p.mass > 0) || !std::isfinite(p.t) || !std::isfinite(p.mu) || !std::isfinite(p.g) ||
      !std::isfinite(p.omega) || !(p.local_width >= 0) || !(p.global_width >= 0)) {
    why = "model parameters must be finite (mass > 0, widths >= 0)";
    return false;
  }
  if (p.proposal != HQ_PROPOSAL_DQMC && p.proposal != HQ_PROPOSAL_NETWORK) { why = "bad proposal"; return false; }
  if (p.proposal == HQ_PROPOSAL_NETWORK && (p.nx % 2 || L % 4)) {
    why = "network proposals need even nx and L divisible by 4";
    return false;
  }
  if (p.proposal == HQ_PROPOSAL_NETWORK && (p.nn_sweeps < 0 || p.nn_sweeps > 64)) {
    why = "nn_sweeps must be 0 .. 64";
    return false;
  }
  if (p.proposal == HQ_PROPOSAL_NETWORK && p.global_width > 0.0 && cnn_lds_bytes(L) > 65536) {
    why = "network block moves need 64 L + 117 weights within 64 KB (L <= 254)";
    return false;
  }
  const int n = p.nx * p.nx;
  if (!qr_supported(n) || !gj_supported(n)) {
    snprintf(b, sizeof b, "N = %d exceeds the factorization kernels (N <= 256)", n);
    why = b;
    return false;
  }
  if (p.proposal == HQ_PROPOSAL_DQMC) {
    const int nt = n <= 64 ? 64 : 256;
    const int kd = o.delay ? o.delay : 16;
    if (!local_supported(n, o.precision, nt, kd)) {
      snprintf(b, sizeof b, "N = %d (precision %d, delay %d) does not fit the local kernel's LDS", n,
               o.precision, kd);
      why = b;
      return false;
    }
  }
  return true;
}

// carve every buffer of every group; returns total bytes
size_t layout(hq_ctx* ctx, std::vector<Group>& gs, void* base, const hq_options& o) {
  Carver cv(base);
  const size_t ts = o.precision ? sizeof(float) : sizeof(double);
  for (Group& g : gs) {
    const long n = g.n, nn = n * n, C = g.C, L = g.L, nb = g.nb;
    g.x = cv.take<double>(C * L * n);
    g.xp = cv.take<double>(C * L * n);
    g.g = cv.take<double>(C);
    g.expk = cv.take<double>(nn);
    g.expkinv = cv.take<double>(nn);
    g.ident = cv.take<double>(nn);
    g.ones = cv.take<double>(C * n);
    g.expk32 = cv.take<float>(nn);
    g.expkinv32 = cv.take<float>(nn);
    g.ek1 = cv.take<double>((long)g.nx * g.nx);
    g.ek1inv = cv.take<double>((long)g.nx * g.nx);
    g.ek1_32 = cv.take<float>((long)g.nx * g.nx);
    g.ek1inv_32 = cv.take<float>((long)g.nx * g.nx);
    g.G = cv.take<char>(C * nn * ts);
    g.G0 = g.G;
    g.Wt = cv.take<char>(C * nn * ts);
    g.Gnew = cv.take<double>(C * nn);
    g.blk = cv.take<double>(C * nb * nn);
    g.blkp = cv.take<double>(C * nb * nn);
    g.blks = cv.take<double>(C * nb * nn);
    g.RU = cv.take<double>(C * nb * nn);
    g.RD = cv.take<double>(C * nb * n);
    g.RT = cv.take<double>(C * nb * nn);
    g.LU = cv.take<double>(C * nn);
    g.LD = cv.take<double>(C * n);
    g.LT[0] = cv.take<double>(C * nn);
    g.LT[1] = cv.take<double>(C * nn);
    g.SU = cv.take<double>(C * nb * nn);
    g.SD = cv.take<double>(C * nb * n);
    g.ST = cv.take<double>(C * nb * nn);
    g.Z = cv.take<double>(C * nn);
    g.Rt = cv.take<double>(C * nn);
    g.M = cv.take<double>(C * nn);
    g.Minv = cv.take<double>(C * nn);
    g.Xm = cv.take<double>(C * nn);
    g.Tq = cv.take<double>(C * (long)qr_t_doubles(g.n));
    // the wide factorizations' scratch, for the largest batch of this group
    // that they take: the group's C matrices, and the levels of the pairwise
    // UDT tree (C * nb, C * pairs, ...) small enough to spread
    long wide_batch = wide_split(g.n, C) > 1 ? C : 0;
    if ((g.global || g.network) && nb > 1) {
      if (wide_split(g.n, (int)(C * nb)) > 1) wide_batch = std::max(wide_batch, C * nb);
      for (long m = nb; m > 1; m = (m + 1) / 2)
        if (wide_split(g.n, (int)(C * (m / 2))) > 1) wide_batch = std::max(wide_batch, C * (m / 2));
    }
    if (wide_batch) g.Xw = cv.take<double>(wide_batch * (long)wide_scratch_doubles(g.n));
    g.dLbinv = cv.take<double>(C * n);
    g.dLs = cv.take<double>(C * n);
    g.dRbinv = cv.take<double>(C * n);
    g.dRs = cv.take<double>(C * n);
    g.sumlog = cv.take<double>(C);
    g.logdet = cv.take<double>(C);
    g.logdet_new = cv.take<double>(C);
    g.shift = cv.take<double>(C);
    g.counters = cv.take<int64_t>(C * N_COUNTERS);
    g.tune_cnt = cv.take<int64_t>(C * N_COUNTERS);
    g.drift = cv.take<double>(C * 5);
    g.dpart = cv.take<double>((long)stab_part_doubles(C));
    g.obs = cv.take<double>(C * 5);
    g.lastpc = cv.take<double>(C * 2);
    g.flags = cv.take<int>(C);
    g.replay_counts = cv.take<int64_t>(C * 2);
    for (int k : KINDS) {
      const long slots = C * g.kind_slots(k);
      g.replay[k] = cv.take<uint8_t>(slots);
      if (o.record) {
        g.log_margin[k] = cv.take<float>(slots);
        g.log_accept[k] = cv.take<uint8_t>(slots);
      }
    }
    if (o.record) {
      g.Gtrk = cv.take<double>(C * nn);
      g.ldtrk = cv.take<double>(C);
    }
    if (g.network) {
      g.sum_y = cv.take<double>(C * L * n);
      g.nn_acc = cv.take<uint8_t>(C * L * n);
      if (g.cnn) {
        g.sum_yb = cv.take<double>(C * n);
        g.acc_b = cv.take<uint8_t>(C * n);
      }
    }
    g.tree = (g.global || g.network) && nb > 1;
    if (g.tree) {
      const long half = (nb + 1) / 2;
      for (int k = 0; k < 2; ++k) {
        g.tU[k] = cv.take<double>(C * nb * nn);
        g.tT[k] = cv.take<double>(C * nb * nn);
        g.tD[k] = cv.take<double>(C * nb * n);
      }
      g.tX = cv.take<double>(C * half * nn);
      g.tUp = cv.take<double>(C * half * nn);
      g.tDp = cv.take<double>(C * half * n);
      g.tQW = cv.take<double>(C * nb * nn);
      g.tQT = cv.take<double>(C * nb * (long)qr_t_doubles(g.n));
    }
  }
  int cnn_L = 0;
  for (const Group& g : gs)
    if (g.cnn) cnn_L = std::max(cnn_L, g.L);
  if (ctx) {
    ctx->sweep_counter = cv.take<int64_t>(1);
    ctx->net = cv.take<float>(7169 + 7);
    ctx->cnn_max_L = cnn_L;
    if (cnn_L) ctx->cnn = cv.take<float>(64L * cnn_L + 117);
  } else {
    cv.take<int64_t>(1);
    cv.take<float>(7169 + 7);
    if (cnn_L) cv.take<float>(64L * cnn_L + 117);
  }
  return cv.off + 256;
}

bool build_groups(const hq_group* gp, int ng, const hq_options& o, std::vector<Group>& out, std::string& why) {
  out.clear();
  int chain0 = 0;
  for (int k = 0; k < ng; ++k) {
    if (!valid_group(gp[k], o, why)) return false;
    Group g;
    g.p = gp[k];
    g.nx = gp[k].nx;
    g.n = g.nx * g.nx;
    g.L = (int)lround(gp[k].beta / gp[k].dtau);
    g.ns = gp[k].n_stab;
    g.nb = g.L / g.ns;
    g.C = gp[k].n_chains;
    g.chain0 = chain0;
    g.global = gp[k].global_width > 0.0 && gp[k].proposal == HQ_PROPOSAL_DQMC;
    g.network = gp[k].proposal == HQ_PROPOSAL_NETWORK;
    g.cnn = g.network && gp[k].global_width > 0.0;
    g.nu = g.network ? std::max(1, (int)gp[k].nn_sweeps) : 1;
    g.alternate = !g.global && !g.network;
    g.nt = g.n <= 64 ? 64 : 256;
    g.kd = o.delay ? o.delay : 16;
    g.tile = g.n <= 32 ? TILE_32x32 : TILE_64x64;
    g.tile32 = g.tile;
    chain0 += g.C;
    out.push_back(g);
  }
  return true;
}

// exp(sign * dtau * K) from the plane-wave decomposition of the periodic
// hopping matrix: (1/N) sum_k cos(k . (r_i - r_j)) exp(-sign' dtau eps_k),
// eps_k = -2t (cos kx + cos ky) - mu.
void exp_hopping(const hq_group& p, double sign, std::vector<double>& out) {
  const int nx = p.nx, n = nx * nx;
  std::vector<double> f((size_t)n, 0.0);
  const double tw = 2.0 * M_PI / nx;
  for (int dy = 0; dy < nx; ++dy)
    for (int dx = 0; dx < nx; ++dx) {
      double s = 0.0;
      for (int my = 0; my < nx; ++my)
        for (int mx = 0; mx < nx; ++mx) {
          const double kx = tw * mx, ky = tw * my;
          const double eps = -2.0 * p.t * (std::cos(kx) + std::cos(ky)) - p.mu;
          s += std::cos(kx * dx + ky * dy) * std::exp(sign * p.dtau * eps);
        }
      f[dx + nx * dy] = s / n;
    }
  out.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int dx = ((i % nx) - (j % nx) + nx) % nx, dy = ((i / nx) - (j / nx) + nx) % nx;
      out[(size_t)i * n + j] = f[dx + nx * dy];
    }
}

// The nx x nx factor E1 of exp(sign * dtau * K) = E1 (x) E1 (site index
// ix + nx iy): the plane-wave energy splits into -2t cos kx - mu/2 and
// -2t cos ky - mu/2, and the sine terms of the sum above cancel between k
// and -k, so E1[a][b] = (1/nx) sum_k cos(k (a - b)) exp(sign dtau (-2t cos k - mu/2)).
void exp_hopping_1d(const hq_group& p, double sign, std::vector<double>& out) {
  const int nx = p.nx;
  std::vector<double> f((size_t)nx, 0.0);
  const double tw = 2.0 * M_PI / nx;
  for (int d = 0; d < nx; ++d) {
    double s = 0.0;
    for (int m = 0; m < nx; ++m) {
      const double k = tw * m;
      s += std::cos(k * d) * std::exp(sign * p.dtau * (-2.0 * p.t * std::cos(k) - 0.5 * p.mu));
    }
    f[d] = s / nx;
  }
  out.assign((size_t)nx * nx, 0.0);
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < nx; ++b) out[(size_t)a * nx + b] = f[(a - b + nx) % nx];
}

// ---------------------------------------------------------------------------
// schedule building blocks (all FP64 unless noted)
// ---------------------------------------------------------------------------
struct Sched {
  hq_ctx* ctx;
  hipStream_t s;
  int phase = -1;   // profiling phase of the launches being issued
};

// the replay log of one kind, or null: replay is a test facility of contexts
// created with options.record = 1, and the kernels of other contexts carry
// none of its work
const uint8_t* replay_of(const hq_ctx* ctx, const Group& g, int kind) {
  return ctx->opt.record ? g.replay[kind] : nullptr;
}

hq_status begin_phase(Sched& S, int ph) {
  hq_ctx* ctx = S.ctx;
  if (!ctx->profiling) return HQ_OK;
  hipEvent_t a, b;
  if (ctx->event_pool.size() >= 2) {
    a = ctx->event_pool.back(); ctx->event_pool.pop_back();
    b = ctx->event_pool.back(); ctx->event_pool.pop_back();
  } else {
    HQ_TRY(hipEventCreate(&a));
    HQ_TRY(hipEventCreate(&b));
  }
  HQ_TRY(hipEventRecord(a, S.s));
  ctx->pending.push_back({a, b});
  ctx->pending_phase.push_back(ph);
  S.phase = ph;
  return HQ_OK;
}
hq_status end_phase(Sched& S) {
  hq_ctx* ctx = S.ctx;
  if (!ctx->profiling || S.phase < 0) return HQ_OK;
  HQ_TRY(hipEventRecord(ctx->pending.back().second, S.s));
  S.phase = -1;
  return HQ_OK;
}
enum { PH_WRAP = 0, PH_LOCAL, PH_STAB, PH_GLOBAL, PH_NETWORK, N_PHASES };
const char* kPhaseNames[N_PHASES] = {"wrap", "local", "stab", "global", "network"};

#define SCHED_TRY(expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(S.ctx, HQ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
#define ST_TRY(expr)                  \
  do {                                \
    hq_status st_ = (expr);           \
    if (st_ != HQ_OK) return st_;     \
  } while (0)

GemmArgs<double> sq(const Group& g, int batch) {
  GemmArgs<double> a;
  a.M = a.N = a.K = g.n;
  a.lda = a.ldb = a.ldc = g.n;
  a.batch = batch;
  return a;
}

// block products C_{c,b} = B_{b ns + ns - 1} ... B_{b ns} of the fields xs for
// blocks b0 .. b0+nblk-1 of every chain, B_l = diag(exp(-dtau g x_l)) expK,
// as Kronecker chains from the identity (one launch while ns * n fits the
// kernel's table of row scales, else chunks through the scratch buffer).
// dst stride per chain: nb*n*n when nblk == 1 (into the cached array), else
// dst is [C][nblk][n][n] contiguous.
hq_status block_products(Sched& S, Group& g, const double* xs, double* dst, long dst_chain_stride, double* scratch,
                         int b0, int nblk) {
  const long nn = (long)g.n * g.n;
  // with nblk == 1 the batch index is the chain; dst advances by dst_chain_stride
  const long sdst = (nblk == 1) ? dst_chain_stride : nn;
  double* bufs[2] = {dst, scratch};
  const long strides[2] = {sdst, nn};
  const int per = KRON_MAX_SCALES / g.n;
  const int chunks = (g.ns + per - 1) / per;
  KronArgs<double> a;
  a.nx = g.nx; a.n = g.n; a.batch = g.C * nblk; a.inner_count = nblk;
  a.A = g.ek1;
  a.X = g.ident; a.sX = 0;
  a.rs.v = xs;
  a.rs.so = (long)g.L * g.n;
  a.rs.si = (long)g.ns * g.n;
  a.rs.coef = g.g;
  a.rs.cmul = -g.p.dtau;
  a.rstep = g.n;
  for (int k = 0, t0 = 0; k < chunks; ++k, t0 += per) {
    const int out = (chunks - 1 - k) % 2;     // the last chunk lands in dst
    a.steps = std::min(per, g.ns - t0);
    a.rs.off = (long)(b0 * g.ns + t0) * g.n;
    a.Y = bufs[out]; a.sY = strides[out];
    SCHED_TRY(launch_kron(a, 0, S.s));
    a.X = bufs[out]; a.sX = strides[out];
  }
  return HQ_OK;
}

hq_status combine_tail(Sched& S, Group& g, const double* Tin, long sT, double* Uout, long sUo, double* Dout, long sDo,
                       double* Tout, long sTo);

// (Uout, Dout, Tout) = QR-UDT of op(A) * Uin * diag(Din) combined with Tin.
// A, Uin, Tin advance by the given per-chain strides.
hq_status combine(Sched& S, Group& g, const double* A, long sA, int tA, const double* Uin, long sU, const double* Din,
                  long sD, const double* Tin, long sT, double* Uout, long sUo, double* Dout, long sDo, double* Tout,
                  long sTo) {
  const long nn = (long)g.n * g.n;
  GemmArgs<double> a = sq(g, g.C);
  a.A = A; a.sA = sA; a.tA = tA;
  a.B = Uin; a.sB = sU;
  a.C = g.Z; a.sC = nn;
  a.cs.v = Din; a.cs.so = sD;
  SCHED_TRY(launch_gemm(a, g.tile, S.s));
  return combine_tail(S, g, Tin, sT, Uout, sUo, Dout, sDo, Tout, sTo);
}

// the part of a combine after Z: QR-UDT of Z, Tout = Rt Tin
hq_status combine_tail(Sched& S, Group& g, const double* Tin, long sT, double* Uout, long sUo, double* Dout, long sDo,
                       double* Tout, long sTo) {
  const long nn = (long)g.n * g.n;
  // Q and D go straight into the UDT arrays, which are contiguous per chain;
  // Rt comes back over Z
  if (sUo != nn || sDo != g.n) return fail(S.ctx, HQ_EINVAL, "internal: strided QR output");
  SCHED_TRY(launch_qr(g.Z, g.Rt, Uout, Dout, g.Tq, g.n, g.C, S.s, g.Xw));
  GemmArgs<double> b = sq(g, g.C);
  b.A = g.Z; b.sA = nn;
  b.B = Tin; b.sB = sT;
  b.C = Tout; b.sC = sTo;
  SCHED_TRY(launch_gemm(b, g.tile, S.s));
  return HQ_OK;
}

// G = (I + L R)^-1 and log|det|, L = U_L D_L T_L, R = T_R^T D_R U_R^T
// (identity R when UR == nullptr).  Results in g.Gnew, g.logdet_new.
hq_status merge(Sched& S, Group& g, const double* UL, long sUL, const double* DL, const double* TL, long sTL,
                const double* UR, long sUR, const double* DR, long sDR, const double* TR, long sTR) {
  const long nn = (long)g.n * g.n;
  const int n = g.n;
  if (!UR) {
    SCHED_TRY(launch_dsplit(DL, g.dLbinv, g.dLs, g.sumlog, 0, n, g.C, S.s));
    // right part the identity (a from-scratch recompute): M = Db_L^-1 U_L^T + Ds_L T_L
    // elementwise, and G = Minv U_L^T straight into Gnew
    SCHED_TRY(launch_merge_identity(UL, sUL, TL, sTL, g.dLbinv, g.dLs, g.M, n, g.C, S.s));
    SCHED_TRY(launch_gj(g.M, g.Minv, g.ones, g.dLbinv, g.sumlog, g.logdet_new, n, g.C, S.s, g.Xw));
    GemmArgs<double> c = sq(g, g.C);
    c.A = g.M; c.sA = nn;
    c.B = UL; c.sB = sUL; c.tB = 1;
    c.C = g.Gnew; c.sC = nn;
    SCHED_TRY(launch_gemm(c, g.tile, S.s));
    return HQ_OK;
  }
  // D_R may be strided (right stack); dsplit wants [C][n] contiguous
  if (sDR != n) return fail(S.ctx, HQ_EINVAL, "internal: strided D_R");
  SCHED_TRY(launch_dsplit2(DL, g.dLbinv, g.dLs, DR, g.dRbinv, g.dRs, g.sumlog, n, g.C, S.s));
  const double *rb = g.dRbinv, *rs_ = g.dRs;
  GemmArgs<double> a = sq(g, g.C);                 // M = Db_L^-1 (U_L^T U_R) Db_R^-1
  a.A = UL; a.sA = sUL; a.tA = 1;
  a.B = UR; a.sB = sUR;
  a.C = g.M; a.sC = nn;
  a.rs.v = g.dLbinv; a.rs.so = n;
  a.cs.v = rb; a.cs.so = n;
  SCHED_TRY(launch_gemm(a, g.tile, S.s));
  GemmArgs<double> b = sq(g, g.C);                 // M += Ds_L (T_L T_R^T) Ds_R
  b.A = TL; b.sA = sTL;
  b.B = TR; b.sB = sTR; b.tB = 1;
  b.C = g.M; b.sC = nn;
  b.beta = 1.0;
  b.rs.v = g.dLs; b.rs.so = n;
  b.cs.v = rs_; b.cs.so = n;
  SCHED_TRY(launch_gemm(b, g.tile, S.s));
  // Minv = Db_R^-1 M^-1 Db_L^-1, logdet_new = sumlog + log|det M|
  SCHED_TRY(launch_gj(g.M, g.Minv, rb, g.dLbinv, g.sumlog, g.logdet_new, n, g.C, S.s, g.Xw));
  GemmArgs<double> c = sq(g, g.C);                 // X = Minv U_L^T (Minv over M)
  c.A = g.M; c.sA = nn;
  c.B = UL; c.sB = sUL; c.tB = 1;
  c.C = g.Xm; c.sC = nn;
  SCHED_TRY(launch_gemm(c, g.tile, S.s));
  GemmArgs<double> d = sq(g, g.C);                 // G = U_R X
  d.A = UR; d.sA = sUR;
  d.B = g.Xm; d.sB = nn;
  d.C = g.Gnew; d.sC = nn;
  SCHED_TRY(launch_gemm(d, g.tile, S.s));
  return HQ_OK;
}

// U D T factors of a set of matrices, with per-chain strides
struct Udt { double *U, *D, *T; long sU, sD, sT; };

// The product C_{nb-1} ... C_0 of a group's block products as one UDT per
// chain by pairwise merges, log2(nb) levels deep instead of nb: every block
// is factored at once, then level by level
//   (U_a D_a T_a)(U_b D_b T_b) = (U_a U') D' (T' T_b),  U' D' T' = QR-UDT of D_a (T_a U_b) D_b
// with a the later block of each pair; an unpaired last block passes to the
// next level.  Levels of few enough large matrices (N > 144) spread each QR
// over several workgroups.  Returns pointers to the [C][1] result.
hq_status tree_product(Sched& S, Group& g, const double* blocks, Udt& out) {
  const long nn = (long)g.n * g.n;
  const int n = g.n, C = g.C;
  int cur = 0, m = g.nb;
  // level 0: Z = C_b (in tT[0], where the QR writes its triangular factor over its input)
  if (blocks != g.tT[0]) SCHED_TRY(launch_copy_f64(g.tT[0], blocks, (long)C * g.nb * nn, S.s));
  SCHED_TRY(launch_qr(g.tT[0], g.tQW, g.tU[0], g.tD[0], g.tQT, n, C * g.nb, S.s, g.Xw));
  while (m > 1) {
    const int pairs = m / 2, m2 = (m + 1) / 2, nxt = 1 - cur;
    const double *U = g.tU[cur], *T = g.tT[cur], *D = g.tD[cur];
    // X = diag(D_a) (T_a U_b) diag(D_b), a = 2j + 1, b = 2j; X is [C][pairs]
    GemmArgs<double> x = sq(g, C * pairs);
    x.split = pairs;
    x.A = T + nn; x.sA = 2 * nn; x.sAo = (long)m * nn;
    x.B = U; x.sB = 2 * nn; x.sBo = (long)m * nn;
    x.C = g.tX; x.sC = nn; x.sCo = (long)pairs * nn;
    x.rs.v = D + n; x.rs.so = (long)m * n; x.rs.si = 2L * n;
    x.cs.v = D; x.cs.so = (long)m * n; x.cs.si = 2L * n;
    x.inner_count = pairs;
    SCHED_TRY(launch_gemm(x, pairs > 2 ? g.tile_wide : g.tile, S.s));
    // with m even the next level's D has the layout of the QR's ([C][pairs])
    double* Dq = (m % 2) ? g.tDp : g.tD[nxt];
    SCHED_TRY(launch_qr(g.tX, g.tQW, g.tUp, Dq, g.tQT, n, C * pairs, S.s, g.Xw));
    // U_next = U_a U', T_next = T' T_b, D_next = D'; entries [C][m2]
    GemmArgs<double> u = sq(g, C * pairs);
    u.split = pairs;
    u.A = U + nn; u.sA = 2 * nn; u.sAo = (long)m * nn;
    u.B = g.tUp; u.sB = nn; u.sBo = (long)pairs * nn;
    u.C = g.tU[nxt]; u.sC = nn; u.sCo = (long)m2 * nn;
    GemmArgs<double> t = sq(g, C * pairs);
    t.split = pairs;
    t.A = g.tX; t.sA = nn; t.sAo = (long)pairs * nn;
    t.B = T; t.sB = 2 * nn; t.sBo = (long)m * nn;
    t.C = g.tT[nxt]; t.sC = nn; t.sCo = (long)m2 * nn;
    SCHED_TRY(launch_gemm_pair(u, t, pairs > 2 ? g.tile_wide : g.tile, S.s));   // independent: one launch
    if (m % 2) {                           // D of the pairs, and the unpaired last block, in one launch
      BlockCopies cp;
      auto add = [&](double* dst, long dso, const double* src, long sso, long len) {
        BlockCopy& q = cp.c[cp.k++];
        q.dst = dst; q.dso = dso; q.src = src; q.sso = sso; q.len = len;
        q.outer = C; q.inner = 1;
      };
      add(g.tD[nxt], (long)m2 * n, g.tDp, (long)pairs * n, (long)pairs * n);
      add(g.tU[nxt] + (m2 - 1) * nn, (long)m2 * nn, U + (m - 1) * nn, (long)m * nn, nn);
      add(g.tT[nxt] + (m2 - 1) * nn, (long)m2 * nn, T + (m - 1) * nn, (long)m * nn, nn);
      add(g.tD[nxt] + (long)(m2 - 1) * n, (long)m2 * n, D + (long)(m - 1) * n, (long)m * n, n);
      SCHED_TRY(launch_copy_blocks_multi(cp, S.s));
    }
    cur = nxt;
    m = m2;
  }
  out = {g.tU[cur], g.tD[cur], g.tT[cur], nn, n, nn};
  return HQ_OK;
}

// G and log|det M| of the fields xs from scratch: all block products, the
// left UDT chain over every block, and the merge with an identity right part.
// Leaves the block products in `blocks`, unless `blocks` is the tree's level-0
// buffer, which the pairwise merges factor in place.
hq_status from_scratch(Sched& S, Group& g, const double* xs, double* blocks) {
  const long nn = (long)g.n * g.n;
  // chain stride nb n^2: the layout [C][nb][n][n] also when nb = 1 (with one
  // block per chain the products are written per chain at this stride)
  ST_TRY(block_products(S, g, xs, blocks, (long)g.nb * nn, g.blks, 0, g.nb));
  if (g.tree) {
    Udt l;
    ST_TRY(tree_product(S, g, blocks, l));
    return merge(S, g, l.U, l.sU, l.D, l.T, l.sT, nullptr, 0, nullptr, 0, nullptr, 0);
  }
  SCHED_TRY(launch_identity(g.LU, g.LD, g.LT[0], g.n, g.C, S.s));
  int t = 0;
  for (int b = 0; b < g.nb; ++b) {
    ST_TRY(combine(S, g, blocks + b * nn, (long)g.nb * nn, 0, g.LU, nn, g.LD, g.n, g.LT[t], nn, g.LU, nn, g.LD, g.n,
                   g.LT[1 - t], nn));
    t = 1 - t;
  }
  return merge(S, g, g.LU, nn, g.LD, g.LT[t], nn, nullptr, 0, nullptr, 0, nullptr, 0);
}

// one launch for both products of a wrap: Wt = diag(rs2) (A1 diag(ks1) G diag(cs1)) A2 diag(cs2),
// then G and Wt trade places
template <typename T>
hq_status fused_wrap(Sched& S, Group& g, const T* A1, const T* A2, Scale ks1, Scale cs1, Scale rs2, Scale cs2) {
  WrapArgs<T> w;
  w.n = g.n; w.batch = g.C;
  w.A1 = A1; w.A2 = A2;
  w.Gin = (const T*)g.G; w.Gout = (T*)g.Wt; w.sG = (long)g.n * g.n;
  w.ks1 = ks1; w.cs1 = cs1; w.rs2 = rs2; w.cs2 = cs2;
  SCHED_TRY(launch_wrap_fused(w, S.s));
  std::swap(g.G, g.Wt);
  return HQ_OK;
}

// the same with the Kronecker passes: Wt = (A1 (x) A1) diag(ks1) G diag(cs1),
// G = diag(rs2) Wt (A2 (x) A2) diag(cs2); G stays in place
template <typename T>
hq_status kron_wrap(Sched& S, Group& g, const T* A1, const T* A2, Scale ks1, Scale cs1, Scale rs2, Scale cs2) {
  KronArgs<T> l;
  l.nx = g.nx; l.n = g.n; l.batch = g.C;
  l.A = A1;
  l.X = (const T*)g.G; l.sX = (long)g.n * g.n;
  l.Y = (T*)g.Wt; l.sY = l.sX;
  l.ks = ks1; l.cs = cs1;
  SCHED_TRY(launch_kron(l, 0, S.s));
  KronArgs<T> r = l;
  r.A = A2;
  r.X = (const T*)g.Wt; r.Y = (T*)g.G;
  r.ks = Scale(); r.cs = cs2; r.rs = rs2;
  SCHED_TRY(launch_kron(r, 1, S.s));
  return HQ_OK;
}

// the four Kronecker passes in one launch, G in LDS; G and Wt trade places
template <typename T>
hq_status kron_lds_wrap(Sched& S, Group& g, const T* A1, const T* A2, Scale ks1, Scale cs1, Scale rs2, Scale cs2) {
  KronWrapArgs<T> w;
  w.nx = g.nx; w.batch = g.C;
  w.A1 = A1; w.A2 = A2;
  w.X = (const T*)g.G; w.sX = (long)g.n * g.n;
  w.Y = (T*)g.Wt; w.sY = w.sX;
  w.ks1 = ks1; w.cs1 = cs1; w.rs2 = rs2; w.cs2 = cs2;
  SCHED_TRY(launch_kron_wrap_lds(w, S.s));
  std::swap(g.G, g.Wt);
  return HQ_OK;
}

// G back in G0 at the end of a group's sweep (after an odd number of one-launch wraps)
hq_status settle_g(Sched& S, Group& g) {
  if (g.G == g.G0) return HQ_OK;
  const size_t ts = S.ctx->opt.precision == HQ_PREC_MIXED ? sizeof(float) : sizeof(double);
  SCHED_TRY(launch_copy_u32((uint32_t*)g.G0, (const uint32_t*)g.G, (long)g.C * g.n * g.n * (long)(ts / 4), S.s));
  std::swap(g.G, g.Wt);
  return HQ_OK;
}

hq_status wrap(Sched& S, Group& g, int slice) {
  const long nn = (long)g.n * g.n;
  Scale rs, cs;
  rs.v = g.x; rs.so = (long)g.L * g.n; rs.off = (long)slice * g.n; rs.coef = g.g; rs.cmul = -g.p.dtau;
  cs = rs; cs.cmul = g.p.dtau;
  if (g.wrap_kind == WRAP_KRON_LDS) {
    if (S.ctx->opt.precision == HQ_PREC_MIXED) return kron_lds_wrap<float>(S, g, g.ek1_32, g.ek1inv_32, Scale(), Scale(), rs, cs);
    return kron_lds_wrap<double>(S, g, g.ek1, g.ek1inv, Scale(), Scale(), rs, cs);
  }
  if (g.wrap_kind == WRAP_KRON) {
    if (S.ctx->opt.precision == HQ_PREC_MIXED) return kron_wrap<float>(S, g, g.ek1_32, g.ek1inv_32, Scale(), Scale(), rs, cs);
    return kron_wrap<double>(S, g, g.ek1, g.ek1inv, Scale(), Scale(), rs, cs);
  }
  if (g.wrap_kind == WRAP_FUSED) {
    if (S.ctx->opt.precision == HQ_PREC_MIXED) return fused_wrap<float>(S, g, g.expk32, g.expkinv32, Scale(), Scale(), rs, cs);
    return fused_wrap<double>(S, g, g.expk, g.expkinv, Scale(), Scale(), rs, cs);
  }
  if (S.ctx->opt.precision == HQ_PREC_MIXED) {
    GemmArgs<float> a;
    a.M = a.N = a.K = g.n; a.lda = a.ldb = a.ldc = g.n; a.batch = g.C;
    a.A = g.expk32; a.sA = 0;
    a.B = (const float*)g.G; a.sB = nn;
    a.C = (float*)g.Wt; a.sC = nn;
    SCHED_TRY(launch_gemm(a, g.tile32, S.s));
    GemmArgs<float> b = a;
    b.A = (const float*)g.Wt; b.sA = nn;
    b.B = g.expkinv32; b.sB = 0;
    b.C = (float*)g.G; b.sC = nn;
    b.rs = rs; b.cs = cs;
    SCHED_TRY(launch_gemm(b, g.tile32, S.s));
  } else {
    GemmArgs<double> a = sq(g, g.C);
    a.A = g.expk; a.sA = 0;
    a.B = (const double*)g.G; a.sB = nn;
    a.C = (double*)g.Wt; a.sC = nn;
    SCHED_TRY(launch_gemm(a, g.tile, S.s));
    GemmArgs<double> b = a;
    b.A = (const double*)g.Wt; b.sA = nn;
    b.B = g.expkinv; b.sB = 0;
    b.C = (double*)g.G; b.sC = nn;
    b.rs = rs; b.cs = cs;
    SCHED_TRY(launch_gemm(b, g.tile, S.s));
  }
  return HQ_OK;
}

hq_status local(Sched& S, Group& g, int slice) {
  LocalArgs a;
  a.n = g.n; a.L = g.L; a.slice = slice;
  a.G = g.G; a.x = g.x; a.g = g.g;
  a.dtau = g.p.dtau; a.mass = g.p.mass; a.omega = g.p.omega; a.width = g.p.local_width;
  a.seed = S.ctx->seed; a.chain0 = g.chain0; a.sweep = S.ctx->sweep_counter;
  a.logdet = g.logdet; a.counters = g.counters;
  a.log_margin = g.log_margin[HQ_KIND_LOCAL]; a.log_accept = g.log_accept[HQ_KIND_LOCAL];
  a.replay = replay_of(S.ctx, g, HQ_KIND_LOCAL); a.band = g.band[HQ_KIND_LOCAL]; a.replay_counts = g.replay_counts;
  SCHED_TRY(launch_local(a, S.ctx->opt.precision, g.nt, g.kd, g.C, S.s));
  return HQ_OK;
}

// G <- B_l^-1 G B_l = expK^-1 D_l^-1 G D_l expK (downward sweeps): the inner
// scale D^-1 on G's rows and the column scale D in the first product, then expK
hq_status unwrap(Sched& S, Group& g, int slice) {
  const long nn = (long)g.n * g.n;
  Scale ks, cs;
  ks.v = g.x; ks.so = (long)g.L * g.n; ks.off = (long)slice * g.n; ks.coef = g.g; ks.cmul = g.p.dtau;
  cs = ks; cs.cmul = -g.p.dtau;
  if (g.wrap_kind == WRAP_KRON_LDS) {
    if (S.ctx->opt.precision == HQ_PREC_MIXED) return kron_lds_wrap<float>(S, g, g.ek1inv_32, g.ek1_32, ks, cs, Scale(), Scale());
    return kron_lds_wrap<double>(S, g, g.ek1inv, g.ek1, ks, cs, Scale(), Scale());
  }
  if (g.wrap_kind == WRAP_KRON) {
    if (S.ctx->opt.precision == HQ_PREC_MIXED) return kron_wrap<float>(S, g, g.ek1inv_32, g.ek1_32, ks, cs, Scale(), Scale());
    return kron_wrap<double>(S, g, g.ek1inv, g.ek1, ks, cs, Scale(), Scale());
  }
  if (g.wrap_kind == WRAP_FUSED) {
    if (S.ctx->opt.precision == HQ_PREC_MIXED) return fused_wrap<float>(S, g, g.expkinv32, g.expk32, ks, cs, Scale(), Scale());
    return fused_wrap<double>(S, g, g.expkinv, g.expk, ks, cs, Scale(), Scale());
  }
  if (S.ctx->opt.precision == HQ_PREC_MIXED) {
    GemmArgs<float> a;
    a.M = a.N = a.K = g.n; a.lda = a.ldb = a.ldc = g.n; a.batch = g.C;
    a.A = g.expkinv32; a.sA = 0;
    a.B = (const float*)g.G; a.sB = nn;
    a.C = (float*)g.Wt; a.sC = nn;
    a.ks = ks; a.cs = cs;
    SCHED_TRY(launch_gemm(a, g.tile32, S.s));
    GemmArgs<float> b = a;
    b.A = (const float*)g.Wt; b.sA = nn;
    b.B = g.expk32; b.sB = 0;
    b.C = (float*)g.G; b.sC = nn;
    b.ks = Scale(); b.cs = Scale();
    SCHED_TRY(launch_gemm(b, g.tile32, S.s));
  } else {
    GemmArgs<double> a = sq(g, g.C);
    a.A = g.expkinv; a.sA = 0;
    a.B = (const double*)g.G; a.sB = nn;
    a.C = (double*)g.Wt; a.sC = nn;
    a.ks = ks; a.cs = cs;
    SCHED_TRY(launch_gemm(a, g.tile, S.s));
    GemmArgs<double> b = a;
    b.A = (const double*)g.Wt; b.sA = nn;
    b.B = g.expk; b.sB = 0;
    b.C = (double*)g.G; b.sC = nn;
    b.ks = Scale(); b.cs = Scale();
    SCHED_TRY(launch_gemm(b, g.tile, S.s));
  }
  return HQ_OK;
}

// stack entries, all chains of the group contiguous per entry
Udt left_entry(Group& g, int b) {       // L_b = C_b ... C_0; b = -1: identity
  const long nn = (long)g.n * g.n;
  if (b < 0) return {g.ident, g.ones, g.ident, 0, g.n, 0};
  return {g.SU + (long)b * g.C * nn, g.SD + (long)b * g.C * g.n, g.ST + (long)b * g.C * nn, nn, g.n, nn};
}
Udt right_entry(Group& g, int b) {      // R_b^T with R_b = C_{nb-1} ... C_{b+1}; R_{nb-1} = identity
  const long nn = (long)g.n * g.n;
  return {g.RU + (long)b * g.C * nn, g.RD + (long)b * g.C * g.n, g.RT + (long)b * g.C * nn, nn, g.n, nn};
}

// A combine straight from the fields, for groups whose cached block products
// are read only by stack rebuilds: Z = C_b U_in diag(D_in) (upward) or
// C_b^T U_in diag(D_in) (downward) by the Kronecker chain applied to U_in,
// C_b = B_{(b+1)ns-1} ... B_{b ns}, B_l = diag(v_l) E, and C_b^T = E diag(v_{b ns})
// ... E diag(v_{(b+1)ns-1}) (E symmetric); then the QR-UDT of Z as in combine.
// The block product itself is not formed.
hq_status chain_combine(Sched& S, Group& g, int b, bool down, const Udt& in, const Udt& out) {
  const long nn = (long)g.n * g.n;
  const int per = KRON_MAX_SCALES / g.n;
  const int chunks = (g.ns + per - 1) / per;
  double* bufs[2] = {g.Z, g.blks};           // the last chunk lands in Z
  KronArgs<double> a;
  a.nx = g.nx; a.n = g.n; a.batch = g.C; a.inner_count = 1;
  a.A = g.ek1;
  a.X = in.U; a.sX = in.sU;
  a.rs.v = g.x; a.rs.so = (long)g.L * g.n; a.rs.coef = g.g; a.rs.cmul = -g.p.dtau;
  a.pre = down ? 1 : 0;
  a.rstep = down ? -(long)g.n : (long)g.n;
  for (int k = 0, t0 = 0; k < chunks; ++k, t0 += per) {
    const int o = (chunks - 1 - k) % 2;
    a.steps = std::min(per, g.ns - t0);
    a.rs.off = (long)(down ? b * g.ns + g.ns - 1 - t0 : b * g.ns + t0) * g.n;
    if (k + 1 == chunks) { a.cs.v = in.D; a.cs.so = in.sD; }
    a.Y = bufs[o]; a.sY = nn;
    SCHED_TRY(launch_kron(a, 0, S.s));
    a.X = bufs[o]; a.sX = nn;
  }
  return combine_tail(S, g, in.T, in.sT, out.U, out.sU, out.D, out.sD, out.T, out.sT);
}

// upward stabilisation after block b: C_b from the new fields, L_b = C_b L_{b-1},
// G = (I + L_b R_b)^-1
hq_status stab_up(Sched& S, Group& g, int b) {
  const long nn = (long)g.n * g.n;
  const Udt in = left_entry(g, b - 1), out = left_entry(g, b), r = right_entry(g, b);
  if (g.alternate) {
    ST_TRY(chain_combine(S, g, b, false, in, out));
  } else {
    ST_TRY(block_products(S, g, g.x, g.blk + b * nn, (long)g.nb * nn, g.Z, b, 1));
    ST_TRY(combine(S, g, g.blk + b * nn, (long)g.nb * nn, 0, in.U, in.sU, in.D, in.sD, in.T, in.sT, out.U, out.sU,
                   out.D, out.sD, out.T, out.sT));
  }
  ST_TRY(merge(S, g, out.U, out.sU, out.D, out.T, out.sT, r.U, r.sU, r.D, r.sD, r.T, r.sT));
  SCHED_TRY(launch_stab_finish(g.G, S.ctx->opt.precision, g.Gnew, g.logdet, g.logdet_new, g.drift, g.dpart, g.n,
                               g.C, 1, S.s, g.Gtrk, g.ldtrk));
  return HQ_OK;
}

// downward stabilisation after block b (G unwrapped to slice b*ns - 1):
// C_b from the new fields, R_{b-1}^T = C_b^T R_b^T, G = (I + L_{b-1} R_{b-1})^-1.
// For b = 0 the full product goes to the scratch UDT (LU, LD, LT[0]).
hq_status stab_down(Sched& S, Group& g, int b) {
  const long nn = (long)g.n * g.n;
  const Udt in = right_entry(g, b);
  const Udt out = (b > 0) ? right_entry(g, b - 1) : Udt{g.LU, g.LD, g.LT[0], nn, g.n, nn};
  if (g.alternate) {
    ST_TRY(chain_combine(S, g, b, true, in, out));
  } else {
    ST_TRY(block_products(S, g, g.x, g.blk + b * nn, (long)g.nb * nn, g.Z, b, 1));
    ST_TRY(combine(S, g, g.blk + b * nn, (long)g.nb * nn, 1, in.U, in.sU, in.D, in.sD, in.T, in.sT, out.U, out.sU,
                   out.D, out.sD, out.T, out.sT));
  }
  const Udt l = left_entry(g, b - 1);
  ST_TRY(merge(S, g, l.U, l.sU, l.D, l.T, l.sT, out.U, out.sU, out.D, out.sD, out.T, out.sT));
  SCHED_TRY(launch_stab_finish(g.G, S.ctx->opt.precision, g.Gnew, g.logdet, g.logdet_new, g.drift, g.dpart, g.n,
                               g.C, 1, S.s, g.Gtrk, g.ldtrk));
  return HQ_OK;
}

// every left stack entry from the block products of the current fields (the
// cache is not kept current across sweeps: alternating sweeps combine straight
// from the fields, and accepted block moves or cumulative updates change
// whole columns of x without touching it)
hq_status left_stack(Sched& S, Group& g) {
  const long nn = (long)g.n * g.n;
  ST_TRY(block_products(S, g, g.x, g.blk, (long)g.nb * nn, g.blks, 0, g.nb));
  for (int b = 0; b < g.nb; ++b) {
    const Udt in = left_entry(g, b - 1), out = left_entry(g, b);
    ST_TRY(combine(S, g, g.blk + b * nn, (long)g.nb * nn, 0, in.U, in.sU, in.D, in.sD, in.T, in.sT, out.U, out.sU,
                   out.D, out.sD, out.T, out.sT));
  }
  return HQ_OK;
}

hq_status right_stack(Sched& S, Group& g) {
  const long nn = (long)g.n * g.n;
  ST_TRY(block_products(S, g, g.x, g.blk, (long)g.nb * nn, g.blks, 0, g.nb));
  const long eU = (long)g.C * nn, eD = (long)g.C * g.n;   // one stack entry, all chains
  SCHED_TRY(launch_identity(g.RU + (g.nb - 1) * eU, g.RD + (g.nb - 1) * eD, g.RT + (g.nb - 1) * eU, g.n, g.C, S.s));
  for (int b = g.nb - 2; b >= 0; --b) {
    // R_b^T = C_{b+1}^T R_{b+1}^T
    ST_TRY(combine(S, g, g.blk + (b + 1) * nn, (long)g.nb * nn, 1, g.RU + (b + 1) * eU, nn, g.RD + (b + 1) * eD, g.n,
                   g.RT + (b + 1) * eU, nn, g.RU + b * eU, nn, g.RD + b * eD, g.n, g.RT + b * eU, nn));
  }
  return HQ_OK;
}

hq_status global_moves(Sched& S, Group& g) {
  for (int i = 0; i < g.n; ++i) {
    GlobalArgs a;
    a.n = g.n; a.L = g.L; a.nb = g.nb; a.site = i;
    a.x = g.x; a.xp = g.xp; a.g = g.g;
    a.dtau = g.p.dtau; a.mass = g.p.mass; a.omega = g.p.omega; a.width = g.p.global_width;
    a.seed = S.ctx->seed; a.chain0 = g.chain0; a.sweep = S.ctx->sweep_counter;
    a.shift = g.shift; a.logdet = g.logdet; a.logdet_new = g.logdet_new;
    a.G = g.G; a.precision = S.ctx->opt.precision; a.Gnew = g.Gnew;
    a.counters = g.counters;
    a.log_margin = g.log_margin[HQ_KIND_GLOBAL]; a.log_accept = g.log_accept[HQ_KIND_GLOBAL];
    a.replay = replay_of(S.ctx, g, HQ_KIND_GLOBAL); a.band = g.band[HQ_KIND_GLOBAL]; a.replay_counts = g.replay_counts;
    SCHED_TRY(launch_global_propose(a, g.C, S.s));
    ST_TRY(from_scratch(S, g, g.xp, g.tree ? g.tT[0] : g.blkp));
    SCHED_TRY(launch_global_accept(a, g.C, S.s));
  }
  return HQ_OK;
}

hq_status network_sweep(Sched& S, Group& g) {
  hq_ctx* ctx = S.ctx;
  const long ln = (long)g.L * g.n;
  SCHED_TRY(launch_copy_f64(g.xp, g.x, (long)g.C * ln, S.s));
  SCHED_TRY(launch_fill_f64(g.sum_y, 0.0, (long)g.C * ln, S.s));
  SCHED_TRY(launch_fill_u8(g.nn_acc, 0, (long)g.C * ln, S.s));
  // the steps of the forward schedule: (kind, inner sweep, colour class);
  // a reversed sweep takes them from the last to the first
  struct Step { int block, u, colour; };
  std::vector<Step> steps;
  for (int u = 0; u < g.nu; ++u)
    for (int colour = 0; colour < 16; ++colour) steps.push_back({0, u, colour});
  if (g.cnn) {
    SCHED_TRY(launch_fill_f64(g.sum_yb, 0.0, (long)g.C * g.n, S.s));
    SCHED_TRY(launch_fill_u8(g.acc_b, 0, (long)g.C * g.n, S.s));
    for (int u = 0; u < g.nu; ++u)
      for (int colour = 0; colour < 4; ++colour) steps.push_back({1, u, colour});
  }
  if (ctx->scan) std::reverse(steps.begin(), steps.end());
  for (const Step& st : steps) {
    const int u = st.u, colour = st.colour;
    if (!st.block) {
      NetArgs a;
      a.nx = g.nx; a.n = g.n; a.L = g.L; a.colour = colour;
      a.inner = u; a.nu = g.nu;
      a.xp = g.xp; a.g = g.g;
      a.dtau = g.p.dtau; a.mass = g.p.mass; a.omega = g.p.omega; a.width = g.p.local_width;
      a.seed = ctx->seed; a.chain0 = g.chain0; a.sweep = ctx->sweep_counter;
      a.w = ctx->net; a.activation = ctx->opt.activation; a.chains = g.C;
      a.sum_y = g.sum_y; a.accepted = g.nn_acc; a.counters = g.counters;
      a.log_margin = g.log_margin[HQ_KIND_NN]; a.log_accept = g.log_accept[HQ_KIND_NN];
      a.replay = replay_of(ctx, g, HQ_KIND_NN); a.band = g.band[HQ_KIND_NN]; a.replay_counts = g.replay_counts;
      SCHED_TRY(launch_network_colour(a, g.C, S.s));
    } else {
      CnnArgs a;
      a.nx = g.nx; a.n = g.n; a.L = g.L; a.colour = colour;
      a.inner = u; a.nu = g.nu;
      a.xp = g.xp; a.g = g.g;
      a.dtau = g.p.dtau; a.mass = g.p.mass; a.omega = g.p.omega; a.width = g.p.global_width;
      a.seed = ctx->seed; a.chain0 = g.chain0; a.sweep = ctx->sweep_counter;
      a.w = ctx->cnn; a.chains = g.C;
      a.sum_y = g.sum_yb; a.accepted = g.acc_b;
      a.log_margin = g.log_margin[HQ_KIND_NN_GLOBAL]; a.log_accept = g.log_accept[HQ_KIND_NN_GLOBAL];
      a.replay = replay_of(ctx, g, HQ_KIND_NN_GLOBAL); a.band = g.band[HQ_KIND_NN_GLOBAL];
      a.replay_counts = g.replay_counts;
      SCHED_TRY(launch_cnn_colour(a, g.C, S.s));
    }
  }
  ST_TRY(from_scratch(S, g, g.xp, g.tree ? g.tT[0] : g.blkp));
  CumulativeArgs c;
  c.n = g.n; c.L = g.L; c.nb = g.nb;
  c.x = g.x; c.xp = g.xp; c.logdet = g.logdet; c.logdet_new = g.logdet_new;
  c.G = g.G; c.precision = ctx->opt.precision; c.Gnew = g.Gnew;
  c.sum_y = g.sum_y; c.accepted = g.nn_acc;
  c.sum_yb = g.sum_yb; c.accepted_b = g.acc_b; c.inner = g.nu;
  c.seed = ctx->seed; c.chain0 = g.chain0; c.sweep = ctx->sweep_counter; c.counters = g.counters;
  c.log_margin = g.log_margin[HQ_KIND_CUMULATIVE]; c.log_accept = g.log_accept[HQ_KIND_CUMULATIVE];
  c.replay = replay_of(ctx, g, HQ_KIND_CUMULATIVE); c.band = g.band[HQ_KIND_CUMULATIVE]; c.replay_counts = g.replay_counts;
  c.last_log_pc = g.lastpc;
  SCHED_TRY(launch_cumulative(c, g.C, S.s));
  return HQ_OK;
}

enum { DIR_UP = 0, DIR_DOWN = 1 };

// One sweep of a group.  Upward: wrap and local moves slice by slice, FP64
// stabilisation after every block against the right stack (rebuilt first
// unless the previous downward sweep left it valid); then the block moves.
// Downward (alternating groups, odd sweeps): local moves and unwrap slice by
// slice from the top, stabilisation against the left stack the previous
// upward sweep left behind (or a rebuilt one).
hq_status sweep_group(Sched& S, Group& g, int dir, bool rebuild) {
  if (g.network) {
    ST_TRY(begin_phase(S, PH_NETWORK));
    ST_TRY(network_sweep(S, g));
    return end_phase(S);
  }
  if (!g.alternate || dir == DIR_UP) {
    if (!g.alternate || rebuild) {
      ST_TRY(begin_phase(S, PH_STAB));
      ST_TRY(right_stack(S, g));
      ST_TRY(end_phase(S));
    }
    for (int b = 0; b < g.nb; ++b) {
      for (int k = 0; k < g.ns; ++k) {
        const int slice = b * g.ns + k;
        ST_TRY(begin_phase(S, PH_WRAP));
        ST_TRY(wrap(S, g, slice));
        ST_TRY(end_phase(S));
        ST_TRY(begin_phase(S, PH_LOCAL));
        ST_TRY(local(S, g, slice));
        ST_TRY(end_phase(S));
      }
      ST_TRY(begin_phase(S, PH_STAB));
      ST_TRY(stab_up(S, g, b));
      ST_TRY(end_phase(S));
    }
    if (g.global) {
      ST_TRY(begin_phase(S, PH_GLOBAL));
      ST_TRY(global_moves(S, g));
      ST_TRY(end_phase(S));
    }
    return HQ_OK;
  }
  ST_TRY(begin_phase(S, PH_STAB));
  if (rebuild) ST_TRY(left_stack(S, g));
  const Udt top = right_entry(g, g.nb - 1);
  SCHED_TRY(launch_identity(top.U, top.D, top.T, g.n, g.C, S.s));
  ST_TRY(end_phase(S));
  for (int b = g.nb - 1; b >= 0; --b) {
    for (int k = g.ns - 1; k >= 0; --k) {
      const int slice = b * g.ns + k;
      ST_TRY(begin_phase(S, PH_LOCAL));
      ST_TRY(local(S, g, slice));
      ST_TRY(end_phase(S));
      ST_TRY(begin_phase(S, PH_WRAP));
      ST_TRY(unwrap(S, g, slice));
      ST_TRY(end_phase(S));
    }
    ST_TRY(begin_phase(S, PH_STAB));
    ST_TRY(stab_down(S, g, b));
    ST_TRY(end_phase(S));
  }
  return HQ_OK;
}

hq_status enqueue_group(hq_ctx* ctx, Group& g, hipStream_t s, int dir, bool rebuild) {
  Sched S{ctx, s};
  hq_status st = sweep_group(S, g, dir, rebuild);
  if (st == HQ_OK) st = settle_g(S, g);
  if (st != HQ_OK) {
    if (g.G != g.G0) std::swap(g.G, g.Wt);   // the enqueue failed part-way: keep the buffers' roles
    return st;
  }
  if (ctx->opt.record)                      // replay logs hold for one sweep only
    for (int k : KINDS)
      SCHED_TRY(launch_fill_u8(g.replay[k], 255, (long)g.C * g.kind_slots(k), S.s));
  return HQ_OK;
}

// One sweep of every group.  Groups share nothing but the read-only network
// and the sweep counter, so with more than one group each runs on its own
// stream (a parallel branch once captured) and the counter is advanced after
// the join.  The profiling mode keeps one stream so that its events time
// each phase alone.
hq_status enqueue_sweep(hq_ctx* ctx, int dir, bool rebuild) {
  const bool fork = !ctx->profiling && ctx->groups.size() > 1;
  if (!fork) {
    for (Group& g : ctx->groups) ST_TRY(enqueue_group(ctx, g, ctx->stream, dir, rebuild));
  } else {
    HQ_TRY(hipEventRecord(ctx->fork, ctx->stream));
    // the branch with the most work per chain (N^3 L) first, so that the
    // longest path starts first; the small groups fill in beside it
    std::vector<size_t> order(ctx->groups.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      const Group &ga = ctx->groups[a], &gb = ctx->groups[b];
      return (double)ga.n * ga.n * ga.n * ga.L > (double)gb.n * gb.n * gb.n * gb.L;
    });
    for (size_t k : order) {
      HQ_TRY(hipStreamWaitEvent(ctx->side[k], ctx->fork, 0));
      ST_TRY(enqueue_group(ctx, ctx->groups[k], ctx->side[k], dir, rebuild));
      HQ_TRY(hipEventRecord(ctx->join[k], ctx->side[k]));
    }
    for (size_t k = 0; k < ctx->groups.size(); ++k) HQ_TRY(hipStreamWaitEvent(ctx->stream, ctx->join[k], 0));
  }
  Sched S{ctx, ctx->stream};
  SCHED_TRY(launch_add_i64(ctx->sweep_counter, 1, S.s));
  return HQ_OK;
}

// GEMM autotuner: time one batched product of the group's shape with every
// tile that fits (operands: expK and scratch buffers, which hold nothing yet)
// and keep the fastest, for FP64 and for the precision of the wraps.
hq_status autotune(hq_ctx* ctx) {
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  HQ_TRY(hipEventCreate(&e0));
  HQ_TRY(hipEventCreate(&e1));
  const int cands[] = {TILE_64x64, TILE_32x32, TILE_48x48, TILE_FK_32x32, TILE_FK_48x48, TILE_FK_64x64,
                       TILE_FK_32x64, TILE_PF_48x48, TILE_PF_64x64, TILE_PF_32x32,
                       TILE_DX_48x48, TILE_DX_32x32, TILE_DX_64x64};
  hq_status st = HQ_OK;
  for (Group& g : ctx->groups) {
    const long nn = (long)g.n * g.n;
    // prec 0: FP64 products of the group's batch; 1: the wraps' products in
    // FP32; 2: FP64 products of every block of every chain at once (block
    // products from scratch), which favour other tiles
    for (int prec = 0; prec < 3 && st == HQ_OK; ++prec) {
      if (prec == 1 && ctx->opt.precision != HQ_PREC_MIXED) continue;
      if (prec == 2 && (g.nb < 3 || !g.tree)) { g.tile_wide = g.tile; continue; }   // only recomputes use it
      double best = 1e30;
      int bt = TILE_64x64;
      for (int tile : cands) {
        if (!gemm_tile_fits(tile, g.n, prec == 1)) continue;
        hipError_t e = hipSuccess;
        auto run = [&]() {
          if (prec == 2) {
            GemmArgs<double> a = sq(g, g.C * g.nb);
            a.A = g.expk; a.sA = 0;
            a.B = g.blkp; a.sB = nn;
            a.C = g.blk; a.sC = nn;
            return launch_gemm(a, tile, s);
          }
          if (prec) {
            GemmArgs<float> a;
            a.M = a.N = a.K = g.n; a.lda = a.ldb = a.ldc = g.n; a.batch = g.C;
            a.A = g.expk32; a.sA = 0;
            a.B = (const float*)g.Wt; a.sB = nn;
            a.C = (float*)g.G; a.sC = nn;
            return launch_gemm(a, tile, s);
          }
          GemmArgs<double> a = sq(g, g.C);
          a.A = g.expk; a.sA = 0;
          a.B = g.blks; a.sB = nn;
          a.C = g.Z; a.sC = nn;
          return launch_gemm(a, tile, s);
        };
        e = run();
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int k = 0; k < 3 && e == hipSuccess; ++k) e = run();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = fail(ctx, HQ_EDEVICE, "autotune: %s", hipGetErrorString(e));
          break;
        }
        const double us = 1e3 * ms / 3.0;
        if (us < best) { best = us; bt = tile; }
      }
      if (prec == 1) { g.tile32 = bt; g.tile32_us = best; }
      else if (prec == 0) { g.tile = bt; g.tile_us = best; }
      else g.tile_wide = bt;
    }
    if (ctx->opt.precision != HQ_PREC_MIXED) { g.tile32 = g.tile; g.tile32_us = g.tile_us; }
    // the wrap: two tiled products, both products in one launch, or the two
    // Kronecker passes (G and Wt hold nothing yet)
    g.wrap_kind = WRAP_TWO;
    g.wrap_us = 2.0 * g.tile32_us;
    const bool mixed = ctx->opt.precision == HQ_PREC_MIXED;
    for (int kind : {WRAP_FUSED, WRAP_KRON, WRAP_KRON_LDS}) {
      if (st != HQ_OK) break;
      if (kind == WRAP_FUSED && !wrap_fused_supported(g.n, mixed)) continue;
      if (kind == WRAP_KRON_LDS && !kron_wrap_lds_supported(g.nx, mixed)) continue;
      auto run = [&]() -> hipError_t {
        if (kind == WRAP_KRON_LDS) {
          if (mixed) {
            KronWrapArgs<float> k;
            k.nx = g.nx; k.batch = g.C; k.A1 = g.ek1_32; k.A2 = g.ek1inv_32;
            k.X = (const float*)g.G; k.sX = nn; k.Y = (float*)g.Wt; k.sY = nn;
            return launch_kron_wrap_lds(k, s);
          }
          KronWrapArgs<double> k;
          k.nx = g.nx; k.batch = g.C; k.A1 = g.ek1; k.A2 = g.ek1inv;
          k.X = (const double*)g.G; k.sX = nn; k.Y = (double*)g.Wt; k.sY = nn;
          return launch_kron_wrap_lds(k, s);
        }
        if (kind == WRAP_KRON) {
          if (mixed) {
            KronArgs<float> k;
            k.nx = g.nx; k.n = g.n; k.batch = g.C; k.A = g.ek1_32;
            k.X = (const float*)g.G; k.sX = nn; k.Y = (float*)g.Wt; k.sY = nn;
            hipError_t e = launch_kron(k, 0, s);
            k.X = (const float*)g.Wt; k.Y = (float*)g.G;
            return e != hipSuccess ? e : launch_kron(k, 1, s);
          }
          KronArgs<double> k;
          k.nx = g.nx; k.n = g.n; k.batch = g.C; k.A = g.ek1;
          k.X = (const double*)g.G; k.sX = nn; k.Y = (double*)g.Wt; k.sY = nn;
          hipError_t e = launch_kron(k, 0, s);
          k.X = (const double*)g.Wt; k.Y = (double*)g.G;
          return e != hipSuccess ? e : launch_kron(k, 1, s);
        }
        if (mixed) {
          WrapArgs<float> w;
          w.n = g.n; w.batch = g.C; w.A1 = g.expk32; w.A2 = g.expkinv32;
          w.Gin = (const float*)g.G; w.Gout = (float*)g.Wt; w.sG = nn;
          return launch_wrap_fused(w, s);
        }
        WrapArgs<double> w;
        w.n = g.n; w.batch = g.C; w.A1 = g.expk; w.A2 = g.expkinv;
        w.Gin = (const double*)g.G; w.Gout = (double*)g.Wt; w.sG = nn;
        return launch_wrap_fused(w, s);
      };
      hipError_t e = run();
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int k = 0; k < 3 && e == hipSuccess; ++k) e = run();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = fail(ctx, HQ_EDEVICE, "autotune: %s", hipGetErrorString(e));
      } else if (1e3 * ms / 3.0 < g.wrap_us) {
        g.wrap_kind = kind;
        g.wrap_us = 1e3 * ms / 3.0;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// The local-move block size, when the caller left it to the library: one
// slice of local moves (slice 0 of the first sweep, the draws the sweep will
// make) timed with each block size the group's lattice supports, on copies
// of G, the fields and the log determinants, so that the chains' state is
// untouched; the faster is kept (32 only when more than 5% faster).
hq_status tune_delay(hq_ctx* ctx) {
  if (ctx->opt.delay) return HQ_OK;
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  HQ_TRY(hipEventCreate(&e0));
  HQ_TRY(hipEventCreate(&e1));
  hq_status st = HQ_OK;
  for (Group& g : ctx->groups) {
    if (g.network || st != HQ_OK) continue;       // network groups make no local-move launches
    const long nn = (long)g.n * g.n;
    const size_t gbytes = (size_t)g.C * nn * (ctx->opt.precision == HQ_PREC_MIXED ? 4 : 8);
    double best = 1e30;
    int bestk = g.kd;
    for (int kd : {16, 32}) {
      if (!local_supported(g.n, ctx->opt.precision, g.nt, kd)) continue;
      LocalArgs a;
      a.n = g.n; a.L = g.L; a.slice = 0;
      a.G = g.Wt; a.x = g.xp; a.g = g.g;
      a.dtau = g.p.dtau; a.mass = g.p.mass; a.omega = g.p.omega; a.width = g.p.local_width;
      a.seed = ctx->seed; a.chain0 = g.chain0; a.sweep = ctx->sweep_counter;
      a.logdet = g.logdet_new; a.counters = g.tune_cnt;
      float ms = 0.f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {   // the first is a warm-up
        e = hipMemcpyAsync(g.Wt, g.G, gbytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(g.xp, g.x, (size_t)g.C * g.L * g.n * sizeof(double), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(g.logdet_new, g.logdet, g.C * sizeof(double), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && rep > 0) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_local(a, ctx->opt.precision, g.nt, kd, g.C, s);
        if (e == hipSuccess && rep > 0) e = hipEventRecord(e1, s);
        if (e == hipSuccess && rep > 0) e = hipEventSynchronize(e1);
        float m = 0.f;
        if (e == hipSuccess && rep > 0) e = hipEventElapsedTime(&m, e0, e1);
        ms += m;
      }
      if (e != hipSuccess) {
        st = fail(ctx, HQ_EDEVICE, "local block tuning: %s", hipGetErrorString(e));
        break;
      }
      const double us = 1e3 * ms / 2.0;
      // 16 (timed first) stays unless 32 is clearly faster: close timings
      // would otherwise pick either from one context to the next
      if (best == 1e30 || us < 0.95 * best) {
        best = us;
        bestk = kd;
      }
    }
    if (st == HQ_OK && best < 1e30) {
      g.kd = bestk;
      g.local_us = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

hq_status recompute_all(hq_ctx* ctx) {
  Sched S{ctx, ctx->stream};
  for (Group& g : ctx->groups) {
    ST_TRY(from_scratch(S, g, g.x, g.blk));
    SCHED_TRY(launch_stab_finish(g.G, ctx->opt.precision, g.Gnew, g.logdet, g.logdet_new, g.drift, g.dpart, g.n, g.C, 0,
                                 S.s));
  }
  return HQ_OK;
}

hq_status check_ctx(hq_ctx* ctx) {
  if (!ctx) return HQ_EINVAL;
  if (ctx->broken) return HQ_ESTATE;
  return HQ_OK;
}

hq_status sync(hq_ctx* ctx) {
  HQ_TRY(hipStreamSynchronize(ctx->stream));
  return HQ_OK;
}

hq_status collect_profile(hq_ctx* ctx) {
  if (ctx->pending.empty()) return HQ_OK;
  ST_TRY(sync(ctx));
  for (size_t k = 0; k < ctx->pending.size(); ++k) {
    float ms = 0.f;
    HQ_TRY(hipEventElapsedTime(&ms, ctx->pending[k].first, ctx->pending[k].second));
    ctx->phases[ctx->pending_phase[k]].ms += ms;
    ctx->phases[ctx->pending_phase[k]].launches += 1;
    ctx->event_pool.push_back(ctx->pending[k].first);
    ctx->event_pool.push_back(ctx->pending[k].second);
  }
  ctx->pending.clear();
  ctx->pending_phase.clear();
  return HQ_OK;
}

Group* find_chain(hq_ctx* ctx, int chain, int& local) {
  for (Group& g : ctx->groups)
    if (chain >= g.chain0 && chain < g.chain0 + g.C) {
      local = chain - g.chain0;
      return &g;
    }
  return nullptr;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

size_t hq_workspace_bytes(const hq_group* groups, int32_t n_groups, const hq_options* opt) {
  if (!groups || n_groups < 1 || !opt) return 0;
  if (opt->precision != HQ_PREC_FP64 && opt->precision != HQ_PREC_MIXED) return 0;
  std::vector<Group> gs;
  std::string why;
  if (!build_groups(groups, n_groups, *opt, gs, why)) return 0;
  return layout(nullptr, gs, nullptr, *opt);
}

namespace {
// the reason of the last failed hq_create / hq_create_static of this thread
thread_local std::string create_error;

hq_status create_fail(hq_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  create_error = buf;
  return st;
}

// fixed tiles and wrap form for a context created without timing runs
void untuned_choices(hq_ctx* ctx) {
  for (Group& g : ctx->groups) {
    g.tile = g.tile32 = g.tile_wide = TILE_64x64;
    g.tile_us = g.tile32_us = 0.0;
    g.wrap_kind = WRAP_KRON;
    g.wrap_us = 0.0;
  }
}

hq_status create_ctx(const hq_group* groups, int32_t n_groups, const hq_options* opt, uint64_t seed, void* workspace,
                     size_t workspace_bytes, void* stream, bool tune, int static_device, hq_ctx** out);
}  // namespace

hq_status hq_create(const hq_group* groups, int32_t n_groups, const hq_options* opt, uint64_t seed, void* workspace,
                    size_t workspace_bytes, void* stream, hq_ctx** out) {
  return create_ctx(groups, n_groups, opt, seed, workspace, workspace_bytes, stream, true, -1, out);
}

// ---------------------------------------------------------------------------
// The workspace of hq_create_static: a file-scope device array.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel or a copy: it is a host-side stand-in
// there.  Its device address, from hipGetSymbolAddress with the device
// current, is kept per device and used instead.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[HQ_STATIC_WORKSPACE_BYTES];

namespace {
std::mutex static_mu;
std::vector<void*> static_ptr;           // device address of `scratch`, per device (null: not looked up)
std::vector<char> static_busy;           // a static context is alive on the device
}  // namespace

hq_status hq_create_static(const hq_group* groups, int32_t n_groups, const hq_options* opt, uint64_t seed,
                           void* stream, hq_ctx** out) {
  if (!out) return create_fail(HQ_EINVAL, "out is null");
  *out = nullptr;
  if (!groups || n_groups != 1 || !opt || !stream)
    return create_fail(HQ_EINVAL, "hq_create_static takes one group, options and a stream");
  const size_t need = hq_workspace_bytes(groups, n_groups, opt);
  if (need == 0) return create_fail(HQ_EINVAL, "invalid group or options");
  if (need + 256 > (size_t)HQ_STATIC_WORKSPACE_BYTES)
    return create_fail(HQ_ENOMEM, "the group needs %zu bytes of workspace; the static workspace holds %zu",
                       need + 256, (size_t)HQ_STATIC_WORKSPACE_BYTES);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0) return create_fail(HQ_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(static_mu);
    if ((int)static_ptr.size() <= dev) {
      static_ptr.resize(dev + 1, nullptr);
      static_busy.resize(dev + 1, 0);
    }
    if (static_busy[dev]) return create_fail(HQ_ESTATE, "a static context is already alive on device %d", dev);
    if (!static_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return create_fail(HQ_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      static_ptr[dev] = ptr;
    }
    base = static_ptr[dev];
    static_busy[dev] = 1;
  }
  const hq_status st = create_ctx(groups, n_groups, opt, seed, base, (size_t)HQ_STATIC_WORKSPACE_BYTES, stream,
                                  false, dev, out);
  if (!*out) {                           // nothing was created: the array is free again
    std::lock_guard<std::mutex> lk(static_mu);
    static_busy[dev] = 0;
  }
  return st;
}

namespace {
hq_status create_ctx(const hq_group* groups, int32_t n_groups, const hq_options* opt, uint64_t seed, void* workspace,
                     size_t workspace_bytes, void* stream, bool tune, int static_device, hq_ctx** out) {
  if (!out) return create_fail(HQ_EINVAL, "out is null");
  *out = nullptr;
  if (!groups || n_groups < 1 || !opt || !workspace || !stream)
    return create_fail(HQ_EINVAL, "null groups, options, workspace or stream");
  if (opt->precision != HQ_PREC_FP64 && opt->precision != HQ_PREC_MIXED)
    return create_fail(HQ_EINVAL, "unknown precision");
  if (opt->delay != 0 && opt->delay != 8 && opt->delay != 16 && opt->delay != 32)
    return create_fail(HQ_EINVAL, "delay must be 0, 8, 16 or 32");
  if (opt->activation != 0 && opt->activation != 1) return create_fail(HQ_EINVAL, "unknown activation");
  hq_ctx* ctx = new hq_ctx();
  ctx->opt = *opt;
  ctx->seed = seed;
  ctx->stream = (hipStream_t)stream;
  std::string why;
  if (!build_groups(groups, n_groups, *opt, ctx->groups, why)) {
    delete ctx;
    return create_fail(HQ_EINVAL, "%s", why.c_str());
  }
  const size_t need = layout(nullptr, ctx->groups, nullptr, *opt);
  if (workspace_bytes < need) {
    delete ctx;
    return create_fail(HQ_ENOMEM, "the workspace holds %zu bytes; %zu are needed", workspace_bytes, need);
  }
  ctx->static_device = static_device;
  ctx->ws = workspace;
  ctx->ws_bytes = workspace_bytes;
  // align the base to 256 bytes
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  layout(ctx, ctx->groups, base, *opt);
  for (int k = 0; k < N_PHASES; ++k) ctx->phases.push_back({kPhaseNames[k], 0.0, 0});
  for (const Group& g : ctx->groups) {
    ctx->n_chains += g.C;
    if (g.network) ctx->any_network = true;
  }
  *out = ctx;

  HQ_TRY(prepare_local());
  HQ_TRY(prepare_gemm());
  if (ctx->groups.size() > 1) {
    HQ_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    for (size_t k = 0; k < ctx->groups.size(); ++k) {
      hipStream_t side = nullptr;
      hipEvent_t ev = nullptr;
      HQ_TRY(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
      ctx->side.push_back(side);
      HQ_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      ctx->join.push_back(ev);
    }
  }
  hipStream_t s = ctx->stream;
  // host-side model set-up and initial state
  for (Group& g : ctx->groups) {
    const int n = g.n, L = g.L, C = g.C;
    std::vector<double> ek, eki, id((size_t)n * n, 0.0), ones((size_t)C * n, 1.0);
    exp_hopping(g.p, -1.0, ek);
    exp_hopping(g.p, +1.0, eki);
    for (int i = 0; i < n; ++i) id[(size_t)i * n + i] = 1.0;
    std::vector<float> ek32(ek.begin(), ek.end()), eki32(eki.begin(), eki.end());
    std::vector<double> e1, e1i;
    exp_hopping_1d(g.p, -1.0, e1);
    exp_hopping_1d(g.p, +1.0, e1i);
    std::vector<float> e1_32(e1.begin(), e1.end()), e1i_32(e1i.begin(), e1i.end());
    std::vector<double> x((size_t)C * L * n), gc((size_t)C);
    for (int c = 0; c < C; ++c) {
      const uint64_t chain = (uint64_t)(g.chain0 + c);
      if (g.p.g_hi > g.p.g_lo) {
        const Philox4 r = philox4x64_10(chain, 0, 0, KIND_COUPLING, seed, 0);
        gc[c] = g.p.g_lo + (g.p.g_hi - g.p.g_lo) * u53(r.w[0]);
      } else {
        gc[c] = g.p.g;
      }
      for (int l = 0; l < L; ++l)
        for (int i = 0; i < n; ++i) {
          const Philox4 r = philox4x64_10(chain, 0, (uint64_t)(l * n + i), KIND_INIT, seed, 0);
          const double u0 = u53(r.w[0]), u1 = u53(r.w[1]);
          x[((size_t)c * L + l) * n + i] = std::sqrt(-2.0 * std::log(1.0 - u0)) * std::cos(2.0 * M_PI * u1);
        }
    }
    HQ_TRY(hipMemcpyAsync(g.expk, ek.data(), ek.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.expkinv, eki.data(), eki.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.expk32, ek32.data(), ek32.size() * 4, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.expkinv32, eki32.data(), eki32.size() * 4, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.ek1, e1.data(), e1.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.ek1inv, e1i.data(), e1i.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.ek1_32, e1_32.data(), e1_32.size() * 4, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.ek1inv_32, e1i_32.data(), e1i_32.size() * 4, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.ident, id.data(), id.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.ones, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.x, x.data(), x.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipMemcpyAsync(g.g, gc.data(), gc.size() * 8, hipMemcpyHostToDevice, s));
    HQ_TRY(hipStreamSynchronize(s));   // host vectors die at the end of this iteration
    HQ_TRY(launch_fill_i64(g.counters, 0, (long)C * N_COUNTERS, s));
    HQ_TRY(launch_fill_i64(g.replay_counts, 0, (long)C * 2, s));
    HQ_TRY(launch_fill_f64(g.drift, 0.0, (long)C * 5, s));
    HQ_TRY(launch_fill_f64(g.lastpc, 0.0, (long)C * 2, s));
    HQ_TRY(launch_fill_i64((int64_t*)g.flags, 0, ((long)C * sizeof(int) + 7) / 8, s));
    for (int k : KINDS) {
      HQ_TRY(launch_fill_u8(g.replay[k], 255, (long)C * g.kind_slots(k), s));
      if (opt->record) {                 // the workspace may hold an earlier context's data
        HQ_TRY(launch_fill_u8(g.log_accept[k], 0, (long)C * g.kind_slots(k), s));
        HQ_TRY(launch_fill_u8((uint8_t*)g.log_margin[k], 0, (long)C * g.kind_slots(k) * (long)sizeof(float), s));
      }
    }
    if (opt->record) {
      HQ_TRY(launch_fill_f64(g.Gtrk, 0.0, (long)C * n * n, s));
      HQ_TRY(launch_fill_f64(g.ldtrk, 0.0, (long)C, s));
    }
  }
  HQ_TRY(launch_fill_i64(ctx->sweep_counter, 0, 1, s));
  if (tune) {
    ST_TRY(autotune(ctx));
  } else {
    untuned_choices(ctx);
  }
  hq_status st = recompute_all(ctx);
  if (st != HQ_OK) return st;
  if (tune) ST_TRY(tune_delay(ctx));
  return sync(ctx);
}
}  // namespace

hq_status hq_set_fields(hq_ctx* ctx, int32_t chain, const double* x_host, int64_t n) {
  ST_TRY(check_ctx(ctx));
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || !x_host || n != (int64_t)g->L * g->n) return fail(ctx, HQ_EINVAL, "bad chain or field count");
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(x_host[k])) return fail(ctx, HQ_EINVAL, "non-finite field");
  ctx->left_valid = ctx->right_valid = false;
  HQ_TRY(hipMemcpyAsync(g->x + (long)lc * n, x_host, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  Sched S{ctx, ctx->stream};
  ST_TRY(from_scratch(S, *g, g->x, g->blk));
  SCHED_TRY(launch_stab_finish(g->G, ctx->opt.precision, g->Gnew, g->logdet, g->logdet_new, g->drift, g->dpart, g->n, g->C, 0,
                               ctx->stream));
  return sync(ctx);
}

hq_status hq_set_network(hq_ctx* ctx, const float* w, int64_t n) {
  ST_TRY(check_ctx(ctx));
  if (!w || n != 7169) return fail(ctx, HQ_EINVAL, "network needs 7169 weights");
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(w[k])) return fail(ctx, HQ_EINVAL, "non-finite weight");
  HQ_TRY(hipMemcpyAsync(ctx->net, w, n * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  ctx->net_loaded = true;
  return sync(ctx);
}

hq_status hq_set_block_network(hq_ctx* ctx, const float* w, int64_t n, int32_t L) {
  ST_TRY(check_ctx(ctx));
  if (!w || L < 2 || L % 2 || L > ctx->cnn_max_L || n != 64L * L + 117)
    return fail(ctx, HQ_EINVAL, "block-move network: %lld weights for L = %d (needs 64 L + 117, L even, and a "
                "network group with block moves of that L)", (long long)n, L);
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(w[k])) return fail(ctx, HQ_EINVAL, "non-finite weight");
  HQ_TRY(hipMemcpyAsync(ctx->cnn, w, n * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  ctx->cnn_L = L;
  return sync(ctx);
}

hq_status hq_sweep(hq_ctx* ctx, int32_t n_sweeps) {
  ST_TRY(check_ctx(ctx));
  if (n_sweeps < 0) return fail(ctx, HQ_EINVAL, "n_sweeps < 0");
  for (const Group& g : ctx->groups) {
    if (g.network && !ctx->net_loaded) return fail(ctx, HQ_EINVAL, "network proposals need hq_set_network first");
    if (g.cnn && ctx->cnn_L != g.L)
      return fail(ctx, HQ_EINVAL, "network block moves need hq_set_block_network for L = %d first", g.L);
  }
  for (int k = 0; k < n_sweeps; ++k) {
    const int dir = (ctx->sweep_index % 2 == 1) ? DIR_DOWN : DIR_UP;
    const bool rebuild = (dir == DIR_UP) ? !ctx->right_valid : !ctx->left_valid;
    // network sweeps visit their schedule forward or in reverse, one draw per
    // sweep shared by the chains (Philox kind 7 at chain 0, slot 0)
    ctx->scan = 0;
    if (ctx->any_network) {
      const Philox4 r = philox4x64_10(0, (uint64_t)ctx->sweep_index, 0, KIND_SCAN, ctx->seed, 0);
      ctx->scan = u53(r.w[0]) >= 0.5 ? 1 : 0;
    }
    if (ctx->profiling) {
      ST_TRY(enqueue_sweep(ctx, dir, rebuild));
    } else {
      hipGraphExec_t& ex = ctx->exec[dir][rebuild ? 1 : 0][ctx->scan];
      if (!ex) {
        HQ_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        hq_status st = enqueue_sweep(ctx, dir, rebuild);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
        if (st != HQ_OK) {
          if (graph) (void)hipGraphDestroy(graph);   // the partial capture is not kept
          return st;
        }
        if (e != hipSuccess) return fail(ctx, HQ_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        ctx->graph[dir][rebuild ? 1 : 0][ctx->scan] = graph;
        HQ_TRY(hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0));
      }
      HQ_TRY(hipGraphLaunch(ex, ctx->stream));
    }
    ctx->sweep_index += 1;
    // an upward sweep leaves every left stack entry current, a downward one every right entry
    ctx->left_valid = (dir == DIR_UP);
    ctx->right_valid = (dir == DIR_DOWN);
  }
  if (ctx->profiling) return collect_profile(ctx);
  return HQ_OK;
}

hq_status hq_recompute(hq_ctx* ctx) {
  ST_TRY(check_ctx(ctx));
  ctx->left_valid = ctx->right_valid = false;
  ST_TRY(recompute_all(ctx));
  return sync(ctx);
}

hq_status hq_read_green(hq_ctx* ctx, int32_t chain, double* out, int64_t n) {
  ST_TRY(check_ctx(ctx));
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || !out || n != (int64_t)g->n * g->n) return fail(ctx, HQ_EINVAL, "bad chain or size");
  ST_TRY(sync(ctx));
  if (ctx->opt.precision == HQ_PREC_MIXED) {
    std::vector<float> tmp((size_t)n);
    HQ_TRY(hipMemcpy(tmp.data(), (float*)g->G + (long)lc * n, n * sizeof(float), hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < n; ++k) out[k] = tmp[k];
  } else {
    HQ_TRY(hipMemcpy(out, (double*)g->G + (long)lc * n, n * sizeof(double), hipMemcpyDeviceToHost));
  }
  return HQ_OK;
}

hq_status hq_read_green_tracked(hq_ctx* ctx, int32_t chain, double* out, int64_t n, double* logdet) {
  ST_TRY(check_ctx(ctx));
  if (!ctx->opt.record) return fail(ctx, HQ_EINVAL, "the tracked state is only kept with options.record = 1");
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || !out || !logdet || n != (int64_t)g->n * g->n) return fail(ctx, HQ_EINVAL, "bad chain or size");
  ST_TRY(sync(ctx));
  HQ_TRY(hipMemcpy(out, g->Gtrk + (long)lc * n, n * sizeof(double), hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(logdet, g->ldtrk + lc, sizeof(double), hipMemcpyDeviceToHost));
  return HQ_OK;
}

hq_status hq_read_fields(hq_ctx* ctx, int32_t chain, double* out, int64_t n) {
  ST_TRY(check_ctx(ctx));
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || !out || n != (int64_t)g->L * g->n) return fail(ctx, HQ_EINVAL, "bad chain or size");
  ST_TRY(sync(ctx));
  HQ_TRY(hipMemcpy(out, g->x + (long)lc * n, n * sizeof(double), hipMemcpyDeviceToHost));
  return HQ_OK;
}

hq_status hq_read_stats(hq_ctx* ctx, int32_t chain, hq_stats* out) {
  ST_TRY(check_ctx(ctx));
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || !out) return fail(ctx, HQ_EINVAL, "bad chain");
  ObsArgs a;                                // this chain only
  const long nn = (long)g->n * g->n;
  const size_t gsz = ctx->opt.precision == HQ_PREC_MIXED ? sizeof(float) : sizeof(double);
  a.n = g->n; a.L = g->L; a.nx = g->nx;
  a.G = (const char*)g->G + lc * nn * gsz; a.precision = ctx->opt.precision; a.x = g->x + (long)lc * g->L * g->n;
  a.out = g->obs + lc * 5; a.flags = g->flags + lc; a.logdet = g->logdet + lc;
  HQ_TRY(launch_observables(a, 1, ctx->stream));
  ST_TRY(sync(ctx));
  double ld = 0, gg = 0, dr[5], ob[5];
  int64_t cnt[N_COUNTERS], rc[2];
  int fl = 0;
  HQ_TRY(hipMemcpy(&ld, g->logdet + lc, 8, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(&gg, g->g + lc, 8, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(dr, g->drift + lc * 5, sizeof dr, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(ob, g->obs + lc * 5, sizeof ob, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(cnt, g->counters + (long)lc * N_COUNTERS, sizeof cnt, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(rc, g->replay_counts + 2 * lc, sizeof rc, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(&fl, g->flags + lc, sizeof fl, hipMemcpyDeviceToHost));
  double pc[2];
  HQ_TRY(hipMemcpy(pc, g->lastpc + 2 * lc, sizeof pc, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->logdet = ld;
  out->g = gg;
  out->local_proposals = cnt[CNT_LOCAL_P]; out->local_accepts = cnt[CNT_LOCAL_A];
  out->global_proposals = cnt[CNT_GLOBAL_P]; out->global_accepts = cnt[CNT_GLOBAL_A];
  out->nn_proposals = cnt[CNT_NN_P]; out->nn_accepts = cnt[CNT_NN_A];
  out->cumulative_proposals = cnt[CNT_CUM_P]; out->cumulative_accepts = cnt[CNT_CUM_A];
  out->max_drift_green = dr[0]; out->max_drift_logdet = dr[1]; out->last_drift_green = dr[2];
  out->density = ob[0]; out->double_occupancy = ob[1]; out->s_cdw = ob[2]; out->x_mean = ob[3]; out->x2_mean = ob[4];
  out->replay_overrides = rc[0]; out->replay_mismatches = rc[1];
  out->last_log_pc = pc[0]; out->last_sum_y = pc[1];
  out->n = g->n; out->L = g->L;
  out->flags = fl | (dr[4] != 0.0 ? 1 : 0);
  if (out->flags & 1) return fail(ctx, HQ_ENUMERIC, "non-finite G or log det in chain %d", chain);
  return HQ_OK;
}

hq_status hq_read_observables(hq_ctx* ctx, double* out, int64_t n) {
  ST_TRY(check_ctx(ctx));
  if (!out || n != 5L * ctx->n_chains)
    return fail(ctx, HQ_EINVAL, "observables: out must hold 5 values for each of the %d chains", ctx->n_chains);
  for (Group& g : ctx->groups) {
    ObsArgs a;                              // every chain of the group
    a.n = g.n; a.L = g.L; a.nx = g.nx;
    a.G = g.G; a.precision = ctx->opt.precision; a.x = g.x;
    a.out = g.obs; a.flags = g.flags; a.logdet = g.logdet;
    HQ_TRY(launch_observables(a, g.C, ctx->stream));
  }
  ST_TRY(sync(ctx));
  long off = 0;
  int bad = -1;
  for (Group& g : ctx->groups) {
    HQ_TRY(hipMemcpy(out + 5 * off, g.obs, sizeof(double) * 5 * g.C, hipMemcpyDeviceToHost));
    std::vector<int> fl(g.C);
    HQ_TRY(hipMemcpy(fl.data(), g.flags, sizeof(int) * g.C, hipMemcpyDeviceToHost));
    for (int c = 0; c < g.C && bad < 0; ++c)
      if (fl[c] & 1) bad = (int)off + c;
    off += g.C;
  }
  if (bad >= 0) return fail(ctx, HQ_ENUMERIC, "non-finite G or log det in chain %d", bad);
  return HQ_OK;
}

hq_status hq_read_decisions(hq_ctx* ctx, int32_t chain, int32_t kind, uint8_t* accept, float* margin, int64_t n) {
  ST_TRY(check_ctx(ctx));
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || (kind != HQ_KIND_LOCAL && kind != HQ_KIND_GLOBAL && kind != HQ_KIND_NN && kind != HQ_KIND_CUMULATIVE &&
             kind != HQ_KIND_NN_GLOBAL))
    return fail(ctx, HQ_EINVAL, "bad chain or kind");
  if (!ctx->opt.record) return fail(ctx, HQ_EINVAL, "decisions are only kept with options.record = 1");
  const long slots = g->kind_slots(kind);
  if (n != slots || !accept || !margin) return fail(ctx, HQ_EINVAL, "expected %ld slots", slots);
  ST_TRY(sync(ctx));
  HQ_TRY(hipMemcpy(accept, g->log_accept[kind] + lc * slots, slots, hipMemcpyDeviceToHost));
  HQ_TRY(hipMemcpy(margin, g->log_margin[kind] + lc * slots, slots * sizeof(float), hipMemcpyDeviceToHost));
  return HQ_OK;
}

// Captured sweeps bake in kernel arguments and launch shapes; after a change
// of either they are captured again on the next hq_sweep.
static void drop_graphs(hq_ctx* ctx) {
  for (int d = 0; d < 2; ++d)
    for (int r = 0; r < 2; ++r)
      for (int v = 0; v < 2; ++v) {
        if (ctx->exec[d][r][v]) (void)hipGraphExecDestroy(ctx->exec[d][r][v]);
        if (ctx->graph[d][r][v]) (void)hipGraphDestroy(ctx->graph[d][r][v]);
        ctx->exec[d][r][v] = nullptr;
        ctx->graph[d][r][v] = nullptr;
      }
}

hq_status hq_set_replay(hq_ctx* ctx, int32_t chain, int32_t kind, const uint8_t* bits, int64_t n, double band) {
  ST_TRY(check_ctx(ctx));
  int lc = 0;
  Group* g = find_chain(ctx, chain, lc);
  if (!g || (kind != HQ_KIND_LOCAL && kind != HQ_KIND_GLOBAL && kind != HQ_KIND_NN && kind != HQ_KIND_CUMULATIVE &&
             kind != HQ_KIND_NN_GLOBAL))
    return fail(ctx, HQ_EINVAL, "bad chain or kind");
  if (!ctx->opt.record) return fail(ctx, HQ_EINVAL, "replay needs options.record = 1");
  const long slots = g->kind_slots(kind);
  if (!(band >= 0) || (n != 0 && (n != slots || !bits))) return fail(ctx, HQ_EINVAL, "expected %ld bits", slots);
  // the band is a kernel argument: the captured graphs are rebuilt on next use
  if (g->band[kind] != band) drop_graphs(ctx);
  g->band[kind] = band;
  if (n == 0) {
    HQ_TRY(launch_fill_u8(g->replay[kind] + lc * slots, 255, slots, ctx->stream));
  } else {
    std::vector<uint8_t> b(bits, bits + n);
    for (auto& v : b) v = v ? 1 : 0;
    HQ_TRY(hipMemcpyAsync(g->replay[kind] + lc * slots, b.data(), n, hipMemcpyHostToDevice, ctx->stream));
    HQ_TRY(hipStreamSynchronize(ctx->stream));
  }
  return HQ_OK;
}

int32_t hq_num_chains(const hq_ctx* ctx) { return ctx ? ctx->n_chains : 0; }

hq_status hq_chain_shape(const hq_ctx* ctx, int32_t chain, int32_t* n, int32_t* L) {
  if (!ctx || !n || !L) return HQ_EINVAL;
  for (const Group& g : ctx->groups)
    if (chain >= g.chain0 && chain < g.chain0 + g.C) {
      *n = g.n;
      *L = g.L;
      return HQ_OK;
    }
  return HQ_EINVAL;
}

hq_status hq_set_profiling(hq_ctx* ctx, int32_t on) {
  ST_TRY(check_ctx(ctx));
  ctx->profiling = on != 0;
  for (auto& p : ctx->phases) { p.ms = 0.0; p.launches = 0; }
  return HQ_OK;
}

hq_status hq_phase_time(hq_ctx* ctx, const char* phase, double* ms_total, int64_t* launches) {
  ST_TRY(check_ctx(ctx));
  if (!phase || !ms_total || !launches) return HQ_EINVAL;
  for (auto& p : ctx->phases)
    if (!std::strcmp(p.name, phase)) {
      *ms_total = p.ms;
      *launches = p.launches;
      return HQ_OK;
    }
  return fail(ctx, HQ_EINVAL, "unknown phase %s", phase);
}

hq_status hq_read_tuning(const hq_ctx* ctx, int32_t group, hq_tuning* out) {
  if (!ctx || !out || group < 0 || group >= (int32_t)ctx->groups.size()) return HQ_EINVAL;
  const Group& g = ctx->groups[group];
  out->gemm_tile_fp64 = g.tile;
  out->gemm_tile_wrap = g.tile32;
  out->local_block = g.kd;
  out->local_us = g.local_us;
  out->gemm_us_fp64 = g.tile_us;
  out->gemm_us_wrap = g.tile32_us;
  out->wrap_kind = g.wrap_kind;
  out->wrap_us = g.wrap_us;
  return HQ_OK;
}

hq_status hq_set_tuning(hq_ctx* ctx, int32_t group, int32_t tile_fp64, int32_t tile_wrap, int32_t wrap_kind) {
  ST_TRY(check_ctx(ctx));
  if (group < 0 || group >= (int32_t)ctx->groups.size()) return fail(ctx, HQ_EINVAL, "bad group %d", group);
  Group& g = ctx->groups[group];
  const bool mixed = ctx->opt.precision == HQ_PREC_MIXED;
  if (tile_fp64 < 0 || tile_fp64 >= N_GEMM_TILES || !gemm_tile_fits(tile_fp64, g.n, 0))
    return fail(ctx, HQ_EINVAL, "GEMM tile %d does not fit FP64 products of size %d", tile_fp64, g.n);
  if (tile_wrap < 0 || tile_wrap >= N_GEMM_TILES || !gemm_tile_fits(tile_wrap, g.n, mixed ? 1 : 0))
    return fail(ctx, HQ_EINVAL, "GEMM tile %d does not fit the wraps' products of size %d", tile_wrap, g.n);
  if (!mixed && tile_wrap != tile_fp64)
    return fail(ctx, HQ_EINVAL, "in FP64 precision the wraps use the FP64 tile");
  if (wrap_kind != WRAP_TWO && wrap_kind != WRAP_FUSED && wrap_kind != WRAP_KRON && wrap_kind != WRAP_KRON_LDS)
    return fail(ctx, HQ_EINVAL, "unknown wrap kind %d", wrap_kind);
  if (wrap_kind == WRAP_KRON_LDS && !kron_wrap_lds_supported(g.nx, mixed))
    return fail(ctx, HQ_EINVAL, "no LDS-resident Kronecker wrap for nx = %d", g.nx);
  if (wrap_kind == WRAP_FUSED && !wrap_fused_supported(g.n, mixed))
    return fail(ctx, HQ_EINVAL, "no fused wrap for N = %d", g.n);
  HQ_TRY(hipStreamSynchronize(ctx->stream));
  drop_graphs(ctx);
  g.tile = g.tile_wide = tile_fp64;
  g.tile32 = tile_wrap;
  g.wrap_kind = wrap_kind;
  g.tile_us = g.tile32_us = g.wrap_us = 0.0;
  return HQ_OK;
}

const char* hq_gemm_tile_name(int32_t tile) {
  switch (tile) {
    case TILE_64x64: return "64x64/k16";
    case TILE_32x32: return "32x32/k16";
    case TILE_48x48: return "48x48/k16";
    case TILE_16x64: return "16x64/k16";
    case TILE_FK_32x32: return "32x32/fullk";
    case TILE_FK_48x48: return "48x48/fullk";
    case TILE_FK_64x64: return "64x64/fullk";
    case TILE_FK_32x64: return "32x64/fullk";
    case TILE_PF_48x48: return "48x48/prefetch";
    case TILE_PF_64x64: return "64x64/prefetch";
    case TILE_PF_32x32: return "32x32/prefetch";
    case TILE_DX_48x48: return "48x48/direct";
    case TILE_DX_32x32: return "32x32/direct";
    case TILE_DX_64x64: return "64x64/direct";
    default: return "?";
  }
}

hq_status hq_synchronize(hq_ctx* ctx) {
  ST_TRY(check_ctx(ctx));
  return sync(ctx);
}

const char* hq_last_error(const hq_ctx* ctx) { return ctx ? ctx->err.c_str() : create_error.c_str(); }

void hq_destroy(hq_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->static_device >= 0) {
    std::lock_guard<std::mutex> lk(static_mu);
    static_busy[ctx->static_device] = 0;
  }
  drop_graphs(ctx);
  for (auto& pe : ctx->pending) { (void)hipEventDestroy(pe.first); (void)hipEventDestroy(pe.second); }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  for (auto st : ctx->side) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto e : ctx->join) (void)hipEventDestroy(e);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  delete ctx;
}

}  // extern "C"
