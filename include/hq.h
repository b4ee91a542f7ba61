/*
 * hq.h -- C ABI of libhq, DQMC sweeps of the 2D Holstein model on one
 * MI355X (gfx950) GPU.
 *
 * The method is the determinant quantum Monte Carlo of Li, Dee, Khatami and
 * Johnston, "Accelerating lattice quantum Monte Carlo simulations using
 * artificial neural networks: an application to the Holstein model":
 *   - Hamiltonian and units: section "Model";
 *   - Trotter slices, weight W = exp(-S_ph dtau) det M_up det M_dn,
 *     M = I + B_L ... B_1, B_l = exp(-dtau H_eph) exp(-dtau H_0), local and
 *     block moves accepted with W'/W: section "Determinant quantum Monte Carlo";
 *   - the network local move and the cumulative update p_c: sections
 *     "Local Updates" and "Global Updates" (the p_c equation).
 *
 * Conventions fixed by this library where the paper is silent:
 *   - site i = ix + nx*iy, periodic hopping -t to four neighbours (with
 *     multiplicity), -mu on the diagonal; slices l = 0..L-1, L = beta/dtau,
 *     periodic in imaginary time;
 *   - coupling g*x_i*(n_i - 1): B_l = diag(exp(-dtau g x[l,:])) exp(-dtau K)
 *     and the bosonic action S_b = dtau*S_ph - dtau*g*sum(x);
 *   - both spins are equal, W = exp(-S_b) det(M)^2; only log|det M| is kept;
 *   - sweep order (the paper fixes none): one local move per (site, slice),
 *     sites ascending within a slice.  Groups without block moves or network
 *     proposals alternate direction: even sweeps (counting from 0) take the
 *     slices ascending, each slice the wrap G <- B_l G B_l^-1 then its sites,
 *     with G and log|det M| recomputed (FP64, QR-stabilised) after slices l
 *     with (l+1) % n_stab == 0; odd sweeps take the slices descending, each
 *     slice its sites then the unwrap G <- B_l^-1 G B_l, recomputed after
 *     slices l with l % n_stab == 0.  Groups with block moves always ascend,
 *     then make one block move per site, sites ascending;
 *   - every random number comes from Philox4x64-10 with key (seed, 0) and
 *     counter (chain, sweep, slot, kind), so results do not depend on the
 *     execution order on the GPU.
 *
 * Memory: the caller owns one device buffer (the workspace, size from
 * hq_workspace_bytes) and the HIP stream; both must outlive the context.
 * The library allocates no device memory of its own.  Host buffers passed
 * to hq_read_* / hq_set_* are caller-owned and only used during the call.
 *
 * Errors: every call returns an hq_status.  Invalid arguments give
 * HQ_EINVAL and change nothing.  A failed HIP call gives HQ_EDEVICE and makes
 * the context unusable (later calls return HQ_ESTATE).  hq_last_error gives a
 * message owned by the context, valid until the next call on it.
 *
 * Threading: one context per host thread; all device work is ordered on the
 * context's stream.
 */
#ifndef HQ_H
#define HQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hq_ctx hq_ctx;

typedef enum {
  HQ_OK = 0,
  HQ_EINVAL = -1,   /* bad argument; nothing changed */
  HQ_ENOMEM = -2,   /* workspace too small */
  HQ_EDEVICE = -3,  /* a HIP call failed */
  HQ_ESTATE = -4,   /* context unusable after an earlier device error */
  HQ_ENUMERIC = -5  /* non-finite G or log det in some chain (see hq_stats.flags) */
} hq_status;

enum { HQ_PREC_FP64 = 0, HQ_PREC_MIXED = 1 };
enum { HQ_PROPOSAL_DQMC = 0, HQ_PROPOSAL_NETWORK = 1 };
/* decision kinds; equal to word 3 of the Philox counter of the draw */
enum { HQ_KIND_LOCAL = 0, HQ_KIND_GLOBAL = 1, HQ_KIND_NN = 3, HQ_KIND_CUMULATIVE = 4, HQ_KIND_NN_GLOBAL = 6,
       HQ_KIND_SCAN = 7 /* the direction draw of a network sweep; no decisions are logged */ };

/* One group of chains sharing a lattice and model parameters.  Chains are
 * numbered consecutively over the groups in the order given. */
typedef struct {
  int32_t nx;            /* lattice is nx*nx, periodic; N = nx*nx <= 256 */
  int32_t n_chains;      /* >= 1 */
  double t, mu;          /* hopping and chemical potential (section "Model") */
  double mass, omega;    /* ion mass M and phonon frequency Omega */
  double g;              /* e-ph coupling, used when g_hi <= g_lo */
  double g_lo, g_hi;     /* if g_hi > g_lo: per-chain g ~ U(g_lo, g_hi) */
  double beta, dtau;     /* L = beta/dtau must be an integer >= 2 */
  int32_t n_stab;        /* FP64 recompute every n_stab slices; must divide L */
  int32_t proposal;      /* HQ_PROPOSAL_DQMC or HQ_PROPOSAL_NETWORK */
  double local_width;    /* local move d ~ U(-w, w) */
  double global_width;   /* 0: no block moves; else one per site per sweep, d ~ U(-w, w).
                            Network groups: block moves proposed by the convolutional
                            network (hq_set_block_network), d ~ U(-w, w) */
  int32_t nn_sweeps;     /* network groups: n_u sweeps of network local moves, then n_u of
                            network block moves, per cumulative accept (0 means 1) */
} hq_group;

typedef struct {
  int32_t precision;     /* HQ_PREC_FP64 or HQ_PREC_MIXED (FP32 wraps and updates) */
  int32_t delay;         /* local-move block size k (8, 16 or 32): the sites are taken k
                            at a time and G gets one delayed rank-(accepts) update per
                            block; 0 = chosen by the library (hq_create times one slice
                            of local moves with each block size the lattice supports,
                            on copies of the chains' state, and keeps the faster;
                            hq_create_static takes 16) */
  int32_t activation;    /* network hidden activation: 0 ReLU, 1 softplus */
  int32_t record;        /* 1: keep every decision of the last sweep (hq_read_decisions) */
} hq_options;

typedef struct {
  double logdet;             /* tracked log|det M| */
  double g;                  /* this chain's coupling */
  int64_t local_proposals, local_accepts;
  int64_t global_proposals, global_accepts;
  int64_t nn_proposals, nn_accepts;
  int64_t cumulative_proposals, cumulative_accepts;
  double max_drift_green;    /* max |G_tracked - G_recomputed| at stabilisation points */
  double max_drift_logdet;   /* max |logdet_tracked - logdet_recomputed| */
  double last_drift_green;   /* the same, last stabilisation point only */
  double density, double_occupancy, s_cdw, x_mean, x2_mean;  /* from the current G, x */
  int64_t replay_overrides;  /* decisions taken from the replay log inside the tie band */
  int64_t replay_mismatches; /* replay disagreements outside the tie band */
  double last_log_pc;        /* network groups: log p_c of the last cumulative accept */
  double last_sum_y;         /* and the sum of the accepted network estimates in it */
  int32_t n, L, flags;       /* flags: bit 0 non-finite G / log det seen */
} hq_stats;

/* Bytes of device workspace needed for these groups and options; 0 if invalid. */
size_t hq_workspace_bytes(const hq_group* groups, int32_t n_groups, const hq_options* opt);

/* Create a context on the current HIP device, carve the workspace, draw the
 * initial fields x[l,i] ~ N(0,1) (Box-Muller on Philox kind 2) and per-chain
 * couplings (kind 5), and compute G and log|det M| from scratch.  stream is a
 * hipStream_t (not the null stream: sweeps are captured into a HIP graph). */
hq_status hq_create(const hq_group* groups, int32_t n_groups, const hq_options* opt,
                    uint64_t seed, void* workspace, size_t workspace_bytes,
                    void* stream, hq_ctx** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hq_create
 * with the library's own workspace, a static device array of
 * HQ_STATIC_WORKSPACE_BYTES that every GPU the library runs on holds until
 * the process ends.  The call allocates no device memory: no hipMalloc, no
 * hipFree, no side streams and no timing events (the autotuner does not run:
 * the products take the 64 x 64 tile and the wraps the Kronecker form, as
 * hq_set_tuning(ctx, 0, 0, 0, HQ_WRAP_KRON) would pin).  Limits: one group
 * (n_groups = 1), and hq_workspace_bytes + 256 <= HQ_STATIC_WORKSPACE_BYTES,
 * else HQ_ENOMEM; one static context per GPU at a time: while one is alive on
 * the current device, another call returns HQ_ESTATE (two contexts on the
 * one array would race; hq_destroy frees it for the next).  Every buffer the
 * sweep reads is initialised here, so nothing of an earlier context leaks
 * into a new one.  Failures of hq_create and hq_create_static are described
 * by hq_last_error(NULL). */
#define HQ_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
hq_status hq_create_static(const hq_group* groups, int32_t n_groups, const hq_options* opt,
                           uint64_t seed, void* stream, hq_ctx** out);

/* Replace one chain's fields (host array x[l*N + i], L*N doubles) and recompute
 * G and log|det M| of its group from scratch.  Counters are kept. */
hq_status hq_set_fields(hq_ctx* ctx, int32_t chain, const double* x_host, int64_t n);

/* Load the 45-64-64-1 network (7169 FP32 values: W1[64][45], b1[64],
 * W2[64][64], b2[64], W3[64], b3) used by HQ_PROPOSAL_NETWORK groups
 * (section "Local Updates").  Inputs of a move of x[l][i] by d:
 * p = 9 (dl+2) + 3 (dy+1) + (dx+1) holds x at slice l+dl, site
 * (ix+dx, iy+dy), periodic, except p = 22, which holds d.  The estimate of
 * the move's fermionic change of log W is the odd part (f(d) - f(-d)) / 2 of
 * the output f.  Each sweep of a network group draws its direction (Philox
 * kind 7, chain 0, slot 0; word 0 >= 1/2: reversed) and visits its colour
 * classes forward or in reverse, so that p_c is the exact Metropolis-Hastings
 * ratio of the whole network sweep (section "Global Updates", the p_c
 * equation). */
hq_status hq_set_network(hq_ctx* ctx, const float* weights, int64_t n);

/* Load the convolutional network of network block moves (paper: "Global
 * Updates" and the caption of its network figure), for groups with L slices:
 * n = 64 L + 117 FP32 values Wc[4][3][4], bc[4], Wd[32][2 L], bd[32], Wo[32],
 * bo.  Input of a move at site i: three channels over l (x[l][i] and the
 * means of the four nearest and the four diagonal next-nearest neighbours);
 * a circular convolution along l (output p reads slices 2p .. 2p+3 mod L),
 * sigmoid; a dense layer of 32 sigmoid units over the conv output flattened
 * as c*(L/2) + p; a linear output f.  The estimate of a move's fermionic
 * change of log W is f(x_i + d) - f(x_i).  HQ_EINVAL for odd L or a count
 * that is not 64 L + 117; a network group with global_width > 0 must have
 * this L. */
hq_status hq_set_block_network(hq_ctx* ctx, const float* weights, int64_t n, int32_t L);

/* Run n_sweeps full sweeps of every chain (asynchronous on the stream): the
 * local moves of section "Determinant quantum Monte Carlo" (ratio
 * r = 1 + delta (1 - G_ii), W'/W = r^2 exp(-dS_b), rank-1 update of G, done
 * in delayed blocks of options.delay sites) with periodic recomputation, the
 * block moves of section "Global Updates" accepted with the exact weight
 * ratio, and, for network groups, the network proposals of sections "Local
 * Updates" and "Global Updates" followed by the cumulative accept p_c.  The
 * sweep is captured into a HIP graph once and replayed; a capture that fails
 * leaves nothing behind. */
hq_status hq_sweep(hq_ctx* ctx, int32_t n_sweeps);

/* Recompute G = M^-1 and log|det M|, M = I + B_{L-1} ... B_0, of every chain
 * from its fields (FP64, QR/UDT-stabilised products; section "Determinant
 * quantum Monte Carlo").  The drift counters are not changed. */
hq_status hq_recompute(hq_ctx* ctx);

/* Copy one chain's state to host memory (synchronises the stream).
 * green: N*N row-major FP64, G_ij = <c_i c_j^dagger> = (M^-1)_ij at the
 * imaginary-time boundary (section "Determinant quantum Monte Carlo"; in
 * mixed precision the FP32 copy, widened).  fields: L*N FP64, x[l*N + i],
 * the phonon field X_{i,l} of section "Model".  stats: counters, drift and
 * the equal-time observables of section "Benchmarks" (density, double
 * occupancy, S_CDW(pi, pi)) from the current G by Wick's theorem. */
hq_status hq_read_green(hq_ctx* ctx, int32_t chain, double* out, int64_t n);
/* The tracked G (N*N, row-major, widened to FP64) and tracked log|det M| of
 * one chain as they stood just before the last stabilisation point of the
 * last sweep replaced them with the FP64 recomputation (section "Determinant
 * quantum Monte Carlo": G is carried from slice to slice by wraps and rank-1
 * updates and periodically recomputed).  In mixed precision this is the
 * FP32 state the sweep produced.  Needs options.record = 1 (HQ_EINVAL
 * otherwise); a context that has not swept yet returns zeros. */
hq_status hq_read_green_tracked(hq_ctx* ctx, int32_t chain, double* out, int64_t n, double* logdet);
hq_status hq_read_fields(hq_ctx* ctx, int32_t chain, double* out, int64_t n);
hq_status hq_read_stats(hq_ctx* ctx, int32_t chain, hq_stats* out);
/* The equal-time observables of section "Benchmarks" for every chain at once
 * (one launch per lattice group, one copy per group; synchronises the
 * stream): out[5c + k] for chain c = 0 .. chains-1 and k = density, double
 * occupancy, S_CDW(pi, pi), mean of x, mean of x^2, the same values as the
 * fields of hq_read_stats.  out: host array of n = 5 * chains doubles,
 * caller-owned.  HQ_EINVAL for a null out or another n; HQ_ENUMERIC if a
 * chain's G holds a non-finite value (out is filled all the same). */
hq_status hq_read_observables(hq_ctx* ctx, double* out, int64_t n);

/* Decisions of the last sweep for one chain and kind, in slot order (local:
 * l*N + i; network local moves: u*L*N + l*N + i and network block moves:
 * u*N + i for inner sweep u < n_u; block: i; cumulative: 0).  accept[k] is 0/1;
 * margin[k] = ln u - ln R (FP32).  Needs options.record = 1. */
hq_status hq_read_decisions(hq_ctx* ctx, int32_t chain, int32_t kind,
                            uint8_t* accept, float* margin, int64_t n);

/* Tie-band replay for the next sweep only: where |ln u - ln R| <= band the
 * chain takes bits[slot] instead of its own decision; elsewhere a
 * disagreement is counted in hq_stats.replay_mismatches.  n = 0 clears.
 * A test facility: needs options.record = 1 (HQ_EINVAL otherwise; the
 * kernels of other contexts carry no replay work). */
hq_status hq_set_replay(hq_ctx* ctx, int32_t chain, int32_t kind,
                        const uint8_t* bits, int64_t n, double band);

/* Number of chains, and one chain's N and L. */
int32_t hq_num_chains(const hq_ctx* ctx);
hq_status hq_chain_shape(const hq_ctx* ctx, int32_t chain, int32_t* n, int32_t* L);

/* Average device time per launch of the named kernel over the last hq_sweep
 * calls, measured with HIP events on the context's stream when profiling is
 * on.  names: "wrap", "local", "stab", "global", "network". */
hq_status hq_set_profiling(hq_ctx* ctx, int32_t on);
hq_status hq_phase_time(hq_ctx* ctx, const char* phase, double* ms_total, int64_t* launches);

/* How a wrap G <- B_l G B_l^-1 (B_l = exp(-dtau V_l) exp(-dtau K), paper:
 * section "Determinant quantum Monte Carlo") multiplies by exp(-+dtau K):
 *   HQ_WRAP_TWO    two tiled dense products;
 *   HQ_WRAP_FUSED  both dense products in one launch (N <= 144);
 *   HQ_WRAP_KRON   exp(s dtau K) = E1 (x) E1 on the periodic square lattice
 *                  (E1 of size nx, site index ix + nx iy), applied as two
 *                  passes of nx-term sums on each side, one launch a side;
 *   HQ_WRAP_KRON_LDS  the same four passes in one launch, the matrix held in
 *                  LDS (nx <= 12 in mixed precision, nx <= 10 in FP64). */
enum { HQ_WRAP_TWO = 0, HQ_WRAP_FUSED = 1, HQ_WRAP_KRON = 2, HQ_WRAP_KRON_LDS = 3 };

/* The configuration chosen at hq_create for one group: the GEMM tile of
 * the FP64 products (UDT combines and merges) and of the wraps' dense
 * products in the context's precision, found by timing every tile that fits
 * on the group's own shape; the wrap form (HQ_WRAP_*) that timed fastest;
 * and the local-move block size (timed when options.delay is 0; local_us
 * is then the chosen size's time of one slice of local moves, else 0).
 * Block products always take the Kronecker
 * form.  Tile names from hq_gemm_tile_name (a static string; "?" for an
 * unknown code). */
typedef struct {
  int32_t gemm_tile_fp64, gemm_tile_wrap, local_block;
  double gemm_us_fp64, gemm_us_wrap;   /* measured time of one batched product */
  int32_t wrap_kind;                   /* HQ_WRAP_* */
  double wrap_us;                      /* measured time of one wrap of all the group's chains */
  double local_us;                     /* measured time of one slice of local moves (see above) */
} hq_tuning;
hq_status hq_read_tuning(const hq_ctx* ctx, int32_t group, hq_tuning* out);

/* Pin one group's GEMM tiles and wrap form in place of the autotuner's
 * choice (for reproducible timings and for testing every path).  Tile codes
 * are those of hq_read_tuning, 0 .. 13; wrap_kind one of HQ_WRAP_*.
 * HQ_EINVAL, with nothing changed, for an unknown code, a tile that does not
 * fit the group's N in that precision, in FP64 precision tile_wrap !=
 * tile_fp64, HQ_WRAP_FUSED with N > 144, or HQ_WRAP_KRON_LDS beyond its
 * sizes.  Waits for the context's
 * stream; the sweep graphs are captured again on the next hq_sweep.  The
 * timings that hq_read_tuning reports become 0. */
hq_status hq_set_tuning(hq_ctx* ctx, int32_t group, int32_t tile_fp64, int32_t tile_wrap, int32_t wrap_kind);
const char* hq_gemm_tile_name(int32_t tile);

/* Wait for all work on the context's stream. */
hq_status hq_synchronize(hq_ctx* ctx);

/* The message of the last failed call on ctx; with ctx = NULL, of the last
 * failed hq_create or hq_create_static on this thread. */
const char* hq_last_error(const hq_ctx* ctx);
void hq_destroy(hq_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* HQ_H */
