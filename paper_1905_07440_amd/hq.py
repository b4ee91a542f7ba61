"""ctypes binding of libhq (include/hq.h).  Argument marshalling only: every
step of the sweep runs in the library's HIP kernels.  PyTorch supplies the
device workspace and the stream.

    ctx = Context(groups, precision=0, seed=1)
    ctx.sweep(5)
    G = ctx.green(0); x = ctx.fields(0); st = ctx.stats(0)
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhq.so")

HQ_OK, HQ_EINVAL, HQ_ENOMEM, HQ_EDEVICE, HQ_ESTATE, HQ_ENUMERIC = 0, -1, -2, -3, -4, -5
KIND_LOCAL, KIND_GLOBAL, KIND_NN, KIND_CUMULATIVE, KIND_NN_GLOBAL = 0, 1, 3, 4, 6
PREC_FP64, PREC_MIXED = 0, 1
PROPOSAL_DQMC, PROPOSAL_NETWORK = 0, 1


class HQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libhq status %d: %s" % (status, msg))
        self.status = status


class Group(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("n_chains", ctypes.c_int32),
        ("t", ctypes.c_double), ("mu", ctypes.c_double),
        ("mass", ctypes.c_double), ("omega", ctypes.c_double),
        ("g", ctypes.c_double), ("g_lo", ctypes.c_double), ("g_hi", ctypes.c_double),
        ("beta", ctypes.c_double), ("dtau", ctypes.c_double),
        ("n_stab", ctypes.c_int32), ("proposal", ctypes.c_int32),
        ("local_width", ctypes.c_double), ("global_width", ctypes.c_double),
        ("nn_sweeps", ctypes.c_int32),
    ]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("delay", ctypes.c_int32),
                ("activation", ctypes.c_int32), ("record", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("logdet", ctypes.c_double), ("g", ctypes.c_double),
        ("local_proposals", ctypes.c_int64), ("local_accepts", ctypes.c_int64),
        ("global_proposals", ctypes.c_int64), ("global_accepts", ctypes.c_int64),
        ("nn_proposals", ctypes.c_int64), ("nn_accepts", ctypes.c_int64),
        ("cumulative_proposals", ctypes.c_int64), ("cumulative_accepts", ctypes.c_int64),
        ("max_drift_green", ctypes.c_double), ("max_drift_logdet", ctypes.c_double),
        ("last_drift_green", ctypes.c_double),
        ("density", ctypes.c_double), ("double_occupancy", ctypes.c_double),
        ("s_cdw", ctypes.c_double), ("x_mean", ctypes.c_double), ("x2_mean", ctypes.c_double),
        ("replay_overrides", ctypes.c_int64), ("replay_mismatches", ctypes.c_int64),
        ("last_log_pc", ctypes.c_double), ("last_sum_y", ctypes.c_double),
        ("n", ctypes.c_int32), ("L", ctypes.c_int32), ("flags", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("gemm_tile_fp64", ctypes.c_int32), ("gemm_tile_wrap", ctypes.c_int32),
                ("local_block", ctypes.c_int32), ("gemm_us_fp64", ctypes.c_double),
                ("gemm_us_wrap", ctypes.c_double), ("wrap_kind", ctypes.c_int32),
                ("wrap_us", ctypes.c_double), ("local_us", ctypes.c_double)]


N_GEMM_TILES = 14
# forms of a wrap (HQ_WRAP_*): two tiled dense products, both in one launch,
# the Kronecker passes of exp(-+dtau K) = E1 (x) E1 in two launches, or in
# one launch with G held in LDS
WRAP_KINDS = ("two", "fused", "kron", "kron_lds")

def tile_name(code):
    """Name of a GEMM tile code ("?" for an unknown one)."""
    return load().hq_gemm_tile_name(code).decode()


EXPORTS = [
    "hq_workspace_bytes", "hq_create", "hq_create_static", "hq_set_fields", "hq_set_network", "hq_set_block_network", "hq_sweep",
    "hq_recompute", "hq_read_green", "hq_read_green_tracked", "hq_read_fields", "hq_read_stats", "hq_read_observables", "hq_read_decisions",
    "hq_set_replay", "hq_num_chains", "hq_chain_shape", "hq_set_profiling", "hq_phase_time",
    "hq_read_tuning", "hq_set_tuning", "hq_gemm_tile_name", "hq_synchronize", "hq_last_error", "hq_destroy",
]

_lib = None


def load(path=LIB_PATH):
    """Load libhq.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libhq.so is not built; run `python -m paper_1905_07440_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    GP = ctypes.POINTER(Group)
    OP = ctypes.POINTER(Options)
    lib.hq_workspace_bytes.argtypes = [GP, I32, OP]
    lib.hq_workspace_bytes.restype = ctypes.c_size_t
    lib.hq_create.argtypes = [GP, I32, OP, ctypes.c_uint64, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.hq_create_static.argtypes = [GP, I32, OP, ctypes.c_uint64, P, ctypes.POINTER(P)]
    lib.hq_set_fields.argtypes = [P, I32, P, I64]
    lib.hq_set_network.argtypes = [P, P, I64]
    lib.hq_set_block_network.argtypes = [P, P, I64, I32]
    lib.hq_sweep.argtypes = [P, I32]
    lib.hq_recompute.argtypes = [P]
    lib.hq_read_green.argtypes = [P, I32, P, I64]
    lib.hq_read_green_tracked.argtypes = [P, I32, P, I64, P]
    lib.hq_read_fields.argtypes = [P, I32, P, I64]
    lib.hq_read_stats.argtypes = [P, I32, ctypes.POINTER(Stats)]
    lib.hq_read_observables.argtypes = [P, P, I64]
    lib.hq_read_decisions.argtypes = [P, I32, I32, P, P, I64]
    lib.hq_set_replay.argtypes = [P, I32, I32, P, I64, D]
    lib.hq_num_chains.argtypes = [P]
    lib.hq_num_chains.restype = I32
    lib.hq_chain_shape.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.hq_set_profiling.argtypes = [P, I32]
    lib.hq_phase_time.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I64)]
    lib.hq_read_tuning.argtypes = [P, I32, ctypes.POINTER(Tuning)]
    lib.hq_set_tuning.argtypes = [P, I32, I32, I32, I32]
    lib.hq_gemm_tile_name.argtypes = [I32]
    lib.hq_gemm_tile_name.restype = ctypes.c_char_p
    lib.hq_synchronize.argtypes = [P]
    lib.hq_last_error.argtypes = [P]
    lib.hq_last_error.restype = ctypes.c_char_p
    lib.hq_destroy.argtypes = [P]
    lib.hq_destroy.restype = None
    for name in EXPORTS:
        if name not in ("hq_workspace_bytes", "hq_num_chains", "hq_last_error", "hq_destroy",
                        "hq_gemm_tile_name"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def make_group(nx, n_chains, t=1.0, mu=0.0, mass=1.0, omega=1.0, g=1.0, g_range=None, beta=4.0,
               dtau=0.1, n_stab=10, proposal=0, local_width=0.5, global_width=0.0, nn_sweeps=1):
    lo, hi = (g_range if g_range is not None else (0.0, 0.0))
    return Group(nx, n_chains, t, mu, mass, omega, g, lo, hi, beta, dtau, n_stab, proposal,
                 local_width, global_width, nn_sweeps)


def groups_from_workload(w):
    return [make_group(gr.nx, gr.n_chains, gr.t, gr.mu, gr.mass, gr.omega, gr.g, gr.g_range, gr.beta,
                       gr.dtau, gr.n_stab, gr.proposal, gr.local_width, gr.global_width,
                       getattr(gr, "nn_sweeps", 1))
            for gr in w.groups]


class Context:
    """A set of Markov chains on the current GPU (torch supplies memory and stream)."""

    def __init__(self, groups, precision=PREC_FP64, seed=1, delay=0, activation=0, record=False,
                 device="cuda", static=False):
        """static=True: the library's own static workspace (hq_create_static:
        one group, no device allocation in the call) instead of a torch buffer."""
        import torch
        lib = load()
        self._lib = lib
        self._groups = (Group * len(groups))(*groups)
        self._opt = Options(precision, delay, activation, 1 if record else 0)
        nbytes = lib.hq_workspace_bytes(self._groups, len(groups), ctypes.byref(self._opt))
        if nbytes == 0:
            raise HQError(HQ_EINVAL, "invalid groups/options (see include/hq.h limits)")
        self.workspace_bytes = int(nbytes)
        self._stream = torch.cuda.Stream(device=device)
        self._ctx = ctypes.c_void_p()
        if static:
            self._ws = None
            st = lib.hq_create_static(self._groups, len(groups), ctypes.byref(self._opt), ctypes.c_uint64(seed),
                                      ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(self._ctx))
        else:
            self._ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
            st = lib.hq_create(self._groups, len(groups), ctypes.byref(self._opt), ctypes.c_uint64(seed),
                               ctypes.c_void_p(self._ws.data_ptr()), ctypes.c_size_t(self._ws.numel()),
                               ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(self._ctx))
        if st != HQ_OK:
            msg = lib.hq_last_error(self._ctx if self._ctx else None).decode()
            if self._ctx:
                lib.hq_destroy(self._ctx)
                self._ctx = ctypes.c_void_p()
            raise HQError(st, msg)
        self.n_chains = lib.hq_num_chains(self._ctx)
        self.precision = precision

    def _check(self, st):
        if st != HQ_OK:
            raise HQError(st, self._lib.hq_last_error(self._ctx).decode())

    def shape(self, chain):
        n, L = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.hq_chain_shape(self._ctx, chain, ctypes.byref(n), ctypes.byref(L)))
        return n.value, L.value

    def sweep(self, n=1):
        self._check(self._lib.hq_sweep(self._ctx, n))

    def recompute(self):
        self._check(self._lib.hq_recompute(self._ctx))

    def synchronize(self):
        self._check(self._lib.hq_synchronize(self._ctx))

    def green(self, chain):
        n, _ = self.shape(chain)
        out = np.empty((n, n))
        self._check(self._lib.hq_read_green(self._ctx, chain, out.ctypes.data, out.size))
        return out

    def green_tracked(self, chain):
        """The tracked G and log|det M| just before the last stabilisation point
        replaced them (needs record=True)."""
        n, _ = self.shape(chain)
        out = np.empty((n, n))
        ld = ctypes.c_double(0.0)
        self._check(self._lib.hq_read_green_tracked(self._ctx, chain, out.ctypes.data, out.size,
                                                    ctypes.byref(ld)))
        return out, ld.value

    def fields(self, chain):
        n, L = self.shape(chain)
        out = np.empty((L, n))
        self._check(self._lib.hq_read_fields(self._ctx, chain, out.ctypes.data, out.size))
        return out

    def set_fields(self, chain, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        self._check(self._lib.hq_set_fields(self._ctx, chain, x.ctypes.data, x.size))

    def set_network(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self._lib.hq_set_network(self._ctx, w.ctypes.data, w.size))

    def set_block_network(self, w, L):
        """Weights of the block-move network (64 L + 117 FP32 values) for the
        network groups with block moves, all of which have L slices."""
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self._lib.hq_set_block_network(self._ctx, w.ctypes.data, w.size, L))

    def stats(self, chain):
        s = Stats()
        st = self._lib.hq_read_stats(self._ctx, chain, ctypes.byref(s))
        if st not in (HQ_OK, HQ_ENUMERIC):
            self._check(st)
        return s.as_dict()

    def observables(self):
        """[chains][5] FP64: density, double occupancy, S_CDW(pi, pi), mean x,
        mean x^2 of every chain from the current G and fields, in one pass."""
        out = np.zeros((self.n_chains, 5))
        st = self._lib.hq_read_observables(self._ctx, out.ctypes.data, out.size)
        if st not in (HQ_OK, HQ_ENUMERIC):
            self._check(st)
        return out

    def _inner_sweeps(self, chain):
        k = 0
        for gr in self._groups:
            if chain < k + gr.n_chains:
                return max(1, gr.nn_sweeps) if gr.proposal == PROPOSAL_NETWORK else 1
            k += gr.n_chains
        raise HQError(HQ_EINVAL, "no chain %d" % chain)

    def decisions(self, chain, kind):
        n, L = self.shape(chain)
        nu = self._inner_sweeps(chain)
        slots = {KIND_LOCAL: n * L, KIND_NN: nu * n * L, KIND_GLOBAL: n, KIND_CUMULATIVE: 1,
                 KIND_NN_GLOBAL: nu * n}[kind]
        acc = np.empty(slots, dtype=np.uint8)
        margin = np.empty(slots, dtype=np.float32)
        self._check(self._lib.hq_read_decisions(self._ctx, chain, kind, acc.ctypes.data,
                                                margin.ctypes.data, slots))
        return acc, margin

    def set_replay(self, chain, kind, bits, band):
        if bits is None:
            self._check(self._lib.hq_set_replay(self._ctx, chain, kind, None, 0, band))
            return
        b = np.ascontiguousarray(bits, dtype=np.uint8)
        self._check(self._lib.hq_set_replay(self._ctx, chain, kind, b.ctypes.data, b.size, band))

    def set_profiling(self, on):
        self._check(self._lib.hq_set_profiling(self._ctx, 1 if on else 0))

    def phase_time(self, phase):
        ms, k = ctypes.c_double(), ctypes.c_int64()
        self._check(self._lib.hq_phase_time(self._ctx, phase.encode(), ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def set_tuning(self, group, tile_fp64, tile_wrap=None, wrap="two"):
        """Pin a group's GEMM tiles (codes 0 .. N_GEMM_TILES-1; the wraps take
        tile_fp64 when tile_wrap is None) and the wrap's form (one of
        WRAP_KINDS)."""
        if wrap not in WRAP_KINDS:
            raise ValueError("wrap must be one of %s" % (WRAP_KINDS,))
        self._check(self._lib.hq_set_tuning(self._ctx, group, tile_fp64,
                                            tile_fp64 if tile_wrap is None else tile_wrap,
                                            WRAP_KINDS.index(wrap)))

    def tuning(self, group):
        """The autotuner's choices for one group (GEMM tiles by name, timings in us)."""
        t = Tuning()
        self._check(self._lib.hq_read_tuning(self._ctx, group, ctypes.byref(t)))
        name = self._lib.hq_gemm_tile_name
        return {"gemm_tile_fp64": name(t.gemm_tile_fp64).decode(), "gemm_us_fp64": t.gemm_us_fp64,
                "gemm_tile_wrap": name(t.gemm_tile_wrap).decode(), "gemm_us_wrap": t.gemm_us_wrap,
                "wrap": WRAP_KINDS[t.wrap_kind] if 0 <= t.wrap_kind < len(WRAP_KINDS) else "?",
                "wrap_us": t.wrap_us, "local_block": t.local_block, "local_us": t.local_us}

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx:
            self._lib.hq_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
