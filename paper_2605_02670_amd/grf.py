"""Thin ctypes binding of libgrf (include/grf.h).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch supplies device memory and the current stream.  If the library has
not been built, every call raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrf.so")
_lib = None

GRF_OK, GRF_EINVAL, GRF_ENOMEM, GRF_EDEVICE, GRF_ENOCONV, GRF_EUNSUP, GRF_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
MESH = {"ceil": 0, "round": 1}
MASS = {"lumped": 0, "consistent": 2}  # GRF_MASS_CONSISTENT_SYS
NOISE = {"lumped": 0, "consistent": 4}  # GRF_NOISE_CONSISTENT
PREC = {"fp64": 0, "mixed": 1}
PRECOND = {"jacobi": 0, "learned": 1, "nn": 2}
ACTIVATIONS = {"fp32": 0, "bf16": 1}  # GRF_ACT_*
PCG_MODES = {"op": 0, "guess": 1, "jacobi": 2}  # grf_stats also reports 3: "global"
PCG_MODES_SET = 1 << 12
KERNELS = ["noise", "coeff", "ends_fwd", "ends_bwd", "condense", "pcg", "scatter", "acc_fwd", "acc_bwd",
           "layout", "mixed", "learned", "table"]


class GrfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgrf error {code}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [("n_shifts", C.c_int32), ("n_systems", C.c_int32), ("n_unconverged", C.c_int32),
                ("max_iterations", C.c_int32), ("total_iterations", C.c_int64),
                ("max_rel_residual", C.c_double), ("refine_steps", C.c_int32),
                ("shift_block", C.c_int32), ("sweep_block", C.c_int32), ("pcg_class_modes", C.c_int32),
                ("kernel_ms", C.c_double * 16), ("kernel_launches", C.c_int32 * 16),
                ("pcg_class_ms", C.c_double * 7), ("pcg_class_launches", C.c_int32 * 7),
                ("n_nonfinite", C.c_int32), ("pcg_class_vertex_its", C.c_int64 * 7),
                ("pcg_class_end_its", C.c_int64 * 7)]
    _ARRAYS = ("kernel_ms", "kernel_launches", "pcg_class_ms", "pcg_class_launches",
               "pcg_class_vertex_its", "pcg_class_end_its")

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in self._ARRAYS}
        d["kernel_ms"] = {k: self.kernel_ms[i] for i, k in enumerate(KERNELS)}
        d["kernel_launches"] = {k: self.kernel_launches[i] for i, k in enumerate(KERNELS)}
        for k in ("pcg_class_ms", "pcg_class_launches", "pcg_class_vertex_its", "pcg_class_end_its"):
            d[k] = list(getattr(self, k))
        return d


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("precision", C.c_int32), ("precond", C.c_int32),
                ("k_minus", C.c_int32), ("k_plus", C.c_int32), ("shift_block", C.c_int32),
                ("sweep_block", C.c_int32), ("refine", C.c_int32), ("timing", C.c_int32),
                ("pcg_class_modes", C.c_int32), ("sample_offset", C.c_int64),
                ("stream", C.c_void_p), ("learned", C.c_void_p), ("stats", C.POINTER(Stats))]


# (name, restype, argtypes) for every function declared in include/grf.h
_SIGS = [
    ("grf_opts_init", None, [C.POINTER(Opts)]),
    ("grf_graph_create", C.c_int, [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_double, C.c_uint32,
                                   C.POINTER(C.c_void_p)]),
    ("grf_graph_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_void_p]),
    ("grf_graph_destroy", C.c_int, [C.c_void_p]),
    ("grf_graph_lumped_mass", C.c_int, [C.c_void_p, C.c_void_p]),
    ("grf_shift_count", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(Opts), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("grf_noise", C.c_int, [C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p, C.POINTER(Opts)]),
    ("grf_sample", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_uint64, C.c_void_p,
                             C.POINTER(Opts)]),
    ("grf_sample_noalloc", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_uint64,
                                     C.c_void_p, C.POINTER(Opts)]),
    ("grf_sample_from_noise", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.POINTER(Opts)]),
    ("grf_solve_shifted", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_void_p,
                                    C.c_void_p, C.POINTER(Opts)]),
    ("grf_sample_batched", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_double, C.c_int64,
                                     C.c_uint64, C.c_void_p, C.POINTER(Opts)]),
    ("grf_learned_param_count", C.c_int, [C.POINTER(C.c_int64)]),
    ("grf_learned_create", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    ("grf_learned_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    ("grf_learned_destroy", C.c_int, [C.c_void_p]),
    ("grf_learned_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int64,
                                        C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.POINTER(Opts)]),
    ("grf_learned_operators", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Opts)]),
    ("grf_learned_train", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_double,
                                    C.c_int64, C.c_uint64, C.c_int32, C.c_int32, C.c_double, C.c_void_p,
                                    C.POINTER(Opts)]),
    ("grf_last_error", C.c_char_p, []),
]


def load():
    """Load libgrf.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2605_02670_amd.build)")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(code: int, allow=(GRF_OK,)) -> int:
    if code not in allow:
        raise GrfError(code, load().grf_last_error().decode())
    return code


def _allowed(noconv: bool, nonfinite: bool) -> tuple:
    """Status codes a call may return without raising: GRF_ENOCONV and
    GRF_ENONFINITE still write the output (the stats say which systems failed)."""
    return (GRF_OK,) + ((GRF_ENOCONV,) if noconv else ()) + ((GRF_ENONFINITE,) if nonfinite else ())


def check_array(t, n_rows: int, n_cols: int, name: str, device=None):
    """Raises ValueError unless t is a contiguous float64 CUDA tensor of shape
    (n_rows, n_cols) (on ``device`` if given): the library writes or reads
    exactly n_rows * n_cols doubles through its pointer."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, got {t.dtype}")
    if tuple(t.shape) != (n_rows, n_cols):
        raise ValueError(f"{name} must have shape ({n_rows}, {n_cols}), got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a CUDA (HIP) device, got {t.device}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the graph on cuda:{device}")
    return t


def _stream_handle(stream=None) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_opts(tol=1e-12, maxit=10000, precision="fp64", precond="jacobi", k_minus=-1, k_plus=-1,
              shift_block=0, sweep_block=0, refine=-1, sample_offset=0, stream=None, learned=None,
              stats: Stats | None = None, timing=False, pcg_class_modes=None) -> Opts:
    """pcg_class_modes: None (automatic) or, with the learned preconditioner, one
    on-chip PCG variant per size class (PCG_MODES: "op", "guess", "jacobi")."""
    o = Opts()
    load().grf_opts_init(C.byref(o))
    o.tol = tol
    o.maxit = maxit
    o.precision = PREC[precision]
    o.precond = PRECOND[precond]
    o.k_minus = k_minus
    o.k_plus = k_plus
    o.shift_block = shift_block
    o.sweep_block = sweep_block
    o.refine = refine
    o.timing = 1 if timing else 0
    o.sample_offset = sample_offset
    o.stream = C.c_void_p(_stream_handle(stream)) if stream is not False else None
    o.learned = C.c_void_p(learned.handle) if learned is not None else None
    if learned is not None and precond == "jacobi":
        o.precond = PRECOND["learned"]
    if pcg_class_modes is not None:
        mw = PCG_MODES_SET
        for c, m in enumerate(pcg_class_modes):
            mw |= PCG_MODES[m] << (2 * c)
        o.pcg_class_modes = mw
    if stats is not None:
        o.stats = C.pointer(stats)
    return o


def class_modes(word: int) -> list[str]:
    """The per-class PCG variants of grf_stats.pcg_class_modes."""
    names = {v: k for k, v in PCG_MODES.items()}
    names[3] = "global"
    return [names[(word >> (2 * c)) & 3] for c in range(6)]


class Graph:
    """A metric graph and its mesh on the current HIP device."""

    def __init__(self, n_vertices: int, edges, lengths, h: float, rule: str = "ceil", mass: str = "lumped",
                 noise: str = "lumped"):
        """mass: the mass matrix of the shifted systems, "lumped" or "consistent"
        (GRF_MASS_CONSISTENT_SYS); noise: M_L^{1/2} xi ("lumped") or the
        consistent-mass noise of the element factors ("consistent",
        GRF_NOISE_CONSISTENT)."""
        lib = load()
        if mass not in MASS:
            raise ValueError(f"mass must be one of {sorted(MASS)}, got {mass!r}")
        if noise not in NOISE:
            raise ValueError(f"noise must be one of {sorted(NOISE)}, got {noise!r}")
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
        L = np.ascontiguousarray(np.asarray(lengths, dtype=np.float64).reshape(-1))
        self.n_vertices = int(n_vertices)
        self.n_edges = int(e.shape[0])
        self.h = float(h)
        self.rule = rule
        self.mass = mass
        self.noise_kind = noise
        handle = C.c_void_p()
        _check(lib.grf_graph_create(self.n_vertices, self.n_edges, e.ctypes.data, L.ctypes.data, self.h,
                                    MESH[rule] | MASS[mass] | NOISE[noise], C.byref(handle)))
        self.handle = handle.value
        nd, ni = C.c_int64(), C.c_int64()
        offs = np.zeros(self.n_edges + 1, dtype=np.int64)
        _check(lib.grf_graph_info(self.handle, C.byref(nd), C.byref(ni), offs.ctypes.data))
        self.n_dof, self.n_interior, self.offsets = nd.value, ni.value, offs
        import torch

        self.device = torch.cuda.current_device()

    def lumped_mass(self) -> np.ndarray:
        """Diagonal of M_L (float64 [n_dof], canonical order), from the library."""
        ml = np.empty(self.n_dof, dtype=np.float64)
        _check(load().grf_graph_lumped_mass(self.handle, ml.ctypes.data))
        return ml

    @classmethod
    def from_workload(cls, g, h: float, rule: str = "ceil") -> "Graph":
        return cls(g.n_vertices, g.edges, g.lengths, h, rule)

    def close(self):
        if getattr(self, "handle", None):
            load().grf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shift_count(self, beta: float, quad_step: float, k_minus: int = -1, k_plus: int = -1):
        o = make_opts(k_minus=k_minus, k_plus=k_plus, stream=False)
        km, kp, k = C.c_int32(), C.c_int32(), C.c_double()
        _check(load().grf_shift_count(self.handle, beta, quad_step, C.byref(o), C.byref(km), C.byref(kp),
                                      C.byref(k)))
        return km.value, kp.value, k.value

    def noise(self, n_samples: int, seed: int, out=None, **kw):
        import torch

        if out is None:
            out = torch.empty((n_samples, self.n_dof), dtype=torch.float64, device=f"cuda:{self.device}")
        check_array(out, n_samples, self.n_dof, "out", self.device)
        o = make_opts(**kw)
        _check(load().grf_noise(self.handle, n_samples, seed, out.data_ptr(), C.byref(o)))
        return out

    def sample(self, kappa: float, beta: float, quad_step: float, n_samples: int, seed: int, out=None,
               allow_noconv: bool = False, allow_nonfinite: bool = False, **kw):
        """Returns (samples [n_samples, n_dof] float64 on cuda, stats dict)."""
        import torch

        if out is None:
            out = torch.empty((n_samples, self.n_dof), dtype=torch.float64, device=f"cuda:{self.device}")
        check_array(out, n_samples, self.n_dof, "out", self.device)
        st = Stats()
        o = make_opts(stats=st, **kw)
        allow = _allowed(allow_noconv, allow_nonfinite)
        _check(load().grf_sample(self.handle, kappa, beta, quad_step, n_samples, seed, out.data_ptr(), C.byref(o)),
               allow)
        return out, st.as_dict()

    def sample_from_noise(self, kappa: float, beta: float, quad_step: float, noise, out=None,
                          allow_noconv: bool = False, allow_nonfinite: bool = False, **kw):
        """The sample for given noise (float64 [n_samples, n_dof] on cuda, e.g. from
        noise()); returns (samples, stats dict)."""
        import torch

        if not isinstance(noise, torch.Tensor) or noise.dim() != 2:
            raise ValueError("noise must be a 2-d tensor [n_samples, n_dof]")
        n = noise.shape[0]
        check_array(noise, n, self.n_dof, "noise", self.device)
        if out is None:
            out = torch.empty((n, self.n_dof), dtype=torch.float64, device=f"cuda:{self.device}")
        check_array(out, n, self.n_dof, "out", self.device)
        if out.data_ptr() == noise.data_ptr():
            raise ValueError("noise and out may not alias")
        st = Stats()
        o = make_opts(stats=st, **kw)
        allow = _allowed(allow_noconv, allow_nonfinite)
        _check(load().grf_sample_from_noise(self.handle, kappa, beta, quad_step, n, noise.data_ptr(), out.data_ptr(),
                                            C.byref(o)), allow)
        return out, st.as_dict()

    def solve_shifted(self, kappa: float, c_I: float, c_L: float, rhs, out=None, allow_noconv=False,
                      allow_nonfinite=False, **kw):
        import torch

        if not isinstance(rhs, torch.Tensor) or rhs.dim() == 0 or rhs.shape[-1] != self.n_dof:
            raise ValueError(f"rhs must be a tensor [..., {self.n_dof}]")
        rhs = rhs.contiguous()
        r2 = rhs.reshape(-1, self.n_dof)
        check_array(r2, r2.shape[0], self.n_dof, "rhs", self.device)
        if out is None:
            out = torch.empty_like(r2)
        else:
            if not isinstance(out, torch.Tensor) or tuple(out.shape) != tuple(rhs.shape):
                raise ValueError(f"out must have the shape of rhs, {tuple(rhs.shape)}")
            if out.is_contiguous():
                out = out.view(-1, self.n_dof)
        check_array(out, r2.shape[0], self.n_dof, "out", self.device)
        if out.data_ptr() == r2.data_ptr():
            raise ValueError("rhs and out may not alias")
        st = Stats()
        o = make_opts(stats=st, **kw)
        allow = _allowed(allow_noconv, allow_nonfinite)
        _check(load().grf_solve_shifted(self.handle, kappa, c_I, c_L, r2.shape[0], r2.data_ptr(), out.data_ptr(),
                                        C.byref(o)), allow)
        return out.reshape(rhs.shape), st.as_dict()


def sample_batched(graphs, kappas, beta: float, quad_step: float, n_samples: int, seed: int, outs=None, **kw):
    """grf_sample_batched over a list of Graph objects; returns (list of outputs, stats dict)."""
    import torch

    n = len(graphs)
    if outs is None:
        outs = [torch.empty((n_samples, g.n_dof), dtype=torch.float64, device=f"cuda:{g.device}") for g in graphs]
    if len(outs) != n:
        raise ValueError(f"need one output per graph: {len(outs)} outputs for {n} graphs")
    for i, (g, o_) in enumerate(zip(graphs, outs)):
        check_array(o_, n_samples, g.n_dof, f"outs[{i}]", g.device)
    harr = (C.c_void_p * n)(*[g.handle for g in graphs])
    karr = (C.c_double * n)(*[float(k) for k in kappas])
    oarr = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    st = Stats()
    o = make_opts(stats=st, **kw)
    _check(load().grf_sample_batched(harr, n, karr, beta, quad_step, n_samples, seed, oarr, C.byref(o)))
    return outs, st.as_dict()


class Learned:
    """The learned vertex preconditioner (network parameters on the device)."""

    def __init__(self, params):
        lib = load()
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        handle = C.c_void_p()
        _check(lib.grf_learned_create(p.ctypes.data, p.size, C.byref(handle)))
        self.handle = handle.value
        self.n_params = p.size

    @staticmethod
    def param_count() -> int:
        n = C.c_int64()
        _check(load().grf_learned_param_count(C.byref(n)))
        return n.value

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(load().grf_learned_params(self.handle, out.ctypes.data, out.size))
        return out

    def loss_grad(self, graph, kappa: float, c_I: float, c_L: float, rhs, sol, **kw):
        """rhs, sol: device float64 tensors [n_rhs][V]; returns (loss, grad numpy float32)."""
        n = rhs.shape[0] if hasattr(rhs, "shape") and len(rhs.shape) == 2 else -1
        check_array(rhs, n, graph.n_vertices, "rhs", graph.device)
        check_array(sol, n, graph.n_vertices, "sol", graph.device)
        loss = C.c_double()
        grad = np.zeros(self.n_params, dtype=np.float32)
        o = make_opts(**kw)
        _check(load().grf_learned_loss_grad(self.handle, graph.handle, kappa, c_I, c_L, rhs.shape[0],
                                            rhs.data_ptr(), sol.data_ptr(), C.byref(loss), grad.ctypes.data,
                                            C.byref(o)))
        return loss.value, grad

    def operators(self, graph, kappa: float, c_I: float, c_L: float, activations: str = "bf16", **kw):
        """The network's operators for one shift: device float64 tensors (P_hat diagonal [V],
        P_hat edge couplings [E], Q_hat diagonal [V], Q_hat edge couplings [E])."""
        import torch

        dev = f"cuda:{graph.device}"
        V, E = graph.n_vertices, graph.n_edges
        pd, qd = (torch.empty(V, dtype=torch.float64, device=dev) for _ in range(2))
        pe, qe = (torch.empty(max(E, 1), dtype=torch.float64, device=dev) for _ in range(2))
        o = make_opts(**kw)
        _check(load().grf_learned_operators(self.handle, graph.handle, kappa, c_I, c_L, ACTIVATIONS[activations],
                                            pd.data_ptr(), pe.data_ptr(), qd.data_ptr(), qe.data_ptr(), C.byref(o)))
        return pd, pe[:E], qd, qe[:E]

    def train(self, graphs, kappas, beta: float, quad_step: float, n_samples: int, seed: int, n_steps: int,
              shifts_per_step: int = 16, lr: float = 1e-3, **kw) -> np.ndarray:
        n = len(graphs)
        harr = (C.c_void_p * n)(*[g.handle for g in graphs])
        karr = (C.c_double * n)(*[float(k) for k in kappas])
        losses = np.zeros(max(1, n_steps), dtype=np.float64)
        o = make_opts(**kw)
        _check(load().grf_learned_train(self.handle, harr, n, karr, beta, quad_step, n_samples, seed, n_steps,
                                        shifts_per_step, lr, losses.ctypes.data, C.byref(o)))
        return losses[:n_steps]

    def close(self):
        if getattr(self, "handle", None):
            load().grf_learned_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
