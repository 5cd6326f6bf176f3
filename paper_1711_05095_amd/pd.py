"""Python binding of the C ABI in include/pd.h (argument marshalling only).

Every function here converts arguments and calls the function of the same
name in libpd.so; all computation runs in the library's HIP kernels.  Device
memory and streams come from PyTorch.  There is no CPU fallback: importing
works without a GPU, but the first call raises if libpd.so is missing or no
GPU is visible.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpd.so")

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EDEVICE, PD_ESTATE, PD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PD_SEL_EQ, PD_SEL_IID = 0, 1
PD_W_MODIFIED, PD_W_DIRECT, PD_W_GUIDED = 0, 1, 2
PD_MAX_L = 512

# Exported functions of include/pd.h (the ABI test checks each one is present).
EXPORTS = ["pd_workspace_bytes", "pd_create", "pd_destroy", "pd_step", "pd_resample", "pd_run",
           "pd_scgf", "pd_estimates_get", "pd_hop_counts", "pd_population_bytes",
           "pd_get_population", "pd_set_population", "pd_get_step_outputs", "pd_get_ancestors",
           "pd_get_log", "pd_save_bytes", "pd_save", "pd_load", "pd_set_guide", "pd_reset_origin",
           "pd_get_origin", "pd_descendant_counts", "pd_density_mode", "pd_mean",
           "pd_histogram", "pd_get_tuning", "pd_set_tuning", "pd_autotune", "pd_time_stages",
           "pd_get_stage_times", "pd_last_error", "pd_status_str"]


class PdParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("N", ctypes.c_int32), ("s", ctypes.c_double),
                ("Nc", ctypes.c_int64), ("t_obs", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("selection", ctypes.c_int32),
                ("weight_mode", ctypes.c_int32), ("instance", ctypes.c_uint32),
                ("log_cycles", ctypes.c_int32), ("burn_in", ctypes.c_int64),
                ("track_origin", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PdEstimates(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_double), ("psi_burn", ctypes.c_double),
                ("k_hat", ctypes.c_double), ("t", ctypes.c_double), ("cycles", ctypes.c_int64),
                ("hops", ctypes.c_uint64), ("k_hat_burn", ctypes.c_double),
                ("draws", ctypes.c_uint64)]


class PdStageTimes(ctypes.Structure):
    _fields_ = [("step_ms", ctypes.c_double), ("prefix_ms", ctypes.c_double),
                ("resample_ms", ctypes.c_double), ("steps", ctypes.c_int64),
                ("resamples", ctypes.c_int64)]


class PdTuning(ctypes.Structure):
    _fields_ = [("step_variant", ctypes.c_int32), ("refill", ctypes.c_int32),
                ("graph_cycles", ctypes.c_int32), ("scan_tiles", ctypes.c_int32)]


class PdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d)" % (message, status))
        self.status = status


_lib = None


def lib():
    """The loaded libpd.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpd.so is not built; run `python -m paper_1711_05095_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        P = c.POINTER
        vp = c.c_void_p
        sig = {
            "pd_workspace_bytes": [P(PdParams), c.c_int32, P(c.c_size_t)],
            "pd_create": [P(PdParams), c.c_int32, vp, c.c_size_t, vp, P(vp)],
            "pd_destroy": [vp],
            "pd_step": [vp],
            "pd_resample": [vp],
            "pd_run": [vp, c.c_int64],
            "pd_scgf": [vp, P(c.c_double), P(c.c_double), P(c.c_int64)],
            "pd_estimates_get": [vp, c.c_int32, P(PdEstimates)],
            "pd_population_bytes": [P(PdParams), P(c.c_size_t)],
            "pd_get_population": [vp, c.c_int32, vp, c.c_size_t],
            "pd_set_population": [vp, c.c_int32, vp, c.c_size_t],
            "pd_get_step_outputs": [vp, c.c_int32, vp, vp, vp],
            "pd_get_ancestors": [vp, c.c_int32, vp],
            "pd_get_log": [vp, c.c_int32, vp, vp, c.c_int32],
            "pd_save_bytes": [vp, P(c.c_size_t)],
            "pd_save": [vp, vp, c.c_size_t],
            "pd_load": [vp, vp, c.c_size_t],
            "pd_set_guide": [vp, vp, c.c_size_t],
            "pd_reset_origin": [vp, c.c_int32],
            "pd_get_origin": [vp, c.c_int32, vp],
            "pd_descendant_counts": [vp, c.c_int32, vp],
            "pd_hop_counts": [vp, vp],
            "pd_density_mode": [vp, c.c_int32, c.c_int32, vp],
            "pd_mean": [vp, c.c_int32, vp, c.c_int32, P(c.c_double)],
            "pd_histogram": [vp, c.c_int32, vp, c.c_int32, c.c_double, c.c_double, c.c_int32, vp],
            "pd_get_tuning": [vp, P(PdTuning)],
            "pd_set_tuning": [vp, P(PdTuning)],
            "pd_autotune": [vp, c.c_int32, P(PdTuning)],
            "pd_time_stages": [vp, c.c_int32],
            "pd_get_stage_times": [vp, P(PdStageTimes)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c.c_int
        L.pd_last_error.argtypes = [vp]
        L.pd_last_error.restype = c.c_char_p
        L.pd_status_str.argtypes = [c.c_int]
        L.pd_status_str.restype = c.c_char_p
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != PD_OK:
        msg = lib().pd_last_error(ctx).decode()
        raise PdError(status, msg or lib().pd_status_str(status).decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def make_params(L, N, s, Nc, t_obs, dt, seed=0, selection=PD_SEL_EQ, weight_mode=PD_W_MODIFIED,
                instance=0, log_cycles=0, burn_in=0, track_origin=0):
    return PdParams(L=L, N=N, s=float(s), Nc=int(Nc), t_obs=float(t_obs), dt=float(dt),
                    seed=int(seed), selection=selection, weight_mode=weight_mode,
                    instance=instance, log_cycles=log_cycles, burn_in=int(burn_in),
                    track_origin=int(track_origin), reserved=0)


def _param_array(params):
    if isinstance(params, PdParams):
        params = [params]
    arr = (PdParams * len(params))(*params)
    return arr, len(params)


def pd_workspace_bytes(params):
    arr, n = _param_array(params)
    out = ctypes.c_size_t()
    _check(lib().pd_workspace_bytes(arr, n, ctypes.byref(out)))
    return out.value


def pd_create(params, workspace_ptr, workspace_bytes, stream_handle):
    arr, n = _param_array(params)
    ctx = ctypes.c_void_p()
    _check(lib().pd_create(arr, n, ctypes.c_void_p(workspace_ptr), workspace_bytes,
                           ctypes.c_void_p(stream_handle), ctypes.byref(ctx)))
    return ctx


def pd_destroy(ctx):
    _check(lib().pd_destroy(ctx))


def pd_step(ctx):
    _check(lib().pd_step(ctx), ctx)


def pd_resample(ctx):
    _check(lib().pd_resample(ctx), ctx)


def pd_run(ctx, cycles):
    _check(lib().pd_run(ctx, int(cycles)), ctx)


def pd_scgf(ctx):
    psi, kh, cy = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().pd_scgf(ctx, ctypes.byref(psi), ctypes.byref(kh), ctypes.byref(cy)), ctx)
    return psi.value, kh.value, cy.value


def pd_estimates_get(ctx, inst=0):
    e = PdEstimates()
    _check(lib().pd_estimates_get(ctx, inst, ctypes.byref(e)), ctx)
    return dict(psi=e.psi, psi_burn=e.psi_burn, k_hat=e.k_hat, k_hat_burn=e.k_hat_burn, t=e.t,
                cycles=e.cycles, hops=e.hops, draws=e.draws)


def words_of(L):
    return (L + 63) // 64


def pd_get_population(ctx, inst, L, Nc):
    """Returns (words uint64 [W, Nc], K uint64 [Nc])."""
    W = words_of(L)
    buf = np.empty((W + 1) * Nc, np.uint64)
    _check(lib().pd_get_population(ctx, inst, _ptr(buf), buf.nbytes), ctx)
    return buf[:W * Nc].reshape(W, Nc).copy(), buf[W * Nc:].copy()


def pd_set_population(ctx, inst, words, K):
    words = np.ascontiguousarray(words, np.uint64)
    buf = np.concatenate([words.reshape(-1), np.ascontiguousarray(K, np.uint64)])
    _check(lib().pd_set_population(ctx, inst, _ptr(buf), buf.nbytes), ctx)


def pd_get_step_outputs(ctx, inst, Nc):
    Kb = np.empty(Nc, np.uint32)
    A = np.empty(Nc, np.float64)
    ell = np.empty(Nc, np.float64)
    _check(lib().pd_get_step_outputs(ctx, inst, _ptr(Kb), _ptr(A), _ptr(ell)), ctx)
    return Kb, A, ell


def pd_get_ancestors(ctx, inst, Nc):
    anc = np.empty(Nc, np.int32)
    _check(lib().pd_get_ancestors(ctx, inst, _ptr(anc)), ctx)
    return anc


def pd_get_log(ctx, inst, n_rows):
    lb = np.empty(n_rows, np.float64)
    mk = np.empty(n_rows, np.float64)
    _check(lib().pd_get_log(ctx, inst, _ptr(lb), _ptr(mk), n_rows), ctx)
    return lb, mk


def pd_save(ctx):
    n = ctypes.c_size_t()
    _check(lib().pd_save_bytes(ctx, ctypes.byref(n)), ctx)
    buf = np.empty(n.value, np.uint8)
    _check(lib().pd_save(ctx, _ptr(buf), buf.nbytes), ctx)
    return buf


def pd_load(ctx, blob):
    blob = np.ascontiguousarray(blob, np.uint8)
    _check(lib().pd_load(ctx, _ptr(blob), blob.nbytes), ctx)


def pd_reset_origin(ctx, inst=0):
    _check(lib().pd_reset_origin(ctx, inst), ctx)


def pd_get_origin(ctx, inst, Nc):
    out = np.empty(Nc, np.int32)
    _check(lib().pd_get_origin(ctx, inst, _ptr(out)), ctx)
    return out


def pd_hop_counts(ctx, hops_ptr):
    _check(lib().pd_hop_counts(ctx, ctypes.c_void_p(hops_ptr)), ctx)


def pd_descendant_counts(ctx, inst, counts_ptr):
    _check(lib().pd_descendant_counts(ctx, inst, ctypes.c_void_p(counts_ptr)), ctx)


def pd_density_mode(ctx, inst, n, out_ptr):
    _check(lib().pd_density_mode(ctx, inst, int(n), ctypes.c_void_p(out_ptr)), ctx)


def pd_histogram(ctx, inst, values_ptr, ancestral, lo, width, nbins, counts_ptr):
    _check(lib().pd_histogram(ctx, inst, ctypes.c_void_p(values_ptr), int(ancestral), float(lo),
                              float(width), int(nbins), ctypes.c_void_p(counts_ptr)), ctx)


def pd_mean(ctx, inst, values_ptr, ancestral):
    m = ctypes.c_double()
    _check(lib().pd_mean(ctx, inst, ctypes.c_void_p(values_ptr), int(ancestral),
                         ctypes.byref(m)), ctx)
    return m.value


def _tuning_dict(t):
    return dict(step_variant=t.step_variant, refill=t.refill, graph_cycles=t.graph_cycles,
                scan_tiles=t.scan_tiles)


def pd_get_tuning(ctx):
    t = PdTuning()
    _check(lib().pd_get_tuning(ctx, ctypes.byref(t)), ctx)
    return _tuning_dict(t)


def pd_set_tuning(ctx, step_variant, refill, graph_cycles, scan_tiles=1):
    t = PdTuning(step_variant=step_variant, refill=refill, graph_cycles=graph_cycles,
                 scan_tiles=scan_tiles)
    _check(lib().pd_set_tuning(ctx, ctypes.byref(t)), ctx)


def pd_autotune(ctx, trial_cycles):
    t = PdTuning()
    _check(lib().pd_autotune(ctx, int(trial_cycles), ctypes.byref(t)), ctx)
    return _tuning_dict(t)


def pd_time_stages(ctx, enable):
    _check(lib().pd_time_stages(ctx, 1 if enable else 0), ctx)


def pd_get_stage_times(ctx):
    t = PdStageTimes()
    _check(lib().pd_get_stage_times(ctx, ctypes.byref(t)), ctx)
    return dict(step_ms=t.step_ms, prefix_ms=t.prefix_ms, resample_ms=t.resample_ms,
                steps=t.steps, resamples=t.resamples)


def pd_set_guide(ctx, table_ptr, n):
    _check(lib().pd_set_guide(ctx, ctypes.c_void_p(table_ptr), n), ctx)


class Sampler:
    """A context together with the torch buffer that backs its workspace.

    params: one PdParams or a list (a batch of instances).  The workspace is
    allocated with torch on `device`, and work is queued on torch's current
    stream of that device (or `stream`)."""

    def __init__(self, params, device="cuda", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the sampler runs only on the GPU")
        arr, n = _param_array(params)
        self.params = list(arr)
        self.n = n
        nbytes = pd_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        # a stream of its own (default priority): graphs cannot be captured on
        # the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        self.ctx = pd_create(self.params, self.workspace.data_ptr(), nbytes,
                             self.stream.cuda_stream)

    def close(self):
        if self.ctx is not None:
            pd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        pd_step(self.ctx)

    def resample(self):
        pd_resample(self.ctx)

    def run(self, cycles):
        pd_run(self.ctx, cycles)

    def scgf(self):
        return pd_scgf(self.ctx)

    def estimates(self, inst=0):
        return pd_estimates_get(self.ctx, inst)

    def get_population(self, inst=0):
        p = self.params[inst]
        return pd_get_population(self.ctx, inst, p.L, p.Nc)

    def set_population(self, words, K, inst=0):
        pd_set_population(self.ctx, inst, words, K)

    def step_outputs(self, inst=0):
        return pd_get_step_outputs(self.ctx, inst, self.params[inst].Nc)

    def ancestors(self, inst=0):
        return pd_get_ancestors(self.ctx, inst, self.params[inst].Nc)

    def log(self, n_rows, inst=0):
        return pd_get_log(self.ctx, inst, n_rows)

    def save(self):
        return pd_save(self.ctx)

    def load(self, blob):
        pd_load(self.ctx, blob)

    def set_guide(self, table):
        """table: a torch uint32-compatible int32 CUDA tensor of 8192 entries;
        the library keeps a copy (a refused table leaves the previous one in
        use)."""
        # the library reads the table on its own stream
        import torch
        torch.cuda.current_stream().synchronize()
        pd_set_guide(self.ctx, table.data_ptr(), table.numel())

    def reset_origin(self, inst=0):
        pd_reset_origin(self.ctx, inst)

    def origin(self, inst=0):
        return pd_get_origin(self.ctx, inst, self.params[inst].Nc)

    def hop_counts(self, out):
        """Queues a copy of every instance's hop count into `out` (an int64
        CUDA tensor of n entries, read as uint64) on the sampler's stream, with
        no synchronisation (the stream first waits for torch's current stream,
        where `out` was allocated)."""
        import torch
        assert out.is_cuda and out.dtype.itemsize == 8 and out.numel() >= self.n
        self.stream.wait_stream(torch.cuda.current_stream())
        pd_hop_counts(self.ctx, out.data_ptr())

    def descendant_counts(self, inst=0):
        """Descendants of each slot of the last origin reset among the current
        clones, as an int32 CUDA tensor of Nc entries (uint32 counts), written
        on the sampler's stream and complete on return."""
        import torch
        out = torch.empty(self.params[inst].Nc, dtype=torch.int32, device=self.workspace.device)
        torch.cuda.current_stream().synchronize()   # the allocation is ordered on torch's stream
        pd_descendant_counts(self.ctx, inst, out.data_ptr())
        self.stream.synchronize()
        return out

    def density_mode(self, n, inst=0):
        """|delta rho_n|^2 of every clone (slot order) as a float64 CUDA tensor."""
        import torch
        out = torch.empty(self.params[inst].Nc, dtype=torch.float64, device=self.workspace.device)
        torch.cuda.current_stream().synchronize()   # the allocation is ordered on torch's stream
        pd_density_mode(self.ctx, inst, n, out.data_ptr())
        self.stream.synchronize()                   # written on the sampler's stream
        return out

    def mean(self, values, ancestral=False, inst=0):
        """(1/Nc) sum_j values[j], or values[origin_j] when ancestral; values is
        a float64 CUDA tensor of Nc entries."""
        import torch
        if values.dtype != torch.float64 or not values.is_cuda or not values.is_contiguous() \
                or values.numel() < self.params[inst].Nc:
            raise TypeError("values must be a contiguous float64 CUDA tensor of Nc entries")
        # the library reads values on its own stream
        torch.cuda.current_stream().synchronize()
        return pd_mean(self.ctx, inst, values.data_ptr(), 1 if ancestral else 0)

    def histogram(self, values, lo, width, nbins, ancestral=False, inst=0):
        """Counts of floor((v_j - lo) / width) in bins 0..nbins-1 over the clones,
        v_j = values[j], or values[origin_j] when ancestral; values is a float64
        CUDA tensor of Nc entries.  Returns a numpy uint64 array."""
        import torch
        if values.dtype != torch.float64 or not values.is_cuda or not values.is_contiguous() \
                or values.numel() < self.params[inst].Nc:
            raise TypeError("values must be a contiguous float64 CUDA tensor of Nc entries")
        counts = torch.empty(max(int(nbins), 1), dtype=torch.int64, device=values.device)
        torch.cuda.current_stream().synchronize()   # values and counts, on torch's stream
        pd_histogram(self.ctx, inst, values.data_ptr(), 1 if ancestral else 0, lo, width, nbins,
                     counts.data_ptr())
        self.stream.synchronize()                   # written on the sampler's stream
        return counts.cpu().numpy().view(np.uint64)

    def tuning(self):
        return pd_get_tuning(self.ctx)

    def set_tuning(self, step_variant, refill=13, graph_cycles=16, scan_tiles=1):
        pd_set_tuning(self.ctx, step_variant, refill, graph_cycles, scan_tiles)

    def autotune(self, trial_cycles=3):
        return pd_autotune(self.ctx, trial_cycles)

    def time_stages(self, enable=True):
        pd_time_stages(self.ctx, enable)

    def stage_times(self):
        return pd_get_stage_times(self.ctx)
