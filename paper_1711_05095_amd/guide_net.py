"""Python binding of include/pd_guide.h (argument marshalling only).

The functions take torch CUDA tensors and call the function of the same name
in libpd.so, which queues the HIP kernels on the given stream (default:
torch's current stream).  Nothing is computed here.
"""
import ctypes

from . import pd

PDG_PARAMS = 5506
PDG_WINDOWS = 8192
PDG_MIN_L = 5
PDG_MAX_GMAX = 3.45
PDG_COND_MIN_L = 26
PDG_COND_WORK_BYTES = 163840

EXPORTS = ["pdg_workspace_bytes", "pdg_forward", "pdg_loss_grad", "pdg_adam", "pdg_train_epoch",
           "pdg_window_table", "pdg_bond_table", "pdg_bond_table_cond",
           "pdg_bond_table_cond_noalloc", "pdg_last_error"]

_bound = False


def lib():
    global _bound
    L = pd.lib()
    if not _bound:
        c = ctypes
        vp = c.c_void_p
        sig = {
            "pdg_workspace_bytes": [c.c_int64, c.POINTER(c.c_size_t)],
            "pdg_forward": [vp, vp, c.c_int64, c.c_int32, c.c_int64, vp, vp],
            "pdg_loss_grad": [vp, vp, c.c_int64, vp, c.c_int32, c.c_int64, vp, vp, vp, c.c_size_t,
                              vp],
            "pdg_adam": [vp, vp, vp, vp, c.c_int32, c.c_float, vp],
            "pdg_train_epoch": [vp, vp, vp, vp, c.c_int64, vp, c.c_int32, c.c_int64, c.c_int64,
                                c.c_int32, c.c_float, vp, vp, c.c_size_t, vp],
            "pdg_window_table": [vp, vp, vp],
            "pdg_bond_table": [vp, c.c_double, vp, vp, vp],
            "pdg_bond_table_cond": [vp, vp, c.c_int64, c.c_int32, c.c_int64, c.c_int32, c.c_double,
                                    vp, vp, vp, vp, c.c_size_t, vp],
            "pdg_bond_table_cond_noalloc": [vp, vp, c.c_int64, c.c_int32, c.c_int64, c.c_int32,
                                            c.c_double, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c.c_int
        L.pdg_last_error.argtypes = []
        L.pdg_last_error.restype = c.c_char_p
        _bound = True
    return L


def _check(status):
    if status != pd.PD_OK:
        msg = lib().pdg_last_error().decode()
        raise pd.PdError(status, msg or lib().pd_status_str(status).decode())


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous CUDA %s tensor" % (name, dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d entries, needs %d" % (name, t.numel(), numel))
    return t


def _states(states, L):
    """states: int64/uint64 CUDA tensor [W, n] (pd_get_population layout),
    possibly a column slice of a wider array (unit stride along columns).
    Returns (n, ld)."""
    import torch
    if states.dtype not in (torch.int64, torch.uint64) or not states.is_cuda or states.dim() != 2:
        raise TypeError("states must be a CUDA 64-bit tensor [W, n]")
    if states.shape[0] != (L + 63) // 64:
        raise ValueError("states has %d words per configuration, L=%d needs %d"
                         % (states.shape[0], L, (L + 63) // 64))
    n = states.shape[1]
    if states.stride(1) != 1 or (states.shape[0] > 1 and states.stride(0) < n):
        raise TypeError("states must have unit column stride and row stride >= n")
    ld = states.stride(0) if states.shape[0] > 1 else n
    return n, ld


def workspace_bytes(n):
    out = ctypes.c_size_t()
    _check(lib().pdg_workspace_bytes(int(n), ctypes.byref(out)))
    return out.value


def forward(theta, states, L, f_out, stream=None):
    import torch
    n, ld = _states(states, L)
    _dev(theta, torch.float32, PDG_PARAMS, "theta")
    _dev(f_out, torch.float32, n, "f_out")
    _check(lib().pdg_forward(_p(theta), _p(states), ld, L, n, _p(f_out), _stream(stream)))


def loss_grad(theta, states, counts, L, grad, loss, work, stream=None):
    import torch
    n, ld = _states(states, L)
    _dev(theta, torch.float32, PDG_PARAMS, "theta")
    _dev(counts, torch.float32, n, "counts")
    _dev(grad, torch.float32, PDG_PARAMS, "grad")
    if loss is not None:
        _dev(loss, torch.float32, 1, "loss")
    _dev(work, torch.uint8, None, "work")
    _check(lib().pdg_loss_grad(_p(theta), _p(states), ld, _p(counts), L, n, _p(grad), _p(loss),
                               _p(work), work.numel(), _stream(stream)))


def adam(theta, m, v, grad, step, lr, stream=None):
    import torch
    for t, nm in ((theta, "theta"), (m, "m"), (v, "v"), (grad, "grad")):
        _dev(t, torch.float32, PDG_PARAMS, nm)
    _check(lib().pdg_adam(_p(theta), _p(m), _p(v), _p(grad), int(step), float(lr),
                          _stream(stream)))


def train_epoch(theta, m, v, states, counts, L, batch, step0, lr, loss_sum, work, stream=None):
    """Minibatches of `batch` columns, one Adam step each (step numbers
    step0 + 1, ...); minibatch losses added to loss_sum (float64 CUDA tensor,
    one entry).  Returns the number of minibatches (steps taken)."""
    import torch
    n, ld = _states(states, L)
    for t, nm in ((theta, "theta"), (m, "m"), (v, "v")):
        _dev(t, torch.float32, PDG_PARAMS, nm)
    _dev(counts, torch.float32, n, "counts")
    _dev(loss_sum, torch.float64, 1, "loss_sum")
    _dev(work, torch.uint8, None, "work")
    _check(lib().pdg_train_epoch(_p(theta), _p(m), _p(v), _p(states), ld, _p(counts), L, n,
                                 int(batch), int(step0), float(lr), _p(loss_sum), _p(work),
                                 work.numel(), _stream(stream)))
    return (n + int(batch) - 1) // int(batch)


def window_table(theta, table, stream=None):
    import torch
    _dev(theta, torch.float32, PDG_PARAMS, "theta")
    _dev(table, torch.float32, PDG_WINDOWS, "table")
    _check(lib().pdg_window_table(_p(theta), _p(table), _stream(stream)))


def bond_table(window, gmax, eg, G=None, stream=None):
    import torch
    _dev(window, torch.float32, PDG_WINDOWS, "window")
    _dev(eg, torch.int32, PDG_WINDOWS, "eg")
    if G is not None:
        _dev(G, torch.float64, PDG_WINDOWS, "G")
    _check(lib().pdg_bond_table(_p(window), float(gmax), _p(eg), _p(G), _stream(stream)))


def bond_table_cond(window, states, L, min_count, gmax, eg, G=None, counts=None, work=None,
                    stream=None):
    import torch
    n, ld = _states(states, L)
    _dev(window, torch.float32, PDG_WINDOWS, "window")
    _dev(eg, torch.int32, PDG_WINDOWS, "eg")
    if G is not None:
        _dev(G, torch.float64, PDG_WINDOWS, "G")
    if counts is not None:
        _dev(counts, torch.int32, PDG_WINDOWS, "counts")
    if work is None:
        work = torch.empty(PDG_COND_WORK_BYTES, dtype=torch.uint8, device=window.device)
    _dev(work, torch.uint8, None, "work")
    _check(lib().pdg_bond_table_cond(_p(window), _p(states), ld, L, n, int(min_count),
                                     float(gmax), _p(eg), _p(G), _p(counts), _p(work),
                                     work.numel(), _stream(stream)))
    return work


def bond_table_cond_noalloc(window, states, L, min_count, gmax, eg, G=None, counts=None,
                            stream=None):
    """bond_table_cond with the library's own scratch (no workspace argument)."""
    import torch
    n, ld = _states(states, L)
    _dev(window, torch.float32, PDG_WINDOWS, "window")
    _dev(eg, torch.int32, PDG_WINDOWS, "eg")
    if G is not None:
        _dev(G, torch.float64, PDG_WINDOWS, "G")
    if counts is not None:
        _dev(counts, torch.int32, PDG_WINDOWS, "counts")
    _check(lib().pdg_bond_table_cond_noalloc(_p(window), _p(states), ld, L, n, int(min_count),
                                             float(gmax), _p(eg), _p(G), _p(counts),
                                             _stream(stream)))
