"""The C-ABI library loads and exports every function include/pd.h declares;
host-side validation (no GPU needed: these calls queue no device work)."""
import ctypes
import os
import re

import pytest

from paper_1711_05095_amd import guide_net, pd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header="pd.h", prefix="pd_"):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^(?:pd_status|const char\*)\s+(%s\w+)\(" % prefix, text,
                                 re.M)))


def test_header_and_binding_agree():
    assert declared() == sorted(pd.EXPORTS)
    assert declared("pd_guide.h", "pdg_") == sorted(guide_net.EXPORTS)


def test_library_exports_every_symbol():
    lib = pd.lib()
    for name in declared() + declared("pd_guide.h", "pdg_"):
        assert hasattr(lib, name), name


def test_guide_constants_match_header():
    text = open(os.path.join(ROOT, "include", "pd_guide.h")).read()
    for name in ("PDG_PARAMS", "PDG_WINDOWS", "PDG_MIN_L", "PDG_MAX_GMAX", "PDG_COND_MIN_L",
                 "PDG_COND_WORK_BYTES"):
        v = re.search(r"#define %s ([0-9.]+)" % name, text).group(1)
        assert float(v) == getattr(guide_net, name), name
    from oracle import guide_net as ref
    assert guide_net.PDG_PARAMS == ref.PARAMS


def test_guide_host_validation():
    """Invalid arguments are rejected before any device work is queued."""
    lib = guide_net.lib()
    vp = ctypes.c_void_p
    out = ctypes.c_size_t()
    assert lib.pdg_workspace_bytes(0, ctypes.byref(out)) == pd.PD_EINVAL
    assert lib.pdg_workspace_bytes(100, ctypes.byref(out)) == pd.PD_OK
    assert out.value == 100 * (guide_net.PDG_PARAMS + 1) * 4
    assert lib.pdg_workspace_bytes(10**6, ctypes.byref(out)) == pd.PD_OK
    assert out.value == 768 * (guide_net.PDG_PARAMS + 1) * 4
    fake = vp(4096)
    assert lib.pdg_forward(fake, fake, 10, 4, 10, fake, None) == pd.PD_EINVAL  # L < 5
    assert lib.pdg_forward(fake, fake, 10, 513, 10, fake, None) == pd.PD_EINVAL
    assert lib.pdg_forward(fake, fake, 10, 20, 0, fake, None) == pd.PD_EINVAL
    assert lib.pdg_forward(fake, fake, 9, 20, 10, fake, None) == pd.PD_EINVAL   # ld < n
    assert lib.pdg_forward(None, fake, 10, 20, 10, fake, None) == pd.PD_EINVAL
    assert lib.pdg_loss_grad(fake, fake, 10, fake, 20, 10, fake, None, vp(4097), 1 << 30,
                             None) == pd.PD_EINVAL                             # misaligned
    assert lib.pdg_loss_grad(fake, fake, 10, fake, 20, 10, fake, None, fake, 100,
                             None) == pd.PD_ENOMEM
    assert b"too small" in lib.pdg_last_error()
    assert lib.pdg_adam(fake, fake, fake, fake, 0, 1e-3, None) == pd.PD_EINVAL
    assert lib.pdg_adam(fake, fake, fake, fake, 1, -1.0, None) == pd.PD_EINVAL
    W = 1 << 30
    te = lib.pdg_train_epoch
    assert te(fake, fake, fake, fake, 10, fake, 20, 10, 0, 0, 1e-3, fake, fake, W,
              None) == pd.PD_EINVAL                                            # batch < 1
    assert te(fake, fake, fake, fake, 10, fake, 20, 10, 4, -1, 1e-3, fake, fake, W,
              None) == pd.PD_EINVAL                                            # step0 < 0
    assert te(fake, fake, fake, fake, 10, fake, 20, 10, 4, 0, 0.0, fake, fake, W,
              None) == pd.PD_EINVAL                                            # lr <= 0
    assert te(fake, fake, fake, fake, 10, fake, 20, 10, 4, 0, 1e-3, None, fake, W,
              None) == pd.PD_EINVAL                                            # loss_sum
    assert te(fake, fake, fake, fake, 10, fake, 20, 10, 4, 0, 1e-3, fake, vp(4097), W,
              None) == pd.PD_EINVAL                                            # misaligned
    assert te(fake, fake, fake, fake, 10, fake, 4, 10, 4, 0, 1e-3, fake, fake, W,
              None) == pd.PD_EINVAL                                            # L < 5
    need = ctypes.c_size_t()
    assert lib.pdg_workspace_bytes(4, ctypes.byref(need)) == pd.PD_OK
    assert te(fake, fake, fake, fake, 10, fake, 20, 10, 4, 0, 1e-3, fake, fake,
              need.value - 1, None) == pd.PD_ENOMEM                            # min(batch, n)
    assert lib.pdg_bond_table(fake, 3.5, fake, None, None) == pd.PD_EINVAL
    assert lib.pdg_bond_table(fake, float("nan"), fake, None, None) == pd.PD_EINVAL
    assert lib.pdg_window_table(None, fake, None) == pd.PD_EINVAL
    big = guide_net.PDG_COND_WORK_BYTES
    assert lib.pdg_bond_table_cond(fake, fake, 10, 25, 10, 1, 1.0, fake, None, None, fake, big,
                                   None) == pd.PD_EINVAL                       # L < 26
    assert lib.pdg_bond_table_cond(fake, fake, 10, 40, 10, 0, 1.0, fake, None, None, fake, big,
                                   None) == pd.PD_EINVAL                       # min_count 0
    assert lib.pdg_bond_table_cond(fake, fake, 10, 40, 10, 1, 1.0, fake, None, None, fake,
                                   big - 1, None) == pd.PD_ENOMEM


def test_status_strings():
    assert pd.lib().pd_status_str(pd.PD_EINVAL) == b"invalid argument"


def good(**kw):
    base = dict(L=100, N=50, s=0.002, Nc=100_000, t_obs=2000.0, dt=0.5)
    base.update(kw)
    return pd.make_params(**base)


def test_workspace_bytes_scales():
    small = pd.pd_workspace_bytes(good(Nc=1000))
    big = pd.pd_workspace_bytes(good())
    # two state buffers of 2 words, two K buffers, K^beta, A, ln Ups, ancestor
    per_clone = (big - small) / 99_000
    assert 2 * 16 + 16 + 4 + 8 + 8 + 4 <= per_clone <= 2 * 16 + 16 + 4 + 8 + 8 + 4 + 2
    batch = pd.pd_workspace_bytes([good(), good(L=400, N=200)])
    assert batch > big


@pytest.mark.parametrize("kw", [dict(L=1), dict(L=513), dict(N=-1), dict(N=101),
                                dict(s=float("nan")), dict(s=701.0), dict(s=-30.0), dict(dt=1e6, t_obs=1e6), dict(Nc=0), dict(Nc=2**31),
                                dict(dt=0.0), dict(t_obs=-1.0), dict(t_obs=1000.25, dt=0.5),
                                dict(selection=7), dict(weight_mode=9),
                                dict(instance=1 << 24), dict(log_cycles=-1), dict(burn_in=-2)])
def test_invalid_parameters_rejected(kw):
    with pytest.raises(pd.PdError) as e:
        pd.pd_workspace_bytes(good(**kw))
    assert e.value.status == pd.PD_EINVAL


def test_create_rejects_without_device_work():
    p = good()
    arr = (pd.PdParams * 1)(p)
    ctx = ctypes.c_void_p()
    # null workspace: rejected before anything touches the GPU
    assert pd.lib().pd_create(arr, 1, None, 0, None, ctypes.byref(ctx)) == pd.PD_EINVAL
    # misaligned workspace pointer
    assert pd.lib().pd_create(arr, 1, ctypes.c_void_p(8), 1 << 40, None,
                              ctypes.byref(ctx)) == pd.PD_EINVAL


def test_context_calls_reject_a_null_context():
    """Calls on a context return PD_EINVAL for a null one, before anything
    reaches the GPU."""
    lib = pd.lib()
    fake = ctypes.c_void_p(256)
    assert lib.pd_histogram(None, 0, fake, 0, 0.0, 1.0, 10, fake) == pd.PD_EINVAL
    m = ctypes.c_double()
    assert lib.pd_mean(None, 0, fake, 0, ctypes.byref(m)) == pd.PD_EINVAL
    assert lib.pd_density_mode(None, 0, 1, fake) == pd.PD_EINVAL
