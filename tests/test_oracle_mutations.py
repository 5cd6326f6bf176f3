"""Planted mistakes.  Each case compiles a copy of oracle/oracle.c with one
plausible mistake (a dropped term or factor, a wrong sign, index, constant or
comparison) and runs the oracle's pins against that copy in a fresh process
(PD_ORACLE_LIB names the copy); some pin must fail.  The control case compiles
the unmodified source the same way and must pass, so a failure is the
mistake's.  The tracked source is never modified.

One plausible mistake is not here because no pin can see it: drawing the
uniform variate in [0, 1) instead of (0, 1] changes one value in 2^53."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
PLAIN = ["tests/test_oracle_dynamics.py", "tests/test_oracle_selection.py",
         "tests/test_oracle_run.py"]
GUIDED = ["tests/test_oracle_guided.py"]

MUTATIONS = [
    ("select_bit_off_by_one", "if (seen == q) return i;", "if (seen == q) return (i + 1) % L;",
     PLAIN),
    ("modified_weight_sign", "? -c * A : -p->s * (double)kb;", "? c * A : -p->s * (double)kb;",
     PLAIN),
    ("integral_drops_r",
     "        A = fma((double)r, w, A);\n        tau = tau + w;\n        /* uniform choice",
     "        A = A + w;\n        tau = tau + w;\n        /* uniform choice", PLAIN),
    ("modified_rate_drops_es",
     "double R = (p->mode == ORC_MODIFIED) ? es * (double)r : (double)r;",
     "double R = (p->mode == ORC_MODIFIED) ? (double)r : (double)r;", PLAIN),
    ("selection_comparison", "at_or_below = (Ck[mid] - (double)j) <= d;",
     "at_or_below = (Ck[mid] - (double)j) < d - 1e-3;", PLAIN),
    ("psi_drops_mean", "return lmax + log(T / (double)Nc);", "return lmax + log(T);", PLAIN),
    ("init_comparison", "< (uint64_t)(p->N - taken)", "<= (uint64_t)(p->N - taken)", PLAIN),
    ("khat_drops_L", "res->k_hat = ksum / ((double)Nc * (double)L * t_obs);",
     "res->k_hat = ksum / ((double)Nc * t_obs);", PLAIN),
    ("philox_constant", "(uint64_t)0xD2511F53u * (uint64_t)c0",
     "(uint64_t)0xCD9E8D57u * (uint64_t)c0", PLAIN),
    ("weights_drop_shift", "acc += exp(ell[i] - lmax);", "acc += exp(ell[i]);", PLAIN),
    ("interval_end_test",
     "        if (tau + w >= dt) {\n            A = fma((double)r, dt - tau, A);\n            break;",
     "        if (tau >= dt) {\n            A = fma((double)r, dt - tau, A);\n            break;",
     PLAIN),
    ("hop_partner_index",
     "        n[(bond + 1) % L] = t;\n        ++kb;\n        r = escape_count(n, L);\n    }",
     "        n[(bond + L - 1) % L] = t;\n        ++kb;\n        r = escape_count(n, L);\n    }",
     PLAIN),
    ("guided_weight_sign", "*ell_out = -G - (A - (es * 0x1p-16) * AS);",
     "*ell_out = +G - (A - (es * 0x1p-16) * AS);", GUIDED),
    ("guided_rate_scale", "*ell_out = -G - (A - (es * 0x1p-16) * AS);",
     "*ell_out = -G - (A - es * AS);", GUIDED),
    ("guided_always_accept",
     "if (mulhi64(word_of(y[0], y[1]), (uint64_t)egmax) < (uint64_t)e) break;",
     "if (1) break;", GUIDED),
    ("guided_drops_jump_term", "G += log((double)e * 0x1p-16);", "G += 0.0;", GUIDED),
]


def _run_pins(tmp_path, source, files):
    src = tmp_path / "oracle.c"
    lib = tmp_path / "liboracle_copy.so"
    src.write_text(source)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-shared", "-fPIC",
                           str(src), "-o", str(lib), "-lm"])
    env = dict(os.environ, PD_ORACLE_LIB=str(lib))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           "-m", "not gpu"] + files, cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=900)


def test_unmodified_copy_passes(tmp_path):
    r = _run_pins(tmp_path, open(ORACLE_C).read(), PLAIN + GUIDED)
    assert r.returncode == 0, r.stdout[-3000:]


@pytest.mark.parametrize("name,orig,mutated,files", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, orig, mutated, files):
    source = open(ORACLE_C).read()
    assert source.count(orig) == 1, name   # the mistake goes where it is meant to
    r = _run_pins(tmp_path, source.replace(orig, mutated), files)
    # 1: a test failed (not a crash, a collection error or an interruption)
    assert r.returncode == 1, (name, r.stdout[-3000:])
