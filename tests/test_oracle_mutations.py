"""Planted mistakes.  Each case compiles a copy of oracle/oracle.c with one
plausible mistake (a dropped term or factor, a wrong sign, index, constant or
comparison) and runs the oracle's pins against that copy in a fresh process
(PD_ORACLE_LIB names the copy); some pin must fail.  The control case compiles
the unmodified source the same way and must pass, so a failure is the
mistake's.  The reference Adam step of the guide (oracle/guide_net.py) gets
the same treatment in-process: each altered copy of the module must fail one
of its pins.  The tracked sources are never modified.

One plausible mistake is not here because no pin can see it: drawing the
uniform variate in [0, 1) instead of (0, 1] changes one value in 2^53."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
PLAIN = ["tests/test_oracle_dynamics.py", "tests/test_oracle_selection.py",
         "tests/test_oracle_run.py"]
GUIDED = ["tests/test_oracle_guided.py"]
ESTIMATORS = ["tests/test_oracle_run.py", "tests/test_oracle_estimators.py"]

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
     "if (mulhi64((uint64_t)pr, (uint64_t)egmax) >= (uint64_t)e) continue;",
     "if (0) continue;", GUIDED),
    ("guided_proposal_rate_drops_bound", "const double unit = es * ((double)egmax * 0x1p-16);",
     "const double unit = es;", GUIDED),
    ("guided_drops_jump_term", "G += log((double)e * 0x1p-16);", "G += 0.0;", GUIDED),
    ("psi_burn_counts_burn_in_interval", "if (beta > p->burn_in) psi_burn_sum += lm;",
     "if (beta >= p->burn_in) psi_burn_sum += lm;", ESTIMATORS),
    ("k_burn_counts_burn_in_interval",
     "if (beta > p->burn_in)\n            for (int64_t j = 0; j < Nc; ++j) Kp[j] += Kb[j];",
     "if (beta >= p->burn_in)\n            for (int64_t j = 0; j < Nc; ++j) Kp[j] += Kb[j];",
     ESTIMATORS),
    ("k_burn_not_inherited", "Kp2[j] = Kp[anc[j]];", "Kp2[j] = Kp[j];", ESTIMATORS),
    ("log_keeps_running_sum", "if (lbeta) lbeta[beta - 1] = lm;",
     "if (lbeta) lbeta[beta - 1] = psi_sum;", ESTIMATORS),
    ("log_mean_hops_cumulative", "mean_kb[beta - 1] = (double)hb / (double)Nc;",
     "mean_kb[beta - 1] = (double)hops / (double)Nc;", ESTIMATORS),
    ("lineage_origin_not_inherited", "org2[j] = origin[anc[j]];", "org2[j] = origin[j];",
     ["tests/test_oracle_estimators.py"]),
]

ADAM_MUTATIONS = [
    ("adam_no_first_bias_correction", "mh = m / (1 - b1 ** step)", "mh = m"),
    ("adam_no_second_bias_correction", "vh = v / (1 - b2 ** step)", "vh = v"),
    ("adam_eps_inside_root", "np.sqrt(vh) + eps", "np.sqrt(vh + eps)"),
    ("adam_second_moment_of_abs", "(1 - b2) * g * g", "(1 - b2) * np.abs(g)"),
    ("adam_first_moment_decay", "m = b1 * m + (1 - b1) * g", "m = b2 * m + (1 - b2) * g"),
    ("adam_ascends", "return theta - lr * mh", "return theta + lr * mh"),
]


def _run_pins(tmp_path, source, files):
    src = tmp_path / "oracle.c"
    lib = tmp_path / "liboracle_copy.so"
    src.write_text(source)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-shared", "-fPIC",
                           str(src), "-o", str(lib), "-lm"])
    # one thread per run: the runs go side by side
    env = dict(os.environ, PD_ORACLE_LIB=str(lib), OMP_NUM_THREADS="1",
               OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           "-m", "not gpu"] + files, cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=900)


@pytest.fixture(scope="module")
def pin_runs(tmp_path_factory):
    """The pins run against every copy (the control and each planted mistake),
    in separate processes side by side."""
    source = open(ORACLE_C).read()
    jobs = {"control": (source, PLAIN + GUIDED + ESTIMATORS[1:])}
    for name, orig, mutated, files in MUTATIONS:
        if source.count(orig) == 1:
            jobs[name] = (source.replace(orig, mutated), files)
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {k: ex.submit(_run_pins, tmp_path_factory.mktemp(k), src, files)
                for k, (src, files) in jobs.items()}
        return {k: f.result() for k, f in futs.items()}


def test_unmodified_copy_passes(pin_runs):
    r = pin_runs["control"]
    assert r.returncode == 0, r.stdout[-3000:]


@pytest.mark.parametrize("name,orig,mutated,files", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(pin_runs, name, orig, mutated, files):
    assert open(ORACLE_C).read().count(orig) == 1, name   # the mistake goes where it is meant to
    r = pin_runs[name]
    # 1: a test failed (not a crash, a collection error or an interruption)
    assert r.returncode == 1, (name, r.stdout[-3000:])


@pytest.mark.parametrize("name,orig,mutated", ADAM_MUTATIONS, ids=[m[0] for m in ADAM_MUTATIONS])
def test_planted_adam_mistake_fails_a_pin(name, orig, mutated):
    import importlib.util
    import test_guide_net_adam as pins
    path = os.path.join(ROOT, "oracle", "guide_net.py")
    source = open(path).read()
    assert source.count(orig) == 1, name
    spec = importlib.util.spec_from_loader("guide_net_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(source.replace(orig, mutated), path, "exec"), mod.__dict__)
    failed = []
    for pin in pins.PINS:
        try:
            pin(mod.adam)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, name
