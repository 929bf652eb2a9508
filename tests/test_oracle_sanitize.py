"""The oracle under the address and undefined-behaviour sanitizers (host
code only, g++): a driver (oracle/orc_sanitize_main.cpp) runs every entry
point of the oracle's C API that the tests use on a small two-temperature
case and must finish cleanly."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import orc
from paper_2403_03440_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def _write_case(path, m, ni, nj, fs, q, x, y):
    def row(a):
        return " ".join(repr(float(v)) if isinstance(v, (float, np.floating)) else str(int(v))
                        for v in np.asarray(a).ravel())
    nr = m.nr
    lines = [f"{m.ns} {nr} {int(m.two_temp)}", row(m.M), row(m.kind), row(m.theta_v), row(m.theta_r), row(m.sigma),
             row(m.g_el), row(m.h_form), row(m.sc), row(m.lt_a), row(m.lt_b),
             row(np.asarray(m.A, float)), row(np.asarray(m.b, float)), row(np.asarray(m.theta, float)),
             row(m.tctl), row(m.third), row(m.nu_f), row(m.nu_b), row(np.asarray(m.eff, float)),
             f"{m.mu_ref!r} {m.T_ref!r} {m.mu_exp!r}", f"{ni} {nj}", row(x), row(y), row(fs[0]),
             f"{fs[1]!r} {fs[2]!r} {fs[3]!r} {fs[4]!r}", row(q)]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    m = I.air5(1)
    ni, nj = 6, 4
    x, y = I.polar_grid(ni, nj)
    Y = np.zeros(m.ns)
    Y[m.ns - 1], Y[m.names.index("O2")] = 0.767, 0.233
    fs = (1e-3 * Y, 5000.0, 0.0, 250.0, 250.0)
    o = orc.setup((x, y), m, fs)
    q = o.prim_to_cons(*I.random_prims(m, ni * nj, 3, T_range=(1500.0, 6000.0), speed=2000.0, y_floor=0.02))
    case = tmp_path / "case.txt"
    _write_case(case, m, ni, nj, fs, q, x, y)
    exe = tmp_path / "orc_san"
    flags = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
    subprocess.run(["g++", "-std=c++17", "-fopenmp", *flags, "-o", str(exe), os.path.join(ORACLE, "orc.cpp"),
                    os.path.join(ORACLE, "orc_sanitize_main.cpp")], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe), str(case)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.startswith("r_rho ")
