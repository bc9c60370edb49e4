"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only).  A child Python process preloads the ASan runtime, loads a
sanitized build of the oracle (``oracle.build.build_sanitized``) and runs
every entry point on small inputs, up to pattern size 9; a memory or
undefined-behaviour error aborts the child.  Its results must equal those of
the normal build, run the same way."""
import json
import os
import shutil
import subprocess
import sys

import pytest

import oracle.build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, ROOT_DIR)
import numpy as np
import oracle, synth
out = {}
for seed in range(6):
    s, t, lab = synth.tiny_graph(5000 + seed, 9, 12, 1 + seed % 3)
    n = len(lab)
    out["mine" + str(seed)] = oracle.mine(n, s, t, lab, 1 + seed % 2, 6)
    out["induced" + str(seed)] = oracle.mine(n, s, t, lab, 1, 5, induced=True)
    out["count" + str(seed)] = [oracle.count_connected(n, s, t, k) for k in range(1, 6)]
    res = out["mine" + str(seed)]
    g = oracle.Graph(n, s, t, lab)
    out["support" + str(seed)] = [g.support(list(l), a) for _, l, a, _ in res[:20]]
    out["bounded" + str(seed)] = [g.support(list(l), a, t=3) for _, l, a, _ in res[:20]]
    g.close()
    out["single" + str(seed)] = [oracle.pattern_support(n, s, t, lab, list(l), a)
                              for _, l, a, _ in res[:5]]
m = 10
s = np.arange(m - 1, dtype=np.int32)
t = np.arange(1, m, dtype=np.int32)
out["path9"] = oracle.mine(m, s, t, np.zeros(m, np.int32), 1, 9)
out["canon"] = [oracle.canonical([k % 3 for k in range(n)], (1 << (n * (n - 1) // 2)) - 1 - n)
                for n in range(2, 10)]
print(json.dumps(out))
""".replace("ROOT_DIR", repr(ROOT))


def run_child(env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True,
                       text=True, timeout=900)
    return r


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime for gcc")
    lib = oracle.build.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    sanitized = run_child({"FSM_ORACLE_LIB": lib, "LD_PRELOAD": asan,
                           "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert sanitized.returncode == 0, sanitized.stderr[-4000:]
    plain = run_child({})
    assert plain.returncode == 0, plain.stderr[-4000:]
    assert json.loads(sanitized.stdout) == json.loads(plain.stdout)
