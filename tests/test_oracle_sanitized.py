"""The CPU oracles under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize_driver.c is compiled with oracle/frnn_oracle.c and
oracle/components_oracle.c, with both sanitizers and no recovery, and run on the
tiny event, every stress input, a dyadic event and crowded cells.  Every run must
end cleanly (any sanitizer report aborts it) and give exactly what the ordinary
oracle libraries give: grid and O(n^2) edges, degrees, distances and labels.
"""

import os
import subprocess

import numpy as np
import pytest

from oracle import components, oracle
from paper_2202_06929_amd import events

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "sanitized_oracle")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "frnn_oracle.c"),
           os.path.join(ROOT, "oracle", "components_oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def cases():
    X, _ = events.generate(events.TINY)
    out = [("tiny", X, events.TINY.r, events.TINY.K)]
    out += [(c.name, c.points, c.r, c.K) for c in events.stress_cases() if c.points.shape[0] > 0]
    out.append(("dyadic", events.dyadic_event(3000, 8, 9)[0], 0.2, 64))
    out.append(("dense_cells_k4", events.dense_cells(8), 0.1, 4))
    return out


@pytest.mark.parametrize("name,X,r,K", cases(), ids=[c[0] for c in cases()])
def test_sanitized_oracle_matches_and_runs_clean(driver, tmp_path, name, X, r, K):
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.int64(n).tobytes() + np.int32(d).tobytes() + np.float32(r).tobytes() + np.int32(K).tobytes())
        f.write(X.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")
    res = subprocess.run([driver, str(inp), str(outp)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, f"{name}: exit {res.returncode}\n{res.stderr[-3000:]}"
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr[-3000:]
    buf = open(outp, "rb").read()
    at = 0

    def take(dtype, count):
        nonlocal at
        a = np.frombuffer(buf, dtype=dtype, count=count, offset=at)
        at += a.nbytes
        return a

    Eg = int(take(np.int64, 1)[0])
    grid = np.stack([take(np.int64, Eg), take(np.int64, Eg)])
    want = oracle.frnn_grid(X, r, K)
    assert np.array_equal(grid, want)
    Eb = int(take(np.int64, 1)[0])
    if n <= 4000:
        brute = np.stack([take(np.int64, Eb), take(np.int64, Eb)])
        assert np.array_equal(brute, oracle.frnn_brute(X, r, K))
        assert np.array_equal(take(np.int64, n), oracle.degrees(X, r))
    else:
        assert Eb == -1
    dist = take(np.float32, Eg)
    assert np.array_equal(dist.view(np.uint32), oracle.pair_dist(X, want[0], want[1]).view(np.uint32))
    assert np.array_equal(take(np.int64, n), components.labels(want[0], want[1], n))
    assert at == len(buf)
