"""Host sanitizer run of the CPU oracle: its source compiled with
AddressSanitizer and UndefinedBehaviorSanitizer into tests/ref/oracle_sanitize.cpp,
which calls every entry point (error paths included) on a small power-law
graph.  The run must end cleanly with no sanitizer report, and each call's
output sum must equal what the oracle library, built without sanitizers,
gives for the same call."""

import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not installed")
    exe = str(tmp_path_factory.mktemp("osan") / "oracle_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", os.path.join(HERE, "ref", "oracle_sanitize.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_oracle_under_address_and_undefined_behaviour_sanitizers(orc, sanitized):
    from synth.graphs import chung_lu

    n = 300
    s, d = chung_lu(n, 2400, 2.1, seed=4)
    s = np.asarray(s, np.int32)
    d = np.asarray(d, np.int32)
    blob = np.int32(n).tobytes() + np.int64(s.size).tobytes() + s.tobytes() + d.tobytes()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sanitized], input=blob, capture_output=True, env=env, timeout=600)
    err = r.stderr.decode(errors="replace")
    assert r.returncode == 0, err[-4000:]
    assert "Sanitizer" not in err and "runtime error" not in err, err[-4000:]
    got = {}
    for line in r.stdout.decode().splitlines():
        name, *vals = line.split()
        got[name] = vals

    G = orc.Graph(n, s, d)
    p = orc.params(n, 0.6, 0.2, 0.01)
    p0 = orc.params(n, 0.6, 0.2, 0.01, eps_p=0.0)
    u = 0

    def same(name, value):
        assert int(got[name][0]) == orc.ORC_OK, name
        assert float(got[name][1]) == pytest.approx(value, rel=1e-12, abs=1e-15), name

    assert int(got["walks"][0]) == sum(len(orc.walk(G, u, k, 3, p)) for k in range(200))
    same("single_source_0", orc.single_source(G, u, p, 5)[0].sum())
    same("single_source_1", orc.single_source(G, u, p, 5, precision="f32")[0].sum())
    same("single_source_2", orc.single_source(G, u, p, 5, probe="randomized")[0].sum())
    for f32, prec in ((0, "f64"), (1, "f32")):
        same(f"batch_{f32}", orc.batch(G, u, p, 7, bias_shift=True, precision=prec)[0].sum())
        same(f"hybrid_{f32}", orc.batch(G, u, p, 7, precision=prec, probe="hybrid", c0=0.01)[0].sum())
    same("merged", orc.merged(G, u, p0, 9)[0].sum())
    path = orc.walk(G, u, 1, 11, p)
    if path.size >= 2:
        same("probe", orc.probe(G, path, 0.6, p.eps_p, precision="f32").sum())
        same("rprobe", orc.rprobe(G, path, 0.6, 11, 1).sum())
    assert int(got["pair_mc"][0]) == orc.ORC_OK
    assert int(got["pair_mc"][1]) == round(orc.pair_mc(G, u, [1], 0.6, 20000, 13)[0] * 20000)
    nodes, vals = orc.topk(orc.batch(G, u, p, 7)[0], u, 10)
    assert int(got["topk"][0]) == orc.ORC_OK and int(got["topk"][1]) == nodes[0]
    assert float(got["topk"][2]) == vals[0]
    want_err = {"err_self": orc.ORC_ESELF, "err_dup": orc.ORC_EDUP, "err_range": orc.ORC_ERANGE,
                "err_params": orc.ORC_EINVAL, "err_node": orc.ORC_ERANGE, "err_walks": orc.ORC_EINVAL,
                "err_merged": orc.ORC_EINVAL, "err_topk": orc.ORC_EINVAL, "err_pair": orc.ORC_EINVAL}
    for name, code in want_err.items():
        assert int(got[name][0]) == code, name
