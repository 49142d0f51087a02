"""Host code under the address and undefined-behaviour sanitizers (no GPU):
the CPU oracle's every entry point and the serving loop's arena allocator and
admission rule, each built with gcc/g++ -fsanitize=address,undefined and run
on small inputs; any sanitizer report fails the test."""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_01579_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(exe, stdin=None):
    r = subprocess.run([exe], input=stdin, capture_output=True, text=True, env=ENV, timeout=120)
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    subprocess.run([gcc, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", *SAN,
                    "-o", exe, os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-lm"],
                   check=True)
    out = _run(exe)
    assert out.startswith("checksum ")


def test_admission_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "admission_san")
    subprocess.run([gxx, "-std=c++17", *SAN, "-I", CSRC, "-o", exe,
                    os.path.join(ROOT, "tests", "admission_harness.cpp")], check=True)
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "adm_model", os.path.join(ROOT, "tests", "test_admission_cpu.py"))
    adm = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(adm)
    rng = random.Random(3)
    cap = 1 << 20
    model = adm.Model(cap)
    ops, expect, live = ["reset %d" % cap], ["ok"], []
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off, b = live.pop(rng.randrange(len(live)))
            model.release(off, b)
            ops.append("release %d %d" % (off, b))
            expect.append("ok")
        else:
            b = rng.choice([0, 1, 255, 4096, rng.randrange(1, 1 << 18)])
            off = model.alloc(b)
            ops.append("alloc %d" % b)
            expect.append("fail" if off is None else "ok %d" % off)
            if off is not None:
                live.append((off, b))
        ops.append("stat")
        expect.append("%d %d %d" % model.stat())
        n = rng.randrange(0, 8)
        fps = [rng.randrange(0, 1 << 19) for _ in range(n)]
        room, mx = rng.randrange(0, 1 << 21), rng.randrange(1, 9)
        ops.append("prefix %d %d %d %s" % (room, mx, n, " ".join(map(str, fps))))
        expect.append(str(adm.prefix_model(fps, room, mx)))
    got = _run(exe, "\n".join(ops) + "\n").split("\n")[:len(ops)]
    assert got == expect


def test_serve_sim_under_sanitizers(tmp_path):
    """The scheduler's admission round and latency accounting on a simulated
    device, built with the sanitizers, on a random mix (checked against the
    Python model as in tests/test_serve_sim_cpu.py)."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "serve_sim_san")
    subprocess.run([gxx, "-std=c++17", *SAN, "-I", CSRC, "-o", exe,
                    os.path.join(ROOT, "tests", "serve_sim_harness.cpp")], check=True)
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "sim_model", os.path.join(ROOT, "tests", "test_serve_sim_cpu.py"))
    sim = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(sim)
    rng = random.Random(11)
    t, jobs = 0, []
    for _ in range(300):
        t += rng.choice([0, 1, 7, rng.randrange(0, 200)])
        jobs.append((t, rng.choice([1, 256, 5000, rng.randrange(1, 40000)]), rng.randrange(1, 500)))
    text = "slots 3 cap 65536 maxjobs 4 deadline 400\n"
    text += "".join("job %d %d %d\n" % j for j in jobs) + "end\n"
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.strip().split("\n")
    per = [None if l == "refused" else tuple(int(v) for v in l.split()) for l in lines[:-1]]
    want_per, want_stats = sim.model(3, 65536, 4, 400, jobs)
    assert per == want_per
    assert tuple(int(v) for v in lines[-1].split()[1:]) == want_stats
