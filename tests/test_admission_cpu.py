"""The serving loop's admission logic (first-fit HBM arena, FIFO prefix rule),
compiled on its own with g++ and checked against a plain Python model on
random operation sequences.  No GPU."""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_01579_amd", "csrc")
ALIGN = 256


def rnd(v):
    v = max(v, 1)
    return (v + ALIGN - 1) // ALIGN * ALIGN


class Model:
    """First fit over sorted free ranges, coalescing on release."""

    def __init__(self, cap):
        self.cap = cap // ALIGN * ALIGN
        self.free = [[0, self.cap]] if self.cap else []

    def alloc(self, b):
        need = rnd(b)
        for r in self.free:
            if r[1] >= need:
                off = r[0]
                r[0] += need
                r[1] -= need
                self.free = [x for x in self.free if x[1] > 0]
                return off
        return None

    def release(self, off, b):
        self.free.append([off, rnd(b)])
        self.free.sort()
        merged = []
        for r in self.free:
            if merged and merged[-1][0] + merged[-1][1] == r[0]:
                merged[-1][1] += r[1]
            else:
                merged.append(list(r))
        self.free = merged

    def stat(self):
        return (sum(r[1] for r in self.free), max([r[1] for r in self.free] or [0]),
                len(self.free))


def prefix_model(fps, room, mx):
    used = k = 0
    while k < len(fps) and k < mx:
        f = rnd(fps[k]) if fps[k] else ALIGN
        if used + f > room:
            break
        used += f
        k += 1
    return k


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("adm") / "admission_harness")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-o", exe,
                    os.path.join(ROOT, "tests", "admission_harness.cpp")], check=True)
    return exe


def run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    return out[:len(lines)]


@pytest.mark.parametrize("seed", range(6))
def test_arena_matches_first_fit_model(harness, seed):
    rng = random.Random(seed)
    cap = rng.choice([1 << 16, 1 << 20, 3 * 4096 + 100])
    model = Model(cap)
    ops, expect, live = ["reset %d" % cap], ["ok"], []
    for _ in range(400):
        if live and rng.random() < 0.45:
            off, b = live.pop(rng.randrange(len(live)))
            model.release(off, b)
            ops.append("release %d %d" % (off, b))
            expect.append("ok")
        else:
            b = rng.choice([0, 1, 255, 256, 257, 1000, 4096, 9000, rng.randrange(1, cap // 3 + 2)])
            off = model.alloc(b)
            ops.append("alloc %d" % b)
            if off is None:
                expect.append("fail")
            else:
                expect.append("ok %d" % off)
                live.append((off, b))
        ops.append("stat")
        expect.append("%d %d %d" % model.stat())
    got = run(harness, ops)
    for i, (g, e) in enumerate(zip(got, expect)):
        assert g == e, f"op {i} ({ops[i]}): got {g!r}, model {e!r}"


def test_arena_returns_to_one_range(harness):
    """Releasing everything, in any order, coalesces back to the whole arena."""
    rng = random.Random(7)
    cap = 1 << 20
    ops = ["reset %d" % cap] + ["alloc %d" % rng.randrange(1, 20000) for _ in range(40)]
    got = run(harness, ops)
    live = [(int(g.split()[1]), int(o.split()[1])) for o, g in zip(ops[1:], got[1:])
            if g.startswith("ok ")]
    assert live
    offs = sorted(o for o, _ in live)
    assert len(set(offs)) == len(offs)
    spans = sorted((o, rnd(b)) for o, b in live)
    for (o1, b1), (o2, _) in zip(spans, spans[1:]):
        assert o1 + b1 <= o2                       # no two ranges overlap
    rng.shuffle(live)
    ops2 = ops + ["release %d %d" % (o, b) for o, b in live] + ["stat"]
    assert run(harness, ops2)[-1] == "%d %d 1" % (cap, cap)


@pytest.mark.parametrize("seed", range(4))
def test_admit_prefix_is_the_fifo_rule(harness, seed):
    rng = random.Random(100 + seed)
    ops, expect = [], []
    for _ in range(200):
        n = rng.randrange(0, 12)
        fps = [rng.choice([0, 100, 256, 5000, rng.randrange(1, 1 << 20)]) for _ in range(n)]
        room = rng.randrange(0, 1 << 21)
        mx = rng.randrange(1, 16)
        ops.append("prefix %d %d %d %s" % (room, mx, n, " ".join(map(str, fps))))
        expect.append(str(prefix_model(fps, room, mx)))
    assert run(harness, ops) == expect
    # a head that does not fit blocks the jobs behind it, however small
    assert run(harness, ["prefix 1000 8 3 5000 10 10"]) == ["0"]
