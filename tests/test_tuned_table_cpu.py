"""The committed tuner table and the runtime bucket choice (no GPU)."""
import json
import math

import numpy as np
import pytest

import paper_2510_01579_amd as M
from paper_2510_01579_amd import tune as T
from workload import synth as W


@pytest.fixture(scope="module")
def table():
    with open(M.TUNED_TABLE) as fh:
        return json.load(fh)


def test_table_covers_every_class_with_sorted_buckets(table):
    assert set(table["classes"]) == set(T.CLASSES)
    for name, rec in table["classes"].items():
        snrs = [b["snr_db"] for b in rec["buckets"]]
        if name.startswith("vpp"):
            assert snrs == [None]
        else:
            assert snrs == sorted(snrs) == T.CLASSES[name]["snr"]


def test_every_choice_meets_the_selection_margin_and_is_not_dearer(table):
    for name, rec in table["classes"].items():
        ref = rec["reference"]
        for b, meas in zip(rec["buckets"], rec["per_snr"]):
            cand = T.parse_key_of(b["tuned"])
            cand_any = T.parse_key_of(b.get("tuned_any", b["tuned"]))
            for c0 in (cand, cand_any):
                q = meas["cands"][T.schedule_key(c0)]
                assert q <= (1 + table["select_tolerance"]) * meas["ref"] + 2e-5, (name, b)
                assert T.cand_cost(name, c0) <= T.cost(name, ref["chains"], ref["sweeps"])
            timed = meas.get("ms", {})
            val = meas.get("val")
            if val:     # a validation slot: the choices meet the margin there too
                assert T.passes_val(meas, cand) and T.passes_val(meas, cand_any), (name, b)
            if T.schedule_key(cand_any) not in timed:
                assert T.cand_cost(name, cand_any) <= T.cand_cost(name, cand)
            # no measured candidate within the margin (and validated, where a
            # validation slot was measured) is cheaper (by the cost model among
            # the plan formulations; by measured time, where timed, among all)
            for key, v in meas["cands"].items():
                c = T.parse_key(key)
                if v <= (1 + table["select_tolerance"]) * meas["ref"] + 2e-5 and \
                        (not val or T.passes_val(meas, c)):
                    assert T.cand_cost(name, c) >= T.cand_cost(name, cand), (name, key)
                    if T.schedule_key(cand_any) in timed:
                        if key in timed:
                            assert timed[key] >= timed[T.schedule_key(cand_any)], (name, key)
                    else:
                        assert T.cand_cost(name, c) >= T.cand_cost(name, cand_any), (name, key)


def test_reselect_reproduces_the_table(table, tmp_path):
    src = tmp_path / "t.json"
    out = tmp_path / "o.json"
    src.write_text(json.dumps(table))
    T.main(["--reselect", str(src), "--out", str(out)])
    again = json.loads(out.read_text())
    for name in table["classes"]:
        assert again["classes"][name]["buckets"] == table["classes"][name]["buckets"]


@pytest.mark.parametrize("snr,bucket", [(0.0, 5.0), (5.0, 5.0), (7.5, 10.0), (15.0, 15.0),
                                        (15.2, 20.0), (25.0, 25.0), (40.0, 25.0)])
def test_bucket_is_the_smallest_tuned_snr_at_or_above(snr, bucket):
    t = M.tuned_schedule(M.KIND_DET, 8, 8, 16, W.noise_var(snr, 8))
    assert t["tuned"] and t["snr_bucket"] == bucket


def test_schedule_table_matches_generator_ranges(table):
    """The beta table of a tuned schedule is the linear schedule between the
    shaped ends of the default range."""
    nv = W.noise_var(15.0, 8)
    t = M.tuned_schedule(M.KIND_DET, 8, 8, 16, nv)
    rec = [b for b in table["classes"]["det-8x8-16"]["buckets"] if b["snr_db"] == 15.0][0]
    lo, hi = T.shaped_range(*W.det_beta_range(16, 8, nv), tuple(rec["tuned"]["shape"]))
    assert np.array_equal(t["beta2"], W.linear_beta2(t["sweeps"], lo, hi))
    assert t["beta2"].dtype == np.float32 and np.all(np.isfinite(t["beta2"]))


def test_unknown_class_gets_the_reference_schedule():
    t = M.tuned_schedule(M.KIND_DET, 6, 6, 16, 0.1)
    assert not t["tuned"] and (t["chains"], t["sweeps"]) == (64, 200)
    t = M.tuned_schedule(M.KIND_DET, 12, 12, 64, 0.1)
    assert not t["tuned"] and (t["chains"], t["sweeps"], t["init"]) == (128, 400, 1)


def test_schedule_keys_round_trip():
    for c in [(64, 50, 1, (0.0, 1.0), 0), (16, 12, 0, (0.0, 1.0), 2),
              (8, 4, 0, (0.0625, 4.0), 0), (16, 4, 0, (0.25, 1.0), 1, 3),
              (4, 2, 0, (0.0, 1.0), 2, 2), (16, 8, 0, (0.25, 1.0), 3)]:
        assert T.parse_key(T.schedule_key(c)) == c
    for c in T.delta_candidates() + T.e_candidates():
        assert T.parse_key(T.schedule_key(c)) == c


def test_any_formulation_returns_the_guess_set(table):
    """tuned_schedule hands the guess set (MMGaP-E, the MMSE-SIC guess) of the
    bucket's choice to plans and detect_e."""
    for name, rec in table["classes"].items():
        kind, rows, cols, qam = T.parse_class(name)
        if kind != "det":
            continue
        for b in rec["buckets"]:
            nv = W.noise_var(b["snr_db"], cols)
            t = M.tuned_schedule(M.KIND_DET, rows, cols, qam, nv)
            ta = M.tuned_schedule(M.KIND_DET, rows, cols, qam, nv, any_formulation=True)
            assert t["guesses"] == b["tuned"].get("guesses", M.GUESS_MMSE if t["stages"] else 0)
            want = b.get("tuned_any", b["tuned"])
            assert ta["guesses"] == want.get("guesses", M.GUESS_MMSE if want["stages"] else 0)
            assert (ta["chains"], ta["sweeps"], ta["stages"]) == \
                (want["chains"], want["sweeps"], want["stages"])


def test_tuned_schedule_returns_the_stage_count(table):
    """A bucket that chose moves around the MMSE guess hands its stage count to
    plans and the server (0 for the binary encoding)."""
    for name, rec in table["classes"].items():
        kind, rows, cols, qam = T.parse_class(name)
        for b in rec["buckets"]:
            snr = b["snr_db"] if b["snr_db"] is not None else 0.0
            nv = W.noise_var(snr, cols) if kind == "det" else 0.0
            t = M.tuned_schedule(M.KIND_DET if kind == "det" else M.KIND_VPP, rows, cols, qam,
                                 nv)
            assert t["stages"] == b["tuned"].get("stages", 0), (name, b["snr_db"])
            if t["stages"]:
                assert kind == "det"
