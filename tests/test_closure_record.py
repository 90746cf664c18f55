"""The recorded end-to-end closure run (profiles/closure_pipeline_heldout.json,
written by paper_1011_2613_amd.closure_pipeline on one MI355X): every one of
the 64 held-out boxes is accounted for (steady boxes scored against their
steady drag, the rest reported against their drag at the step cap), the
closure beats the Wen-Yu-type correlation by a wide margin, and the held-out
figures are the ones stated for this run."""
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load():
    with open(os.path.join(ROOT, "profiles", "closure_pipeline_heldout.json")) as f:
        return json.load(f)


def test_every_heldout_box_is_reported():
    d = load()
    run = d["heldout_run"]
    assert run["boxes"] == 64
    steady, unsteady = d["heldout"], d["heldout_unsteady_boxes"]
    assert steady["boxes"] == run["steady_boxes"]
    assert steady["boxes"] + (unsteady["boxes"] if unsteady else 0) == run["boxes"]
    assert steady["n"] == run["samples"] and (unsteady["n"] if unsteady else 0) == run["unsteady_samples"]
    assert steady["fallback_fraction"] == 0.0  # no held-out particle outside the training envelope


def test_recorded_heldout_figures():
    d = load()
    h = d["heldout"]
    assert d["train_samples"] >= 490000
    # per particle and per box (mean of the box-mean drag errors), as stated
    assert h["mlp_rel_err_mean"] < 0.056
    assert h["mlp_box_mean_rel_err"] < 0.051
    # the learned closure against the correlation without learning
    assert h["mlp_rel_err_mean"] < 0.25 * h["wen_yu_rel_err_mean"]
    assert h["mlp_box_mean_rel_err"] < 0.25 * h["wen_yu_box_mean_rel_err"]
    # boxes not steady at the step cap: still well below the correlation
    u = d["heldout_unsteady_boxes"]
    assert u["mlp_rel_err_mean"] < 0.5 * u["wen_yu_rel_err_mean"]
