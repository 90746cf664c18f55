"""End-to-end learned closure on a small ensemble: batched LB-IMB drag data,
MLP training on the GPU, held-out evaluation against the resolved drag with
resolved drag as fallback outside the training envelope."""
import numpy as np
import pytest

from paper_1011_2613_amd import binding, ensemble as E

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def run(boxes, steps):
    b = binding.Batch(boxes, samples=4)
    steady, stop = E.run_to_steady(b, boxes, check_every=250, max_steps=steps, tol=1e-4)
    U = b.mean_velocity()
    X, y, box_of, st = E.drag_dataset(boxes, b, steady, U)
    return X[st], y[st], steady


def test_closure_pipeline_small():
    kw = dict(edges=(32, 48), r_range=(4.0, 6.0), re_range=(0.1, 10.0))
    train = E.sample_boxes(40, 11, **kw)
    test = E.sample_boxes(10, 9011, **kw)
    Xtr, ytr, st = run(train, 3000)
    Xte, yte, st2 = run(test, 3000)
    say("train samples %d (steady boxes %d/%d), test samples %d" % (len(ytr), st.sum(), len(st), len(yte)))
    assert len(ytr) > 100 and len(yte) > 10
    assert np.all(ytr > 0)
    mlp, norm, losses = E.train_closure(Xtr, ytr, epochs=150, batch=512, lr=3e-3, log=say)
    assert losses[-1] < 0.5 * losses[0]
    res = E.evaluate(mlp, norm, Xte, yte)
    const = float(np.mean(np.abs(np.exp(np.mean(np.log(ytr))) - yte) / yte))
    say("held-out:", res, "constant-predictor error %.3f" % const)
    assert res["mlp_rel_err_mean_all_rows"] < const
    # 450 training particles: a gain over the Wen-Yu-type correlation and a
    # stated bound (the recorded 40-ensemble run is checked by
    # test_closure_record.py)
    assert res["mlp_rel_err_mean_all_rows"] < 0.8 * res["wen_yu_rel_err_mean"]
    assert res["mlp_rel_err_mean_all_rows"] < 0.35
