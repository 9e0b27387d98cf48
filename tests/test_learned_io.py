"""Model files of the learned preconditioner: FP32 blob + JSON metadata round trip, and
rejection of blobs that do not match their metadata (host only)."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2508_17522_amd import _capi as C  # noqa: E402
from paper_2508_17522_amd.learned import NPARAM, LearnedModel  # noqa: E402


def test_parameter_count_matches_layout():
    F, H = C.QCPD_NFEAT, C.QCPD_MLP_HIDDEN
    assert NPARAM == 2 * F + (F * H + H) + (H * H + H) + (2 * H + 2)


def test_round_trip(tmp_path):
    w = torch.tensor(np.random.default_rng(0).standard_normal(NPARAM), dtype=torch.float32)
    m = LearnedModel(w, dict(steps=3, note="x"))
    p = str(tmp_path / "model")
    m.save(p)
    raw = open(p + ".bin", "rb").read()
    assert len(raw) == 4 * NPARAM
    assert np.array_equal(np.frombuffer(raw, dtype="<f4"), w.numpy())
    m2 = LearnedModel.load(p, device="cpu")
    assert torch.equal(m2.weights, w)
    assert m2.meta["steps"] == 3 and m2.meta["params"] == NPARAM
    assert len(m2.meta["feature_schema"]) == C.QCPD_NFEAT


def test_rejects_corrupt_or_foreign_files(tmp_path):
    w = torch.zeros(NPARAM, dtype=torch.float32)
    p = str(tmp_path / "model")
    LearnedModel(w).save(p)
    with open(p + ".bin", "r+b") as f:
        f.write(b"\x01")
    with pytest.raises(ValueError, match="checksum"):
        LearnedModel.load(p, device="cpu")
    LearnedModel(w).save(p)
    meta = json.load(open(p + ".json"))
    meta["params"] = NPARAM + 1
    json.dump(meta, open(p + ".json", "w"))
    with pytest.raises(ValueError, match="parameters"):
        LearnedModel.load(p, device="cpu")
