"""Launch-shape tuning: every launch shape gives the same derivative (up to the order of
floating-point sums), and the autotuner's cache round-trips."""
import numpy as np
import pytest

import qcpgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from paper_2508_17522_amd import tune as T  # noqa: E402
from paper_2508_17522_amd.batch import qcpd_batch_get_launch, qcpd_batch_set_launch  # noqa: E402
from qcpgen.torch_io import batch_create_args, batch_to_device, cones_of, to_device  # noqa: E402


def rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make(qcp, **kw):
    t = to_device(qcp)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(qcp), t["x"], t["y"], t["s"],
                      opts=Q.Opts(tol=1e-12, **kw))
    return h, t


@pytest.mark.parametrize("precond", [Q.QCPD_PRECOND_JACOBI, Q.QCPD_PRECOND_EQUIL])
def test_launch_shapes_agree(precond):
    qcp = qcpgen.small_mixed(1, n=301, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                             psd=(4, 7, 12, 9), n_exp=23, A_density=0.04, P_rank=150,
                             nonneg_active=100)
    h, t = make(qcp, precond=precond)
    ref_j = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    ref_v = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
    gF, gT, mF, mT = Q.qcpd_get_launch(h)
    print(f"default launch {gF} {gT} of {mF} {mT}", flush=True)
    for shape in ((1, 1), (3, 7), (mF, mT), (4 * mF, 4 * mT), (0, 0)):
        Q.qcpd_set_launch(h, *shape)
        got = Q.qcpd_get_launch(h)
        assert 1 <= got[0] <= mF and 1 <= got[1] <= mT
        j = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
        v = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
        assert j[4] == Q.QCPD_OK and v[5] == Q.QCPD_OK
        ej = max(rel(a, b) for a, b in zip(j[:3], ref_j[:3]))
        ev = max(rel(a, b) for a, b in zip(v[:4], ref_v[:4]))
        print(f"shape {shape} -> {got[:2]}: iters {j[3].iters}/{v[4].iters} diff {ej:.1e} {ev:.1e}",
              flush=True)
        assert ej <= 1e-9 and ev <= 1e-9
    assert Q.qcpd_get_launch(h)[:2] == (gF, gT)
    with pytest.raises(Q.QCPDError):
        Q.qcpd_set_launch(h, -1, 0)
    h.close()


def test_tune_handle_and_cache(tmp_path):
    qcp = qcpgen.small_mixed(1)
    h, t = make(qcp, precond=Q.QCPD_PRECOND_EQUIL)
    cache = T.TuneCache(str(tmp_path / "tune.json"))
    opts = Q.Opts(tol=1e-12, precond=Q.QCPD_PRECOND_EQUIL)
    r = T.tune_handle(h, opts, iters=60, reps=1, cache=cache,
                      candidates=[(1, 1, 8), (4, 4, 16), (0, 0, 32)])
    print("tuned", r, flush=True)
    assert not r["cached"] and r["tried"] == 3 and r["ms_per_iter"] > 0
    # the handle solves with the chosen shape and the caller's tolerance
    j = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    assert j[4] == Q.QCPD_OK and j[3].rel_residual <= 1e-11
    cache2 = T.TuneCache(str(tmp_path / "tune.json"))
    r2 = T.tune_handle(h, opts, cache=cache2)
    assert r2["cached"] and r2["grid_F"] == r["grid_F"] and r2["graph_chunk"] == r["graph_chunk"]
    h.close()


def small_batch(count=10):
    rng = np.random.default_rng(5)
    out = []
    for i in range(count):
        n = int(rng.integers(15, 70))
        nn = int(rng.integers(n // 4, n // 2))
        soc = tuple(int(k) for k in rng.integers(1, 6, size=int(rng.integers(0, 4))))
        psd = tuple(int(k) for k in rng.integers(1, 5, size=int(rng.integers(0, 3))))
        out.append(qcpgen.small_mixed(200 + i, n=n, n_zero=n // 8, n_nonneg=nn, soc=soc, psd=psd,
                                      n_exp=int(rng.integers(0, 3)), A_density=0.15,
                                      P_rank=max(1, (3 * n) // 4), P_eps=0.05,
                                      nonneg_active=nn // 3))
    return out


def test_batch_grid_agrees_and_tunes(tmp_path):
    qs = small_batch()
    bt = batch_to_device(qs)
    hb = Q.qcpd_batch_create(*batch_create_args(bt), opts=Q.Opts(tol=1e-10))
    ref = Q.qcpd_batch_jvp(hb, bt["dP"], bt["dA"], bt["dq"], bt["db"])
    print("batch iters", [i.iters for i in ref[3]], flush=True)
    assert ref[4] == Q.QCPD_OK
    grid, dflt = qcpd_batch_get_launch(hb)
    assert grid == dflt and 1 <= grid <= len(qs)
    for g in (1, 3, 100, 0):
        qcpd_batch_set_launch(hb, g)
        out = Q.qcpd_batch_jvp(hb, bt["dP"], bt["dA"], bt["dq"], bt["db"])
        print(f"grid {g}: status {out[4]}, {out[3][0].ms_total:.2f} ms", flush=True)
        assert out[4] == Q.QCPD_OK
        # each problem runs on one workgroup whatever the grid: identical bits
        for a, b in zip(out[:3], ref[:3]):
            assert torch.equal(a, b)
    r = T.tune_batch(hb, (bt["dP"], bt["dA"], bt["dq"], bt["db"]), Q.Opts(tol=1e-10),
                     iters=30, reps=1, cache=T.TuneCache(str(tmp_path / "t.json")),
                     grids=[1, 4, len(qs)])
    print("batch tuned", r, flush=True)
    assert r["grid"] in (1, 4, len(qs)) and qcpd_batch_get_launch(hb)[0] == r["grid"]
    out = Q.qcpd_batch_jvp(hb, bt["dP"], bt["dA"], bt["dq"], bt["db"])
    for a, b in zip(out[:3], ref[:3]):
        assert torch.equal(a, b)
    hb.close()


def test_batch_lane_schedule_tunes_and_agrees(tmp_path):
    """The batch's entries per lane (a create-time choice): every candidate gives the same
    derivative up to the order of sums; the tuner returns a handle built with its choice,
    and the cache hands the same choice back."""
    qs = small_batch()
    bt = batch_to_device(qs)
    args = batch_create_args(bt)
    inputs = (bt["dP"], bt["dA"], bt["dq"], bt["db"])
    refs = {}
    for spl in (4, 32, 128):
        hb = Q.qcpd_batch_create(*args, opts=Q.Opts(tol=1e-12, nnz_per_lane_F=spl))
        out = Q.qcpd_batch_jvp(hb, *inputs)
        hb.close()
        assert out[4] == Q.QCPD_OK
        refs[spl] = out[:3]
    for spl in (4, 128):
        d = max(rel(a, b) for a, b in zip(refs[spl], refs[32]))
        print(f"entries per lane {spl} vs 32: {d:.2e}", flush=True)
        assert d <= 1e-9
    cache = T.TuneCache(str(tmp_path / "lanes.json"))
    make = lambda o: Q.qcpd_batch_create(*args, opts=o)
    hb, o, r = T.tune_batch_lanes(make, inputs, Q.Opts(tol=1e-12), candidates=(4, 32, 128),
                                  iters=30, reps=1, cache=cache)
    print("lanes tuned", r, flush=True)
    assert not r["cached"] and r["nnz_per_lane"] in (4, 32, 128)
    assert o.nnz_per_lane_F == r["nnz_per_lane"] and o.tol == 1e-12
    out = Q.qcpd_batch_jvp(hb, *inputs)
    assert out[4] == Q.QCPD_OK
    assert max(rel(a, b) for a, b in zip(out[:3], refs[32])) <= 1e-9
    hb.close()
    hb2, o2, r2 = T.tune_batch_lanes(make, inputs, Q.Opts(tol=1e-12), cache=cache)
    assert r2["cached"] and o2.nnz_per_lane_F == r["nnz_per_lane"]
    hb2.close()
