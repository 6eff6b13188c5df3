"""Serving loop: requests of uneven size batched as they arrive; every result equals the
structure evaluated alone, and admission respects the HBM budget."""
import time

import numpy as np
import pytest

from gpu_common import log, write_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from paper_2402_03789_amd.serve import Server, replay, latency_summary  # noqa: E402
from synth import model_spec_real, serving_stream  # noqa: E402

ALL_Z = tuple(range(1, 90))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    path, _ = write_model(tmp_path_factory.mktemp("m"), model_spec_real(ALL_Z), 105)
    return sn.Model(path)


def _drain(srv, count, timeout_s=120):
    out = {}
    t_end = time.time() + timeout_s
    while len(out) < count and time.time() < t_end:
        for r in srv.poll(timeout_ms=100):
            out[r["ticket"]] = r
    assert len(out) == count
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_served_results_equal_alone(model, precision):
    stream = serving_stream(count=40, seed=21, n_min=8, n_max=600)
    log(f"serve {precision}: {len(stream)} requests")
    srv = Server(model, n_streams=3, precision=precision, max_batch_atoms=2000)
    tickets = [srv.submit(s.pos, s.Z, s.cell) for _, s in stream]
    res = _drain(srv, len(tickets))
    srv.close()
    ctx = sn.Context(model, precision=precision)
    batched = 0
    for tk, (_, s) in zip(tickets, stream):
        r = res[tk]
        assert r["status"] == 0
        batched += r["batch_structures"] > 1
        alone = ctx.compute(s.pos, s.Z, s.cell)
        assert r["energy"] == alone["energy"]
        np.testing.assert_array_equal(r["forces"], alone["forces"])
        np.testing.assert_array_equal(r["atom_energy"], alone["atom_energy"])
        np.testing.assert_array_equal(r["virial"], alone["virial"])
        assert r["batch_atoms"] <= 2000 or r["batch_structures"] == 1
    log(f"  {batched} of {len(tickets)} requests ran in batches of more than one structure")
    assert batched > 0


def test_replay_with_arrivals_and_budget(model):
    stream = serving_stream(count=60, seed=22, n_min=8, n_max=300, rate=400.0)
    budget = 3 * 512 * 2 ** 20  # 512 MiB per worker
    srv = Server(model, n_streams=3, precision="fp32", hbm_budget=budget)
    rep = replay(srv, stream)
    srv.close()
    summ = latency_summary(rep)
    log(f"  replay: {summ}")
    ctx = sn.Context(model, precision="fp32")
    for r, (_, s) in zip(rep["results"], stream[:5]):
        alone = ctx.compute(s.pos, s.Z, s.cell)
        assert r["energy"] == alone["energy"]
    assert summ["p99_ms"] >= summ["p50_ms"] > 0


def test_structure_too_large_for_budget(model):
    from synth import sio2_box
    big = sio2_box(400, seed=3)  # 1200 atoms
    small = sio2_box(8, seed=4)
    srv = Server(model, n_streams=1, precision="fp32", hbm_budget=64 * 2 ** 20)
    t_big = srv.submit(big.pos, big.Z, big.cell)
    t_small = srv.submit(small.pos, small.Z, small.cell)
    res = _drain(srv, 2)
    srv.close()
    assert res[t_big]["status"] == sn._lib.SN_ENOMEM
    assert res[t_small]["status"] == 0


def test_bad_request_fails_alone(model):
    """A request the device rejects (two atoms at one position) fails by itself; the
    requests batched with it get the results they get alone.  One with an atomic number
    outside the model is refused at submit."""
    from synth import sio2_box
    good = [sio2_box(n, seed=40 + n) for n in (8, 12, 16)]
    bad = sio2_box(10, seed=45)
    bad_pos = bad.pos.copy()
    bad_pos[3] = bad_pos[7]  # r = 0 pair: found only by the graph build on the device
    log("serve: one r = 0 request among good ones")
    srv = Server(model, n_streams=1, precision="fp32", max_batch_atoms=4000)
    with pytest.raises(sn.SNError):
        srv.submit(good[0].pos, np.full(good[0].n, 120, np.int32), good[0].cell)
    with pytest.raises(sn.SNError):
        p = good[0].pos.copy()
        p[0, 0] = np.nan
        srv.submit(p, good[0].Z, good[0].cell)
    # hold the worker on a first request so the next four queue up and form one batch
    first = srv.submit(good[0].pos, good[0].Z, good[0].cell)
    tickets = [srv.submit(s.pos, s.Z, s.cell) for s in good[1:2]]
    t_bad = srv.submit(bad_pos, bad.Z, bad.cell)
    tickets += [srv.submit(s.pos, s.Z, s.cell) for s in good[2:]]
    res = _drain(srv, 4, timeout_s=60)
    srv.close()
    log(f"  batch sizes: {[res[t]['batch_structures'] for t in [first] + tickets + [t_bad]]}")
    assert res[t_bad]["status"] == sn._lib.SN_EINVAL
    assert res[first]["status"] == 0
    ctx = sn.Context(model, precision="fp32")
    for tk, s in zip(tickets, good[1:]):
        assert res[tk]["status"] == 0
        alone = ctx.compute(s.pos, s.Z, s.cell)
        assert res[tk]["energy"] == alone["energy"]
        np.testing.assert_array_equal(res[tk]["forces"], alone["forces"])


def test_warmup_every_worker_then_results_unchanged(model):
    from paper_2402_03789_amd._lib import SNError
    stream = serving_stream(count=12, seed=23, n_min=8, n_max=400)
    srv = Server(model, n_streams=3, precision="fp32", max_batch_atoms=2000)
    big = max((s for _, s in stream), key=lambda s: s.n)
    log(f"warm-up with {big.n} atoms on 3 workers")
    srv.warmup(big.pos, big.Z, big.cell)
    srv.warmup(stream[0][1].pos, stream[0][1].Z, stream[0][1].cell)  # a second round
    bad_Z = np.array(big.Z, copy=True)
    bad_Z[0] = 120  # outside the model's species table
    with pytest.raises(SNError):
        srv.warmup(big.pos, bad_Z, big.cell)
    tickets = [srv.submit(s.pos, s.Z, s.cell) for _, s in stream]
    res = _drain(srv, len(tickets))
    srv.close()
    ctx = sn.Context(model, precision="fp32")
    for tk, (_, s) in zip(tickets, stream):
        r = res[tk]
        assert r["status"] == 0
        alone = ctx.compute(s.pos, s.Z, s.cell)
        assert r["energy"] == alone["energy"]
        np.testing.assert_array_equal(r["forces"], alone["forces"])
