"""Serving by continuous batching: queries admitted by memory footprint into a
resident slot table, one round per step for every resident query (a two-deep
pipeline: a step enqueues a round and reads back the previous one).  Each
result equals what the query gives alone; admission respects the pools; a
failing query fails alone."""
import numpy as np
import pytest

from paper_2601_04185_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_2601_04185_amd as pk
    assert torch.cuda.is_available()
    return pk


def _queries():
    specs = [(3000, 0.4, dict(fixed_samples=2048, batch=1024)),
             (15000, 0.12, dict(confidence=0.999, batch=1024, min_iters=1024, max_iters=8192)),
             (800, 0.6, dict(confidence=0.999, batch=512, min_iters=512, max_iters=4096, lo_top_k=2)),
             (2, 0.5, dict(fixed_samples=64)),
             (30000, 0.3, dict(confidence=0.9999, batch=1024, min_iters=1024, max_iters=6000,
                               max_score_points=4000)),
             (6000, 0.25, dict(fixed_samples=3000, batch=1024))]
    qs, ps = [], []
    for i, (n, e, kw) in enumerate(specs):
        qs.append(synth.make_query(600 + i, n, e, 1.0, weights="conf" if i % 2 else "ones"))
        ps.append(dict(threshold_px=4.0, query_id=i, **kw))
    return qs, ps


def _run_server(pk, srv, qs, P, arrive_every=0):
    tickets, out, pending, i, steps = {}, {}, set(), 0, 0
    while len(out) < len(qs):
        while i < len(qs) and (arrive_every == 0 or steps >= i * arrive_every):
            tickets[srv.submit(pk.to_device(qs[i]), qs[i].K, P[i])] = i
            pending.add(i)
            i += 1
        done, resident, queued = srv.step()
        steps += 1
        cand, byt = srv.usage()
        assert cand <= srv.cfg.candidate_pool and byt <= srv.cfg.byte_pool
        for t in done:
            out[tickets[t]] = srv.poll(t)
        assert steps < 500
    return out, steps


def _check_alone(pk, qs, P, out):
    ctx = pk.Context(0)
    for k, (q, p) in enumerate(zip(qs, P)):
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, pk.to_device(q), q.K, p)
        src, sR, stt, sst = out[k]
        assert src == rc, k
        assert np.array_equal(sR, R) and np.array_equal(stt, t), k
        for key in ("samples", "candidates", "best_count", "full_count", "batches", "best_h", "best_j", "best_msac"):
            assert sst[key] == st[key], (k, key)


def test_server_results_equal_alone(pk):
    qs, ps = _queries()
    P = [pk.make_params(**p) for p in ps]
    srv = pk.Server(0, max_slots=8, max_top_k=8, max_n=40000)
    out, steps = _run_server(pk, srv, qs, P)
    _check_alone(pk, qs, P, out)
    assert out[3][0] == pk.IMLOC_NO_POSE  # the 2-point query fails alone
    srv.close()


def test_server_small_pools_queue_and_finish(pk):
    qs, ps = _queries()
    P = [pk.make_params(**p) for p in ps]
    # two slots and room for about two rounds' candidates: queries wait in the queue
    srv = pk.Server(0, max_slots=2, max_top_k=8, max_n=40000, candidate_pool=4 * 3000 + 4 * 1024,
                    byte_pool=300000)
    out, steps = _run_server(pk, srv, qs, P)
    _check_alone(pk, qs, P, out)
    srv.close()


def test_server_interleaved_arrivals(pk):
    qs, ps = _queries()
    P = [pk.make_params(**p) for p in ps]
    srv = pk.Server(0, max_slots=4, max_top_k=8, max_n=40000)
    out, steps = _run_server(pk, srv, qs, P, arrive_every=2)
    _check_alone(pk, qs, P, out)
    srv.close()


def test_server_one_slot_pipeline(pk):
    """One slot: every query reuses it right after the previous one leaves,
    while the pipeline has a round in flight; results equal alone, and once
    everything is reported further steps do nothing."""
    qs, ps = _queries()
    P = [pk.make_params(**p) for p in ps]
    srv = pk.Server(0, max_slots=1, max_top_k=8, max_n=40000, candidate_pool=4 * 3000 + 4 * 1024,
                    byte_pool=300000)
    out, steps = _run_server(pk, srv, qs, P)
    _check_alone(pk, qs, P, out)
    for _ in range(3):
        done, resident, queued = srv.step()
        assert done == [] and resident == 0 and queued == 0
    srv.close()
