"""GPU: the job server.  A job's results are the same alone and in a mix
(bit for bit: lattice, accepted moves, N_AB, histogram), whatever the chunk
size, arrival pattern or HBM budget; admission is FIFO and never exceeds the
budget; invalid or oversized jobs are refused at submission."""
import sys

import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import serve
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mix():
    # resident and tiled, int8 and bit-packed, a job of 1 sweep, omega of both signs
    specs = [(64, "int8", 0.5, 0.5, 75), (96, "bitpacked", 0.3, 1.2, 1), (100, "int8", 0.6, 0.9, 40),
             (128, "bitpacked", 0.7, -0.4, 111), (320, "bitpacked", 0.35, 1.1, 23), (36, "int8", 0.5, 0.0, 64),
             (256, "int8", 0.2, 1.4, 50), (544, "bitpacked", 0.5, 0.88, 9)]
    return [wl.Job(L=L, composition=x, omega=w, seed=wl.job_seed(88, i), sweeps=n, layout=lay)
            for i, (L, lay, x, w, n) in enumerate(specs)]


def alone_result(j):
    s = kk.Sim(j.L, j.composition, j.omega, j.seed, layout=j.layout)
    s.sweep(j.sweeps)
    out = (s.get_lattice(), s.stats(), s.energy(), s.cluster_hist(1))
    s.close()
    return out


def check_same(srv, jid, res, j):
    lat, stats, (nab, e), hist = alone_result(j)
    assert res["status"] == kk.KK_OK
    assert res["sweeps"] == j.sweeps and res["attempts"] == stats[1]
    assert res["accepted"] == stats[2], (j.L, res["accepted"], stats[2])
    assert res["n_unlike"] == nab and res["energy_kT"] == e
    assert srv.job_hist(jid) == hist
    assert np.array_equal(srv.job_lattice(jid), lat)


@pytest.mark.parametrize("chunk", [37, 1000])
def test_server_mix_equals_alone(chunk):
    jobs = mix()
    say(f"case server mix of {len(jobs)} jobs, chunk {chunk}")
    srv = kk.Server(chunk_sweeps=chunk, keep_lattice=True)
    ids = {}
    # staggered arrivals: half now, the rest after two steps (they join mid-way)
    for j in jobs[:4]:
        ids[srv.submit(j)] = j
    srv.step()
    srv.step()
    for j in jobs[4:]:
        ids[srv.submit(j)] = j
    results = []
    for _ in range(10_000):
        active, queued = srv.step()
        results += srv.poll()
        if active == 0 and queued == 0 and len(results) == len(jobs):
            break
    assert len(results) == len(jobs)
    for r in results:
        say(f"  job {r['id']}: L={r['L']} sweeps={r['sweeps']}")
        check_same(srv, r["id"], r, ids[r["id"]])
        srv.release(r["id"])
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["bytes_in_use"] == 0
    srv.close()


def test_server_small_budget_queues_fifo():
    jobs = mix()
    fp = [kk.server_job_bytes(j, keep_lattice=True) for j in jobs]
    budget = max(fp) + min(fp)   # the largest job fits, but rarely with much beside it
    say(f"case server budget {budget} bytes")
    srv = kk.Server(hbm_budget_bytes=budget, chunk_sweeps=20, keep_lattice=True)
    ids = {srv.submit(j): j for j in jobs}
    a, q = srv.step()
    assert q > 0, "the budget should hold some jobs back"
    results = srv.poll()
    for _ in range(10_000):
        a, q = srv.step()
        results += srv.poll()
        if a == 0 and q == 0:
            break
    assert len(results) == len(jobs)
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["budget"] == budget
    # FIFO admission: admission times follow submission order
    adm = [r["t_admit"] for r in sorted(results, key=lambda r: r["id"])]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    for r in results:
        check_same(srv, r["id"], r, ids[r["id"]])
    srv.close()


def test_server_matches_oracle():
    j = wl.Job(L=64, composition=0.45, omega=0.8, seed=12345, sweeps=33, layout="int8")
    srv = kk.Server(chunk_sweeps=10, keep_lattice=True)
    jid = srv.submit(j)
    while srv.step() != (0, 0):
        pass
    (r,) = srv.poll()
    ref = oracle.init(j.L, j.composition, j.seed)
    acc = oracle.sweeps(ref, j.omega, j.seed, 0, j.sweeps)
    assert np.array_equal(srv.job_lattice(jid), ref)
    assert r["accepted"] == acc
    assert r["n_unlike"] == oracle.energy(ref)
    assert srv.job_hist(jid) == oracle.cluster_hist(ref, 1)
    srv.close()


def test_server_refuses_bad_jobs():
    srv = kk.Server(hbm_budget_bytes=1 << 20)
    with pytest.raises(kk.KKError) as e:
        srv.submit(wl.Job(L=1024, composition=0.5, omega=1.0, seed=1, sweeps=1, layout="bitpacked"))
    assert e.value.status == kk.KK_ENOMEM
    with pytest.raises(kk.KKError) as e:
        srv.submit(wl.Job(L=66, composition=0.5, omega=1.0, seed=1, sweeps=1, layout="int8"))
    assert e.value.status == kk.KK_EINVAL
    with pytest.raises(kk.KKError) as e:
        srv.submit(wl.Job(L=96, composition=0.5, omega=float("nan"), seed=1, sweeps=1, layout="int8"))
    assert e.value.status == kk.KK_EINVAL
    with pytest.raises(kk.KKError) as e:
        srv.submit(wl.Job(L=100, composition=0.5, omega=1.0, seed=1, sweeps=1, layout="bitpacked"))
    assert e.value.status == kk.KK_EINVAL
    # a job of zero sweeps finishes at admission with the placed lattice
    jid = srv.submit(wl.Job(L=64, composition=0.5, omega=1.0, seed=3, sweeps=0, layout="int8"))
    srv.step()
    (r,) = srv.poll()
    assert r["id"] == jid and r["status"] == kk.KK_OK and r["sweeps"] == 0
    assert r["n_unlike"] == oracle.energy(oracle.init(64, 0.5, 3))
    with pytest.raises(kk.KKError):
        srv.job_lattice(jid)   # keep_lattice is off
    srv.close()


def test_replay_small_trace():
    jobs = wl.serving_trace(n_jobs=24, rate=400.0, sides=(64, 96, 128, 256, 320), sweeps_lo=10, sweeps_hi=400)
    say("case replay of a 24-job trace")
    srv = kk.Server(chunk_sweeps=50)
    out = serve.replay(jobs, srv)
    srv.close()
    assert out["jobs"] == 24 and out["failed"] == 0
    assert 0 < out["latency_p50_s"] <= out["latency_p99_s"]
    assert out["attempts"] == sum(j.L * j.L * j.sweeps for j in jobs)


def test_server_segregated_job_matches_oracle():
    j = wl.Job(L=64, composition=0.45, omega=0.8, seed=12345, sweeps=25, layout="int8", start="segregated")
    srv = kk.Server(chunk_sweeps=10, keep_lattice=True)
    jid = srv.submit(j)
    while srv.step() != (0, 0):
        pass
    (r,) = srv.poll()
    ref = oracle.init_segregated(j.L, j.composition)
    acc = oracle.sweeps(ref, j.omega, j.seed, 0, j.sweeps)
    assert np.array_equal(srv.job_lattice(jid), ref)
    assert r["accepted"] == acc
    srv.close()
