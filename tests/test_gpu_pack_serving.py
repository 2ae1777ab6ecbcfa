"""GPU tests of the batched pack (one launch per kernel per step over many
domains, captured in a HIP graph) and of the continuous-batching server:
every domain's result is bitwise the same alone and in the mix."""
import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import lib, log

pytestmark = pytest.mark.gpu


def _domains(prec, count, seed):
    r = pfinputs.SplitMix64(seed)
    out = []
    for i in range(count):
        L = 20 + int(60 * r.u())
        ny = 10 + int(50 * r.u())
        nz = 12 + int(40 * r.u())
        G = 5e-4 + 1.5e-3 * r.u()
        v = 0.005 + 0.015 * r.u()
        hs = nz // 4
        p = pfinputs.p0_params(solid_height=hs, G=G, v=v)
        out.append({"shape": (nz, ny, L), "prec": prec, "params": p, "seed": r.next(),
                    "nseeds": max(3, L * ny // 300), "hs": hs, "steps": 5 + int(30 * r.u())})
    return out


def _alone(pf, w):
    d = pf.Domain(w["shape"], w["prec"])
    d.set_params(w["params"])
    d.init_voronoi(w["seed"], w["nseeds"], w["hs"])
    d.step(w["steps"])
    out = d.read()
    d.close()
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_pack_matches_single_domain_bitwise(prec):
    pf = lib()
    pf.set_variant(1)
    ws = _domains(prec, 7, 11 if prec == "fp32" else 12)
    log(f"case pack {prec}: " + ", ".join(f"{w['shape']}x{w['steps']}" for w in ws))
    alone = [_alone(pf, w) for w in ws]
    pk = pf.Pack(prec, max_domains=16)
    doms = []
    for w in ws:
        d = pf.Domain(w["shape"], prec)
        d.set_params(w["params"])
        d.init_voronoi(w["seed"], w["nseeds"], w["hs"])
        pk.add(d, w["steps"])
        doms.append(d)
    longest = max(w["steps"] for w in ws)
    # uneven rounds; every member idles once its own steps are done; the
    # fields of some members are read to the host between rounds (staged in
    # their second copy), which must not change what follows
    done = 0
    for i, r in enumerate((3, 1, 7, longest)):
        fin = pk.step(r, count_finished=True)
        done += r
        assert fin == sum(w["steps"] <= done for w in ws)
        if i < 2:
            for d in doms[i::3]:
                d.read()
    for w, d, a in zip(ws, doms, alone):
        assert pk.remaining(d) == 0
        assert d.step_index == w["steps"]
        got = d.read()
        assert np.array_equal(got[0], a[0]) and np.array_equal(got[1], a[1])
    # a member removed from the pack continues on its own like any domain
    pk.remove(doms[0])
    doms[0].step(2)
    assert doms[0].step_index == ws[0]["steps"] + 2
    pk.close()
    for d in doms:
        d.close()


def test_pack_member_refuses_reconfiguration():
    """A member's descriptor and step budget belong to its pack's captured
    step: set_params, init_fields and set_time on a member are refused with
    STATE and leave it stepping as before; after removal they work again."""
    import paper_1506_01684_amd as pfmod

    pf = lib()
    pf.set_variant(1)
    w = _domains("fp64", 1, 5)[0]
    log(f"case pack member refusal: {w['shape']}")
    ref = _alone(pf, w)
    pk = pf.Pack("fp64", max_domains=4)
    d = pf.Domain(w["shape"], "fp64")
    d.set_params(w["params"])
    d.init_voronoi(w["seed"], w["nseeds"], w["hs"])
    pk.add(d, w["steps"])
    pk.step(2)
    for call in (lambda: d.set_params(w["params"]),
                 lambda: d.init_voronoi(w["seed"], w["nseeds"], w["hs"]),
                 lambda: d.set_time(0)):
        with pytest.raises(pfmod.PfError) as e:
            call()
        assert e.value.status == 2  # PF_ERR_STATE
    pk.step(w["steps"])
    assert pk.remaining(d) == 0 and d.step_index == w["steps"]
    got = d.read()
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    pk.remove(d)
    d.set_time(0)
    assert d.step_index == 0
    d.close()
    pk.close()


def test_pack_graph_replays_match_eager_oracle_on_small_domain():
    """A graph-replayed pack step equals the oracle (FP64, 1e-12)."""
    pf = lib()
    shape = (16, 12, 20)
    p = pfinputs.p0_params(solid_height=4)
    p["dt"] = oracle.default_dt(p, shape)
    d = pf.Domain(shape, "fp64")
    d.set_params(p)
    d.init_voronoi(5, 4, 4)
    pk = pf.Pack("fp64", max_domains=4)
    pk.add(d, 12)
    for _ in range(4):
        pk.step(3)
        pk.sync()  # eager synchronisation between replays
    phi_g, mu_g = d.read()
    phi0, mu0 = oracle.init_voronoi(shape, 5, 4, 4)
    phi_o, mu_o = oracle.run(p, phi0, mu0, 12)
    err = max(np.max(np.abs(phi_g - phi_o)), np.max(np.abs(mu_g - mu_o)) / np.max(np.abs(mu_o)))
    log(f"graph replay vs oracle: {err:.2e}")
    assert err <= 1e-12
    pk.close()
    d.close()


def _requests(n, seed, nan_id=None):
    from paper_1506_01684_amd.serving import Request, request_from_trace

    tr = pfinputs.serving_trace(count=n, rate=200.0, seed=seed, lateral=(16, 48), steps=(10, 60))
    reqs = [request_from_trace(t, keep_fields=True) for t in tr]
    if nan_id is not None:
        r = reqs[nan_id]
        phi, mu = pfinputs.random_state(r.shape, 1)
        phi[0, 1, 2, 3] = np.nan
        reqs[nan_id] = Request(r.id, r.arrival, r.shape, r.prec, r.steps, r.params, r.seed,
                               r.nseeds, r.solid_height, True, (phi, mu))
    return reqs


def test_server_results_equal_alone_runs_bitwise():
    from paper_1506_01684_amd.serving import GpuBackend, Server, run_serial_gpu, summarize

    lib().set_variant(1)
    reqs = _requests(10, 21)
    log("case server mix: " + ", ".join(f"{r.prec}{r.shape}x{r.steps}" for r in reqs))
    be = GpuBackend(max_domains=16)
    budget = 3 * max(be.required_bytes(r) for r in reqs)  # forces queueing
    srv = Server(be, budget_bytes=budget, max_slots=4, round_steps=7)
    res = srv.run(reqs)
    be.shutdown()
    alone = run_serial_gpu(reqs)
    for a, b in zip(res, alone):
        assert a.ok and b.ok, (a.error, b.error)
        assert np.array_equal(a.fields[0], b.fields[0]) and np.array_equal(a.fields[1], b.fields[1])
    s = summarize(res)
    log(f"server: {s}")
    assert max(u for *_, u in srv.events) <= budget


def test_server_isolates_a_failing_request():
    from paper_1506_01684_amd.serving import GpuBackend, Server, run_serial_gpu

    reqs = _requests(6, 22, nan_id=2)
    be = GpuBackend(max_domains=8)
    res = Server(be, budget_bytes=64e9, max_slots=8, round_steps=5).run(reqs)
    be.shutdown()
    assert not res[2].ok and "non-finite" in res[2].error
    good = [r for r in reqs if r.id != 2]
    alone = {r.id: r for r in run_serial_gpu(good)}
    for r in res:
        if r.id == 2:
            continue
        assert r.ok
        a = alone[r.id]
        assert np.array_equal(r.fields[0], a.fields[0]) and np.array_equal(r.fields[1], a.fields[1])


def test_server_cancellation_leaves_others_unchanged():
    """A request withdrawn early (in the queue or after its first round)
    ends as cancelled; every other request's fields are bitwise those of its
    run alone."""
    import dataclasses

    from paper_1506_01684_amd.serving import GpuBackend, Server, run_serial_gpu

    lib().set_variant(1)
    reqs = _requests(6, 23)
    reqs[1] = dataclasses.replace(reqs[1], steps=400, cancel_at=reqs[1].arrival + 1e-6)
    be = GpuBackend(max_domains=8)
    res = Server(be, budget_bytes=64e9, max_slots=8, round_steps=5).run(reqs)
    be.shutdown()
    log("case cancel: " + ", ".join(f"{r.id}:{'ok' if r.ok else r.error}" for r in res))
    assert not res[1].ok and res[1].error.startswith("cancelled")
    good = [r for r in reqs if r.id != 1]
    alone = {r.id: r for r in run_serial_gpu(good)}
    for r in res:
        if r.id == 1:
            continue
        assert r.ok
        a = alone[r.id]
        assert np.array_equal(r.fields[0], a.fields[0]) and np.array_equal(r.fields[1], a.fields[1])
