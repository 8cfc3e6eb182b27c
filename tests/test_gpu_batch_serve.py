"""The batched plan (one persistent launch over several codes, replayed
from a HIP graph) and the continuous-batching server give every shot
exactly the result it gets alone (and that the oracle gives)."""
import numpy as np
import pytest

from paper_2609_38139_amd import codes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2609_38139_amd import laim
    laim.lib()
    return laim


MIX = [  # code, p, q, bp, rounds, shots, shot0
    ("toric2d:8", 0.05, 0.05, "minsum", 32, 500, 0),
    ("bb:12x6", 0.01, 0.05, "minsum", 64, 300, 1000),
    ("toric3d_point:4", 0.02, 0.05, "sumproduct", 16, 200, 7),
    ("toric3d_membrane:3", 0.05, 0.125, "minsum", 12, 150, 3),
    ("toric2d:16", 0.05, 0.05, "sumproduct", 64, 100, 99),
    ("bb:6x6", 0.02, 0.05, "sumproduct", 32, 257, 5),
]


def _mix(L):
    import torch
    out = []
    for name, p, q, bp, R, S, s0 in MIX:
        spec = codes.by_name(name)
        code = L.Code(spec, 0)
        P = L.DecodeParams(bp=bp, q=q, rounds=R)
        e0 = L.sample_noise(code, p, 1, s0, S)
        out.append({"spec": spec, "code": code, "params": P, "e0": e0, "shot0": s0})
    torch.cuda.synchronize()
    return out


def test_batch_plan_matches_single_launches_and_oracle(L, orc):
    import torch
    mix = _mix(L)
    plan = L.BatchPlan(mix)
    singles = []
    for it in mix:
        r = L.decode_rounds(it["code"], it["params"], it["e0"], shot0=it["shot0"])
        r["fail"] = L.logical_failure(it["code"], it["e0"], r["z"])
        singles.append(r)
    torch.cuda.synchronize()
    for replay in range(3):
        print(f"[batch] replay {replay}", flush=True)
        outs = plan.launch()
        torch.cuda.synchronize()
        for it, o, ref in zip(mix, outs, singles):
            for k in ("z", "s", "tclr", "fail"):
                assert torch.equal(o[k], ref[k]), (it["spec"].name, k, replay)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
    # and the oracle on a slice of every item
    for it, ref in zip(mix, singles):
        P = it["params"]
        e0 = it["e0"][:40].cpu().numpy()
        o = orc.decode(it["spec"], orc.DecodeParams(bp=P.bp, q=P.q, rounds=P.rounds), e0,
                       shot0=it["shot0"], nthreads=8)
        assert np.array_equal(ref["z"][:40].cpu().numpy(), o["z"])
        assert np.array_equal(ref["tclr"][:40].cpu().numpy(), o["tclr"])


def _serve(L, mix, order, budget=1 << 30, slots=4096):
    srv = L.Server(0, budget, slots)
    pending = {}
    rounds_seen = {}
    submitted = 0
    results = {}
    it_order = list(order)
    while it_order or pending:
        # admit a few new requests per step: arrivals interleave with work
        for _ in range(7):
            if not it_order:
                break
            i, k = it_order.pop(0)
            it = mix[i]
            e0 = it["e0"][k].cpu().numpy()
            t = srv.submit(it["code"], it["params"], it["shot0"] + k, e0)
            pending[t] = (i, k)
            submitted += 1
        for ev in srv.step():
            assert ev["round"] == rounds_seen.get(ev["ticket"], 0) + 1
            rounds_seen[ev["ticket"]] = ev["round"]
            if ev["done"]:
                i, k = pending.pop(ev["ticket"])
                r = srv.result(ev["ticket"])
                r["fail"] = ev["fail"]
                results[(i, k)] = r
    return results, srv


def test_server_results_equal_alone_and_in_any_mix(L):
    import torch
    mix = _mix(L)
    singles = []
    for it in mix:
        r = L.decode_rounds(it["code"], it["params"], it["e0"], shot0=it["shot0"])
        r["fail"] = L.logical_failure(it["code"], it["e0"], r["z"])
        singles.append({k: v.cpu().numpy() for k, v in r.items() if k != "workspace" and v is not None})
    torch.cuda.synchronize()
    reqs = [(i, k) for i, it in enumerate(mix) for k in range(0, it["e0"].shape[0], 9)]
    rng = np.random.default_rng(3)
    for trial, order in enumerate([reqs, [reqs[j] for j in rng.permutation(len(reqs))]]):
        print(f"[serve] trial {trial}: {len(order)} requests", flush=True)
        res, _ = _serve(L, mix, order)
        assert len(res) == len(order)
        for (i, k), r in res.items():
            ref = singles[i]
            assert np.array_equal(r["z"], ref["z"][k]), (i, k)
            assert np.array_equal(r["s"], ref["s"][k]), (i, k)
            assert r["tclr"] == ref["tclr"][k], (i, k)
            assert r["fail"] == ref["fail"][k], (i, k)


def test_server_admits_by_memory(L):
    """With room for only a few requests the rest wait (FIFO) and still get
    the same results."""
    import torch
    mix = _mix(L)[:2]
    singles = [L.decode_rounds(it["code"], it["params"], it["e0"], shot0=it["shot0"]) for it in mix]
    torch.cuda.synchronize()
    order = [(i, k) for i in range(2) for k in range(12)]
    res, srv = _serve(L, mix, order, budget=64 * 1024, slots=64)
    for (i, k), r in res.items():
        assert np.array_equal(r["z"], singles[i]["z"][k].cpu().numpy())
        assert r["tclr"] == int(singles[i]["tclr"][k])
    st = srv.stats()
    assert st["resident"] == 0 and st["waiting"] == 0 and st["bytes"] == 0


def _plan_sampled(L, orc, spec_list, nsample=4, seed=1):
    """Builds one batched plan over (name, p, q, rounds, shots) items,
    launches it twice and checks sampled shots of every item against the
    oracle and every shot against s = H (e0 ^ z) and t_clr >= 0 <=> s = 0."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    items = []
    for name, p, q, R, S in spec_list:
        spec = codes.by_name(name)
        code = L.Code(spec, 0)
        P = L.DecodeParams(q=q, rounds=R)
        e0 = L.sample_noise(code, p, seed, 0, S)
        items.append({"spec": spec, "code": code, "params": P, "e0": e0, "shot0": 0})
    torch.cuda.synchronize()
    plan = L.BatchPlan(items)
    for replay in range(2):
        print(f"[batch] {len(items)} items, replay {replay}", flush=True)
        outs = plan.launch()
        torch.cuda.synchronize()
        if replay == 0:
            first = [{k: o[k].clone() for k in ("z", "s", "tclr", "fail")} for o in outs]
    for it, o, f0 in zip(items, outs, first):
        for k in ("z", "s", "tclr", "fail"):
            assert torch.equal(o[k], f0[k]), (it["spec"].name, k)
        s_full = L.syndrome(it["code"], it["e0"] ^ o["z"])
        assert torch.equal(s_full, o["s"]), it["spec"].name
        assert torch.equal(o["s"].any(1), o["tclr"] < 0), it["spec"].name
    jobs = []
    rng = np.random.default_rng(7)
    for j, (it, o) in enumerate(zip(items, outs)):
        S = it["e0"].shape[0]
        for i in sorted(set([0, S - 1] + rng.integers(0, S, nsample - 2).tolist())):
            jobs.append((j, int(i)))
    P_or = [orc.DecodeParams(q=it["params"].q, rounds=it["params"].rounds) for it in items]
    e0s = {(j, i): items[j]["e0"][i:i + 1].cpu().numpy() for j, i in jobs}
    with ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(lambda ji: orc.decode(items[ji[0]]["spec"], P_or[ji[0]], e0s[ji], shot0=ji[1]), jobs))
    for (j, i), r in zip(jobs, refs):
        o = outs[j]
        assert np.array_equal(o["z"][i].cpu().numpy(), r["z"][0]), (items[j]["spec"].name, i)
        assert int(o["tclr"][i]) == int(r["tclr"][0]), (items[j]["spec"].name, i)
        fo = orc.logical_failure(items[j]["spec"], e0s[(j, i)], r["z"])
        assert int(o["fail"][i]) == int(fo[0]), (items[j]["spec"].name, i)


@pytest.mark.timeout(900)
def test_batch_plan_3d_toric_mixed_sizes(L, orc):
    """Both 3D toric sectors at L = 8, 16, 24 in one plan, 16384 shots each,
    4L rounds (min-sum). Codes whose shot does not fit the LDS (point L=24,
    membrane L=16 and 24) run in the stream form inside the same graph."""
    _plan_sampled(L, orc, [("toric3d_point:8", 0.03, 0.05, 32, 16384),
                           ("toric3d_point:16", 0.03, 0.05, 64, 16384),
                           ("toric3d_point:24", 0.03, 0.05, 96, 16384),
                           ("toric3d_membrane:8", 0.03, 0.125, 32, 16384),
                           ("toric3d_membrane:16", 0.03, 0.125, 64, 16384),
                           ("toric3d_membrane:24", 0.03, 0.125, 96, 16384)], nsample=3)


@pytest.mark.timeout(900)
def test_batch_plan_bivariate_bicycle_with_toric(L, orc):
    """BB (6,6) and (12,6) at 262144 shots each with 2D toric L=16 and 32 in
    one plan (min-sum, 64 rounds for BB, 4L for toric)."""
    _plan_sampled(L, orc, [("bb:6x6", 0.005, 0.05, 64, 262144),
                           ("bb:12x6", 0.008, 0.05, 64, 262144),
                           ("toric2d:16", 0.05, 0.05, 64, 16384),
                           ("toric2d:32", 0.05, 0.05, 128, 16384)], nsample=6)


@pytest.mark.timeout(600)
def test_server_serving_mix_equals_alone_and_oracle(L, orc):
    """The serving workload's code mix (2D toric L=16/32/48, 3D toric point
    sector L=12, BB (12,6); p = 0.03; 8L rounds, 96 for the 3D and BB codes):
    requests interleaved in arrival order give each shot exactly the result
    of its own decode alone, and a sample matches the oracle."""
    import torch
    mix = []
    for name, R in (("toric2d:16", 128), ("toric2d:32", 256), ("toric2d:48", 384),
                    ("toric3d_point:12", 96), ("bb:12x6", 96)):
        spec = codes.by_name(name)
        code = L.Code(spec, 0)
        P = L.DecodeParams(rounds=R)
        e0 = L.sample_noise(code, 0.03, 0, 100, 24)
        mix.append({"spec": spec, "code": code, "params": P, "e0": e0, "shot0": 100})
    alone = []
    for it in mix:
        r = L.decode_rounds(it["code"], it["params"], it["e0"], shot0=it["shot0"])
        r["fail"] = L.logical_failure(it["code"], it["e0"], r["z"])
        alone.append({k: v.cpu().numpy() for k, v in r.items() if k != "workspace" and v is not None})
    torch.cuda.synchronize()
    order = [(i % 5, i // 5) for i in range(5 * 24)]
    print(f"[serve] serving mix, {len(order)} requests", flush=True)
    res, srv = _serve(L, mix, order)
    assert len(res) == len(order)
    for (i, k), r in res.items():
        assert np.array_equal(r["z"], alone[i]["z"][k]), (mix[i]["spec"].name, k)
        assert np.array_equal(r["s"], alone[i]["s"][k]), (mix[i]["spec"].name, k)
        assert r["tclr"] == alone[i]["tclr"][k] and r["fail"] == alone[i]["fail"][k], (mix[i]["spec"].name, k)
    for i, it in enumerate(mix):
        e0 = it["e0"][:2].cpu().numpy()
        o = orc.decode(it["spec"], orc.DecodeParams(rounds=it["params"].rounds), e0, shot0=it["shot0"], nthreads=2)
        assert np.array_equal(alone[i]["z"][:2], o["z"]), it["spec"].name
        assert np.array_equal(alone[i]["tclr"][:2], o["tclr"]), it["spec"].name
    st = srv.stats()
    assert st["resident"] == 0 and st["waiting"] == 0


def test_batch_plan_clamp_binding_items(L, orc):
    """Min-sum items whose qubit-side clamp can bind (alpha = 1, or a small
    CLAMP) run in the padded kernel variant, beside items of the same code
    that run the exact variant; all match their single launches and the
    oracle."""
    import torch
    spec = codes.by_name("toric2d:8")
    code = L.Code(spec, 0)
    e0 = L.sample_noise(code, 0.06, 2, 0, 200)
    items = [{"spec": spec, "code": code, "params": L.DecodeParams(rounds=24, **kw), "e0": e0, "shot0": 0}
             for kw in ({}, {"alpha": 1.0}, {"clamp": 4.0}, {"clamp": 4.0, "bp": "sumproduct"})]
    plan = L.BatchPlan(items)
    outs = plan.launch()
    torch.cuda.synchronize()
    e0n = e0.cpu().numpy()
    for it, o in zip(items, outs):
        ref = L.decode_rounds(code, it["params"], e0)
        for k in ("z", "s", "tclr"):
            assert torch.equal(o[k], ref[k]), (it["params"], k)
        P = it["params"]
        od = orc.decode(spec, orc.DecodeParams(bp=P.bp, alpha=P.alpha, clamp=P.clamp, rounds=P.rounds),
                        e0n[:40], nthreads=8)
        assert np.array_equal(o["z"][:40].cpu().numpy(), od["z"]), P
        assert np.array_equal(o["tclr"][:40].cpu().numpy(), od["tclr"]), P


def test_batch_plan_with_empty_and_single_items(L, orc):
    """Items with no shots and with one shot, in both the persistent kernel
    and the stream form (membrane L=16 does not fit the LDS), next to a
    normal item."""
    import torch
    specs = [codes.by_name("toric2d:8"), codes.by_name("toric3d_membrane:16")]
    cds = [L.Code(s, 0) for s in specs]
    items = []
    for spec, code, S in ((specs[0], cds[0], 0), (specs[1], cds[1], 0), (specs[0], cds[0], 1),
                          (specs[1], cds[1], 1), (specs[0], cds[0], 77)):
        q = 0.125 if "membrane" in spec.name else 0.05
        e0 = L.sample_noise(code, 0.03, 5, 11, S) if S else torch.zeros((0, code.n), dtype=torch.uint8,
                                                                           device="cuda")
        items.append({"spec": spec, "code": code, "params": L.DecodeParams(q=q, rounds=8), "e0": e0, "shot0": 11})
    plan = L.BatchPlan(items)
    outs = plan.launch()
    torch.cuda.synchronize()
    for it, o in zip(items, outs):
        S = it["e0"].shape[0]
        assert o["z"].shape[0] == S
        if S == 0:
            continue
        P = it["params"]
        od = orc.decode(it["spec"], orc.DecodeParams(q=P.q, rounds=P.rounds), it["e0"][:1].cpu().numpy(),
                        shot0=11)
        assert np.array_equal(o["z"][:1].cpu().numpy(), od["z"]), it["spec"].name
        assert int(o["tclr"][0]) == int(od["tclr"][0]), it["spec"].name


def test_batch_plan_and_server_skip_equals_every_sweep(L):
    """The exact shortcuts (skip_fixed, the default) inside the batched plan
    and the server: the same items with every sweep computed give the same
    z, s, t_clr and failures; in the server, requests that freeze finish
    early with the result of all their rounds."""
    import dataclasses

    import torch
    mix_on = _mix(L)
    mix_off = [dict(it, params=dataclasses.replace(it["params"], skip_fixed=False)) for it in mix_on]
    outs_on = L.BatchPlan(mix_on).launch()
    outs_off = L.BatchPlan(mix_off).launch()
    torch.cuda.synchronize()
    for it, a, b in zip(mix_on, outs_on, outs_off):
        for k in ("z", "s", "tclr", "fail"):
            assert torch.equal(a[k], b[k]), (it["spec"].name, k)
    order = [(i, k) for i, it in enumerate(mix_on) for k in range(0, it["e0"].shape[0], 13)]
    ra, _ = _serve(L, mix_on, order)
    rb, _ = _serve(L, mix_off, order)
    assert ra.keys() == rb.keys()
    for key in ra:
        for k in ("z", "s", "tclr", "fail"):
            assert np.array_equal(np.asarray(ra[key][k]), np.asarray(rb[key][k])), (key, k)


def test_server_samples_the_error_on_the_device_when_e0_is_null(L):
    """laim_server_submit with e0_host NULL draws the request's error on the
    device from (params.seed, shot id, p), as laim_sample_noise does: the
    results equal those of the same request with that error given, and of a
    plain decode of it."""
    import torch
    for name, p, bp, R in (("toric2d:16", 0.05, "minsum", 64), ("bb:12x6", 0.01, "sumproduct", 64),
                           ("toric3d_point:6", 0.03, "minsum", 24)):
        spec = codes.by_name(name)
        code = L.Code(spec, 0)
        P = L.DecodeParams(bp=bp, rounds=R, seed=9)
        shots = [0, 1, 5, 2**33 + 17, 123456]
        e0 = torch.stack([L.sample_noise(code, p, 9, s, 1)[0] for s in shots])
        torch.cuda.synchronize()
        ref = [L.decode_rounds(code, P, e0[i:i + 1], shot0=s) for i, s in enumerate(shots)]
        srv = L.Server(0, 1 << 26, 64)
        tickets = {}
        for i, s in enumerate(shots):
            tickets[srv.submit(code, P, s, None, p)] = ("null", i)
            tickets[srv.submit(code, P, s, e0[i].cpu().numpy())] = ("given", i)
        res = {}
        while len(res) < len(tickets):
            evs = srv.step()
            assert evs, "a step with resident requests reported nothing"
            for ev in evs:
                if ev["done"]:
                    r = srv.result(ev["ticket"])
                    r["fail"] = ev["fail"]
                    res[tickets[ev["ticket"]]] = r
        for i, s in enumerate(shots):
            a, b = res[("null", i)], res[("given", i)]
            assert np.array_equal(a["z"], b["z"]) and np.array_equal(a["s"], b["s"]), (name, s)
            assert a["tclr"] == b["tclr"] and a["fail"] == b["fail"], (name, s)
            assert np.array_equal(a["z"], ref[i]["z"][0].cpu().numpy()), (name, s)
            assert a["tclr"] == int(ref[i]["tclr"][0]), (name, s)


def test_server_rejects_a_request_larger_than_its_budget(L):
    """A request whose state exceeds the server's whole budget could never be
    admitted: submit refuses it with LAIM_ENOMEM instead of queueing it in
    front of the others, and smaller requests still run."""
    small = L.Code(codes.by_name("toric2d:4"), 0)
    big = L.Code(codes.by_name("toric2d:48"), 0)
    srv = L.Server(0, 16 * 1024, 8)
    P = L.DecodeParams(rounds=8)
    with pytest.raises(L.LaimError) as ei:
        srv.submit(big, P, 0, None, 0.05)
    assert ei.value.status == L.ENOMEM
    t = srv.submit(small, P, 3, None, 0.1)
    done = False
    for _ in range(20):
        for ev in srv.step():
            assert ev["ticket"] == t
            if ev["done"]:
                srv.result(t)
                done = True
        if done:
            break
    assert done
    st = srv.stats()
    assert st["resident"] == 0 and st["waiting"] == 0 and st["bytes"] == 0


def test_server_request_with_no_rounds_finishes_at_its_first_step(L, orc):
    """rounds = 0: no round runs; the first step reports the start state
    (t_clr 0 for a clear syndrome, else -1 and a failure) with round 0, and
    the result is z = 0, s = H e0 -- as laim_decode_rounds gives it."""
    spec = codes.by_name("toric2d:8")
    code = L.Code(spec, 0)
    P = L.DecodeParams(rounds=0)
    srv = L.Server(0, 1 << 24, 16)
    e_clear = np.zeros(code.n, dtype=np.uint8)
    e_one = np.zeros(code.n, dtype=np.uint8)
    e_one[5] = 1
    ta = srv.submit(code, P, 0, e_clear)
    tb = srv.submit(code, P, 1, e_one)
    tc = srv.submit(code, L.DecodeParams(rounds=4), 2, e_one)
    evs = {ev["ticket"]: ev for ev in srv.step()}
    assert evs[ta]["done"] and evs[ta]["round"] == 0 and evs[ta]["tclr"] == 0 and evs[ta]["fail"] == 0
    assert evs[tb]["done"] and evs[tb]["round"] == 0 and evs[tb]["tclr"] == -1 and evs[tb]["fail"] == 1
    assert evs[tb]["flips"] == 0 and evs[tb]["defects"] == 2
    assert evs[tc]["round"] == 1
    rb = srv.result(tb)
    assert rb["z"].sum() == 0 and np.array_equal(rb["s"], orc.syndrome(spec, e_one)[0])
    srv.result(ta)


def test_server_step_advances_at_most_max_events(L):
    """With fewer event slots than resident requests, a step advances only
    that many (the oldest first); every request still reports each of its
    rounds and its done event, and results equal the plain decode."""
    import torch
    spec = codes.by_name("toric2d:8")
    code = L.Code(spec, 0)
    P = L.DecodeParams(rounds=16)
    e0 = L.sample_noise(code, 0.06, 0, 0, 10)
    ref = L.decode_rounds(code, P, e0)
    torch.cuda.synchronize()
    srv = L.Server(0, 1 << 24, 32)
    tk = {srv.submit(code, P, i, e0[i].cpu().numpy()): i for i in range(10)}
    seen = {}
    res = {}
    while len(res) < 10:
        evs = srv.step(max_events=3)
        assert 1 <= len(evs) <= 3
        for ev in evs:
            assert ev["round"] == seen.get(ev["ticket"], 0) + 1
            seen[ev["ticket"]] = ev["round"]
            if ev["done"]:
                res[tk[ev["ticket"]]] = srv.result(ev["ticket"])
    for i in range(10):
        assert np.array_equal(res[i]["z"], ref["z"][i].cpu().numpy()), i
        assert res[i]["tclr"] == int(ref["tclr"][i]), i
    assert srv.stats()["bytes"] == 0
