"""Serving runtime (continuous batching with footprint admission) on the GPU.

Checks: the exact footprint of a call is what the call lays out (a budget one
byte smaller is refused); each request's result is bitwise the same alone and
in a concurrent mix; admission keeps the pool within its size and refuses a
request larger than the pool; a served request matches the oracle at the
mixed-precision bound.
"""
import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE
from workloads import configs as C
from tests.gpu_common import method_params, oracle_params

pytestmark = pytest.mark.gpu


def _req(st, cut):
    return dict(pos=st.pos, species=st.species, v_ratio=st.nu, cell=st.cell,
                pbc=tuple(int(x) for x in st.pbc), cutoffs=cut)


def _requests(n=12, seed=700):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        size = int(round(np.exp(rng.uniform(np.log(40), np.log(400)))))
        rc = float(rng.uniform(4.0, 5.0))
        if i % 2 == 0:
            st = C.hcno_cluster(size, seed + i)
        else:
            st = C.hcno_box(size, seed + i)
        out.append(_req(st, C.cutoffs(rc)))
    return out


def test_footprint_is_exact():
    from paper_2407_06409_amd import Context, LmbdError, compute_batch, estimate_footprint
    st, cut = C.carbon_box(96, 21), C.cutoffs(4.5)
    r = _req(st, cut)
    mp = method_params(precision="mixed")
    need = estimate_footprint([r], mp, forces=True)
    print(f"footprint of 96-atom box: {need} bytes", flush=True)
    ctx = Context(0, memory_budget=need)
    out = compute_batch([r], mp, SPECIES_TABLE, ctx=ctx)[0]
    assert np.all(np.isfinite(out["energies"]))
    ctx.set_memory_budget(need - 1)
    with pytest.raises(LmbdError) as ei:
        compute_batch([r], mp, SPECIES_TABLE, ctx=ctx)
    assert ei.value.code == "LMBD_E_OOM_ADMISSION"
    # a batch of two structures is one layout, not the sum of two
    r2 = _req(C.hcno_cluster(60, 3), C.cutoffs(5.0))
    need2 = estimate_footprint([r, r2], mp, forces=True)
    ctx.set_memory_budget(need2)
    outs = compute_batch([r, r2], mp, SPECIES_TABLE, ctx=ctx)
    assert np.array_equal(outs[0]["energies"], out["energies"])
    ctx.close()


def _serve(reqs, mp, **kw):
    from paper_2407_06409_amd import Server
    with Server(mp, SPECIES_TABLE, **kw) as srv:
        if kw.get("max_batch_requests") == 1 and kw.get("n_slots", 2) == 1:
            res = []
            for r in reqs:
                t = srv.submit(r)
                res.append(srv.wait(t))
        else:
            tickets = [srv.submit(r) for r in reqs]
            res = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    return res, stats


def test_alone_and_in_the_mix_are_identical():
    reqs = _requests()
    mp = method_params(precision="mixed")
    print(f"{len(reqs)} requests, sizes {[len(r['pos']) for r in reqs]}", flush=True)
    alone, s1 = _serve(reqs, mp, n_slots=1, max_batch_requests=1, memory_budget=8 << 30)
    mix, s2 = _serve(reqs, mp, n_slots=3, memory_budget=8 << 30, max_batch_atoms=1500)
    print(f"alone: {s1}", flush=True)
    print(f"mix:   {s2}", flush=True)
    print("batch sizes in the mix:", sorted({(m['batch'], m['batch_requests']) for m in mix}), flush=True)
    for a, m in zip(alone, mix):
        assert a["status"] == "LMBD_OK" and m["status"] == "LMBD_OK", (a["detail"], m["detail"])
        assert np.array_equal(a["energies"], m["energies"])
        assert np.array_equal(a["forces"], m["forces"])
    assert s1["batches"] == len(reqs)
    assert s2["batches"] < len(reqs) or s2["max_concurrent"] > 1
    assert s2["pool_peak"] <= s2["pool_bytes"]
    # and the same as a direct call
    from paper_2407_06409_amd import compute_batch
    d = compute_batch([reqs[3]], mp, SPECIES_TABLE)[0]
    assert np.array_equal(d["energies"], alone[3]["energies"])


def test_admission_by_footprint():
    from paper_2407_06409_amd import LmbdError, Server, estimate_footprint
    reqs = _requests(6, seed=800)
    mp = method_params(precision="mixed")
    fps = [estimate_footprint([r], mp) for r in reqs]
    pool = int(max(fps) * 1.3) + (1 << 20)
    with Server(mp, SPECIES_TABLE, n_slots=3, memory_budget=pool) as srv:
        big = _req(C.carbon_box(1728, 5), C.cutoffs(6.0))
        with pytest.raises(LmbdError) as ei:
            srv.submit(big)
        assert ei.value.code == "LMBD_E_OOM_ADMISSION"
        tickets = [srv.submit(r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    print(f"pool {pool} bytes, footprints {fps}, stats {stats}", flush=True)
    assert all(r["status"] == "LMBD_OK" for r in res)
    assert stats["pool_peak"] <= stats["pool_bytes"]
    assert [r["footprint"] for r in res] == fps


def test_served_request_against_oracle():
    st, cut = C.hcno_cluster(70, 31), C.cutoffs(4.5)
    mp = method_params(precision="mixed")
    res, _ = _serve([_req(st, cut)], mp, n_slots=2, memory_budget=1 << 30)
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut), SPECIES_TABLE)
    de = np.abs(res[0]["energies"] - e).max()
    df = np.abs(res[0]["forces"] - f).max()
    print(f"served vs oracle: max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A", flush=True)
    assert de < 1e-5 and df < 1e-4


def test_two_point_model_served_in_the_mix_equals_alone():
    """The two-point SCS frequency model through the continuous-batching server.
    On these H/C/N/O structures some strongly screened atoms have a polarisability
    that rises between 0 and omega_ref, which the model cannot represent: exactly
    the requests for which the oracle refuses the model fail with
    LMBD_E_SCS_BREAKDOWN, alone and in the mix; the others give bitwise the
    results of the request evaluated alone, and the oracle's model."""
    from workloads import Structure
    from workloads.configs import OMEGA_REF
    lor = dict(scs_freq="lorentz", omega_ref=OMEGA_REF)
    reqs = _requests(8, seed=900)
    refused = []
    for r in reqs:
        st = Structure(np.asarray(r["pos"]), np.asarray(r["species"]), np.asarray(r["v_ratio"]), r["cell"],
                       np.array(r["pbc"], bool))
        try:
            oracle.lmbd_energies(st, oracle_params(r["cutoffs"], **lor), SPECIES_TABLE)
            refused.append(False)
        except ValueError:
            refused.append(True)
    mp = method_params(precision="mixed", **lor)
    alone, _ = _serve(reqs, mp, n_slots=1, max_batch_requests=1, memory_budget=8 << 30)
    mix, s2 = _serve(reqs, mp, n_slots=3, memory_budget=8 << 30, max_batch_atoms=1500)
    print(f"two-point model served: {s2}; refused by the oracle: {refused}", flush=True)
    assert 0 < sum(refused) < len(reqs)
    for a, m, bad in zip(alone, mix, refused):
        want = "LMBD_E_SCS_BREAKDOWN" if bad else "LMBD_OK"
        assert a["status"] == want and m["status"] == want, (a["detail"], m["detail"])
        if not bad:
            assert np.array_equal(a["energies"], m["energies"])
            assert np.array_equal(a["forces"], m["forces"])
    st, cut = C.hcno_cluster(70, 31), C.cutoffs(4.5)
    res, _ = _serve([_req(st, cut)], mp, n_slots=2, memory_budget=1 << 30)
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut, **lor), SPECIES_TABLE)
    de, df = np.abs(res[0]["energies"] - e).max(), np.abs(res[0]["forces"] - f).max()
    print(f"  served two-point model vs oracle: max |dE| {de:.3e}, max |dF| {df:.3e}", flush=True)
    assert de < 1e-5 and df < 1e-4


def test_destroy_cancels_queued_requests():
    from paper_2407_06409_amd import Server
    reqs = _requests(8, seed=900)
    mp = method_params(precision="mixed")
    srv = Server(mp, SPECIES_TABLE, n_slots=1, max_batch_requests=1, memory_budget=1 << 30)
    tickets = [srv.submit(r) for r in reqs]
    srv.lib.lmbd_server_destroy(srv.handle)  # outputs of finished requests stay valid
    srv.handle = None
