"""GPU tests of the serving engine (mcs_server_*): results against the FP64
oracle, the same result for a request alone and in a mix, admission under
the arena budget (oversized requests fail, the budget is never exceeded),
and overlap of micro-batches on the device."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (dim, n, k, viscosity seed, force seed)
REQ = [(3, 2, 2, 31, 41), (3, 3, 3, 32, 42), (2, 4, 2, 33, 43), (3, 2, 4, 34, 44), (2, 3, 5, 35, 45)]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_cache = {}


def request(i):
    if i in _cache:
        return _cache[i]
    d, n, k, s_nu, s_f = REQ[i]
    mesh = W.unit_square_mesh(n) if d == 2 else W.unit_cube_mesh(n)
    nu = W.lognormal_nu(mesh.n_elements, seed=s_nu, contrast=10.0)
    f = W.RandomForce(d, seed=s_f).f(W.lattice_points(mesh, k + 1))
    _cache[i] = dict(mesh=mesh, nu=nu, f=f, k=k)
    return _cache[i]


def n_dof(c):
    from paper_2207_08481_amd import Problem
    return Problem(c["mesh"].vertices, c["mesh"].elements, c["mesh"].lattice, c["k"]).n_dof


def submit(srv, i):
    c = request(i)
    return srv.submit(c["mesh"].vertices, c["mesh"].elements, c["mesh"].lattice, c["k"], c["nu"], c["f"])


def make_server(arena_gb=2.0, **kw):
    _need_gpu()
    from paper_2207_08481_amd import Server
    print(f"[server] arena {arena_gb} GB {kw}", flush=True)
    return Server(int(arena_gb * (1 << 30)), **kw)


def test_server_results_match_oracle():
    from oracle.system import GlobalSystem
    from tests.test_gpu_batch import _l2_rel
    srv = make_server(tol=1e-10)
    ids = [submit(srv, i) for i in range(len(REQ))]
    for i, rid in enumerate(ids):
        c = request(i)
        x, info = srv.wait(rid, n_dof(c))
        assert info["status"] == 0, info
        gs = GlobalSystem(c["mesh"].vertices, c["mesh"].elements, c["nu"], c["k"], c["f"])
        eu, ep = _l2_rel(gs, x, gs.direct_solve())
        assert eu < 1e-8 and ep < 1e-8, (i, eu, ep, info)
    srv.close()


def test_request_same_alone_and_in_mix():
    srv = make_server(max_inflight=1)
    c = request(1)
    nd = n_dof(c)
    x_alone, i_alone = srv.wait(submit(srv, 1), nd)
    assert i_alone["status"] == 0 and i_alone["batch_size"] == 1
    # a burst: the request among others, at another position of the queue
    ids = [submit(srv, j) for j in (0, 2, 1, 3, 4)]
    xs = {}
    for j, rid in zip((0, 2, 1, 3, 4), ids):
        xs[j] = srv.wait(rid, n_dof(request(j)))
    x_mix, i_mix = xs[1]
    assert i_mix["status"] == 0
    assert i_mix["batch_size"] > 1, i_mix
    assert i_mix["iterations"] == i_alone["iterations"]
    assert np.array_equal(x_mix, x_alone)
    srv.close()


def test_admission_under_budget():
    """An arena that holds only part of the burst: every request completes,
    the arena is never oversubscribed, several micro-batches are formed, and
    a request larger than the whole arena fails with MCS_ERR_WORKSPACE."""
    from paper_2207_08481_amd import Batch
    c3 = request(3)
    b = Batch([(c3["mesh"].vertices, c3["mesh"].elements, c3["mesh"].lattice)], [c3["k"]], precision=1)
    one = b.info.workspace_bytes
    srv = make_server(arena_gb=2.5 * one / (1 << 30), max_inflight=2)
    ids = [(j, submit(srv, j)) for j in (3, 3, 3, 0, 2)]
    big = W.unit_cube_mesh(8)
    fbig = W.RandomForce(3, seed=9).f(W.lattice_points(big, 6))
    rid_big = srv.submit(big.vertices, big.elements, big.lattice, 5, np.ones(big.n_elements), fbig)
    for j, rid in ids:
        x, info = srv.wait(rid, n_dof(request(j)))
        assert info["status"] == 0, (j, info)
    _, info = srv.wait(rid_big, 1)
    assert info["status"] == -3, info
    st = srv.stats()
    assert st["arena_peak"] <= st["arena_bytes"]
    assert st["batches"] >= 2, st
    srv.close()


def test_micro_batches_overlap():
    """With two slots, requests submitted while a larger micro-batch runs are
    admitted into the second slot before it finishes."""
    srv = make_server(max_inflight=2, arena_gb=8.0)
    big = W.unit_cube_mesh(6)
    fbig = W.RandomForce(3, seed=19).f(W.lattice_points(big, 5))
    rid_big = srv.submit(big.vertices, big.elements, big.lattice, 4, np.ones(big.n_elements), fbig)
    time.sleep(0.05)
    ids = [(j, submit(srv, j)) for j in (1, 3)]
    seen = 0
    t_end = time.time() + 60
    while time.time() < t_end:
        st = srv.stats()
        seen = max(seen, st["inflight"])
        if st["solved"] >= 3:
            break
        time.sleep(0.002)
    for j, rid in ids:
        _, info = srv.wait(rid, n_dof(request(j)))
        assert info["status"] == 0, info
    from paper_2207_08481_amd import Problem
    nd_big = Problem(big.vertices, big.elements, big.lattice, 4).n_dof
    _, info = srv.wait(rid_big, nd_big)
    assert info["status"] == 0, info
    assert seen == 2, seen
    srv.close()
