"""tadmm_solve_noalloc (the solve on the library's static device workspace,
for callers that cannot allocate) against tadmm_solve on the same batch:
identical results, bit for bit, on two calls in a row, the second with a
smaller batch (the static array keeps the first call's contents), in the
plain and the batched mode.  Also its argument errors."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_15838_amd as tadmm  # noqa: E402

KEYS = ("x", "u", "w", "pair_active", "status", "iters", "r_norm", "s_norm", "eps_pri", "eps_dual")


def _prep(p, scs, **kw):
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p, **kw))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    return solver, prep, pk


def _host(prep):
    return {k: prep.o[k].cpu().numpy().copy() for k in KEYS}


def _same(a, b):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("mode", [tadmm.MODE_PLAIN, tadmm.MODE_BATCHED])
def test_noalloc_equals_solve_on_two_calls(mode):
    p, big = synth.config2(S=12)
    _, small = synth.config2(S=5, scenario_ids=range(40, 45))
    solver, prep_big, _ = _prep(p, big, max_iter=60)
    pk = synth.pack(p, small)   # the same context serves both batches
    prep_small = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    for prep, name in ((prep_big, "first call, 12 scenarios"), (prep_small, "second call, 5 scenarios")):
        print(f"noalloc mode={mode}: {name}", flush=True)
        prep.run(mode)
        ref = _host(prep)
        for t in prep.o.values():
            if t is not None:
                t.zero_()
        prep.run_noalloc(mode)
        got = _host(prep)
        _same(ref, got)
        assert got["iters"].min() >= 1
    solver.close()


def test_noalloc_rejects_what_it_cannot_do():
    p, scs = synth.config2(S=2)
    solver, prep, pk = _prep(p, scs)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.run_noalloc(tadmm.MODE_WIDE)
    assert e.value.code == 1
    # a batch whose workspace exceeds the static array
    nb = solver.workspace_bytes(np.full(4096, 32), np.full(4096, 40))
    assert nb > 64 << 20
    N = np.full(4096, 32, dtype=np.int32)
    T = np.full(4096, 40, dtype=np.int32)
    b = tadmm.Batch(4096, N.ctypes.data_as(tadmm._ip), T.ctypes.data_as(tadmm._ip), *([None] * 11))
    import ctypes as C
    rc = tadmm.lib().tadmm_solve_noalloc(solver._h, C.byref(b), C.byref(prep.out), tadmm.MODE_BATCHED)
    assert rc == 6 and b"static workspace" in tadmm.lib().tadmm_last_error(solver._h)
    solver.close()
