"""Checkpoint and resume of md_step: a run of n steps equals k steps then
n - k steps bit for bit (eager and graph replay), with k inside an exchange
interval (where consecutive steps share the fused closing / opening kernel)
and k on an exchange step; and the state saved to the host after k steps
(positions, velocities, charges, site states, exchange targets, grid map,
step index) continues bit for bit in a fresh context.  The counter-based
random numbers depend on the step index alone, so nothing else is needed."""
import numpy as np
import pytest
import torch

from common import with_oracle_gref
from paper_1809_07726_amd import synth

pytestmark = pytest.mark.gpu

N_STEPS = 30
KEYS = ("xyz", "v", "q", "site_state", "target_idx", "grid_rep")


def _batch():
    b = with_oracle_gref(synth.make_config(2, n_atoms=300, n_rep=8, per_replica_jitter=True))
    b["mc_every"], b["ex_every"] = 5, 10       # attempts after steps 5, 10, ...; exchanges after 10, 20, 30
    return b


def _state(md, d):
    out = {k: d.t[k].cpu().numpy().copy() for k in KEYS}
    out["force_fx"] = md.force_fx.cpu().numpy().copy()
    out["energy_fx"] = md.energy_fx.cpu().numpy().copy()
    return out


def _run(b, chunks, graph):
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=2002)
    for i, n in enumerate(chunks):
        md.run(n, init_forces=i == 0, graph=graph)
    torch.cuda.synchronize()
    ctx.check()
    st = _state(md, d)
    ctx.close()
    return st


def _assert_same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("graph", [False, True])
def test_split_runs_equal_one_run_bitwise(graph):
    b = _batch()
    print(f"case: 8 x 300 atoms, {N_STEPS} steps, graph={graph}", flush=True)
    ref = _run(b, [N_STEPS], graph)
    for k in (13, 20):                      # inside an exchange interval; right after an exchange step
        _assert_same(ref, _run(b, [k, N_STEPS - k], graph), f"split at {k}")
    _assert_same(ref, _run(b, [7, 6, 7, 10], graph), "four calls")
    assert not np.array_equal(ref["target_idx"], b["target_idx"].reshape(-1))   # exchanges happened


def test_state_saved_to_host_continues_bitwise_in_a_fresh_context():
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    b = _batch()
    ref = _run(b, [N_STEPS], False)
    for k in (13, 20):
        print(f"case: checkpoint after {k} steps", flush=True)
        ctx = Context(b["atom_off"])
        d = DeviceBatch.from_numpy(b)
        md = MD(ctx, d, b, seed=2002)
        md.run(k, init_forces=True)
        torch.cuda.synchronize()
        saved = {kk: d.t[kk].cpu().numpy().copy() for kk in KEYS}
        step = md.step
        ctx.close()
        # a fresh context and fresh device arrays from the saved host state
        b2 = dict(b)
        N = int(b["atom_off"][-1])
        b2["xyz"] = saved["xyz"].reshape(3, N).T.copy()
        b2["v"] = saved["v"].reshape(3, N).T.copy()
        b2["q"] = saved["q"]
        b2["site_state"] = saved["site_state"]
        b2["target_idx"] = saved["target_idx"].reshape(-1, 4)
        b2["grid_rep"] = saved["grid_rep"]
        ctx = Context(b2["atom_off"])
        d = DeviceBatch.from_numpy(b2)
        md = MD(ctx, d, b2, seed=2002)
        md.step = step
        md.run(N_STEPS - k, init_forces=True)
        torch.cuda.synchronize()
        ctx.check()
        _assert_same(ref, _state(md, d), f"restored after {k}")
        ctx.close()
