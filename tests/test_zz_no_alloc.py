"""GPU: jx_rollout_noalloc (work-queue counters in the library's static device
array, no allocation) against jx_rollout with the same flags, through the C-ABI.

Two calls in a row, the second on a smaller batch, so the second call starts
from the counts the first one left in the shared array.  Outputs (frames,
rewards, dones) and the final state must be identical byte for byte."""
import numpy as np
import pytest

import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

PERSIST = dict(form=1, waves_per_group=2, groups_per_cu=4, store_mode=0)


def _pair_outputs(cfgs, seeds, idx, T, launch, fused):
    """The same batch run by jx_rollout and by jx_rollout_noalloc from the same
    reset state; returns both (obs, reward, done, state image) tuples."""
    import torch
    n_act = max(c["n_actions"] for c in cfgs)
    acts = torch.from_numpy(W.actions(21, T, len(seeds), n_act)).to("cuda")
    outs = []
    for noalloc in (False, True):
        env = U.env_of(cfgs, seeds, idx, obs=False)
        env.set_launch(**launch)
        n, ob = env.n, env.obs_bytes
        obs = torch.zeros(T * ob, dtype=torch.uint8, device=env.dev)
        rew = torch.zeros(T * n, dtype=torch.float32, device=env.dev)
        done = torch.zeros(T * n, dtype=torch.uint8, device=env.dev)
        prev = torch.zeros(T * n, dtype=torch.uint8, device=env.dev)
        if noalloc:
            env.rollout_noalloc(acts, obs, rew, done, T, obs_stride=ob, fused=fused, prev=prev)
        else:
            env.rollout(acts, obs, rew, done, T, obs_stride=ob, graph=False, fused=fused, prev=prev)
        torch.cuda.synchronize()
        outs.append((obs.cpu().numpy(), rew.cpu().numpy(), done.cpu().numpy(), prev.cpu().numpy(),
                     env.get_state_bytes()))
        env.close()
    return outs


def _assert_same(a, b, what):
    for k, name in enumerate(("obs", "reward", "done", "prev", "state")):
        assert np.array_equal(a[k], b[k]), f"{what}: {name} differs"


@pytest.mark.parametrize("fused", [False, True])
def test_noalloc_equals_rollout_two_calls_second_smaller(fused):
    # first call: 3000 mixed-shape envs (sides 8..64, frames 32..128, key-door
    # on half), persistent mapping, 12 steps
    cfgs, idx = W.batch_cfgs(3000)
    ref, got = _pair_outputs(cfgs, W.seeds(W.BATCH["number"], 3000), idx, 12, PERSIST, fused)
    _assert_same(ref, got, "first call (3000 envs)")
    # second call, smaller: 300 envs of the headline configuration, 7 steps,
    # another persistent mapping
    cfg = W.SCALE["cfg"]
    ref, got = _pair_outputs([cfg], W.seeds(W.SCALE["number"], 300), None, 7,
                             dict(form=1, waves_per_group=4, groups_per_cu=2, store_mode=1), fused)
    _assert_same(ref, got, "second call (300 envs)")


def test_noalloc_plain_and_pipelined_mappings_and_flags():
    from paper_2605_19926_amd import jx
    cfgs, idx = W.batch_cfgs(512, number=31)
    seeds = W.seeds(31, 512)
    for launch in (dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0),
                   dict(form=2, waves_per_group=2, groups_per_cu=2, store_mode=0)):
        ref, got = _pair_outputs(cfgs, seeds, idx, 5, launch, False)
        _assert_same(ref, got, f"mapping {launch}")
    import torch
    env = U.env_of([W.SCALE["cfg"]], W.seeds(2, 8), None, obs=False)
    buf = torch.zeros(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    a = torch.zeros(8, dtype=torch.uint8, device=env.dev)
    r = torch.zeros(8, dtype=torch.float32, device=env.dev)
    d = torch.zeros(8, dtype=torch.uint8, device=env.dev)
    with pytest.raises(jx.JxError) as e:
        env.rollout_noalloc(a, buf, r, d, 1, flags=jx.JX_ROLLOUT_GRAPH)
    assert e.value.code == jx.JX_EINVAL and "allocates" in str(e.value)
    with pytest.raises(jx.JxError) as e:
        env.rollout_noalloc(a, buf, r, d, 1, flags=8)
    assert e.value.code == jx.JX_EINVAL
    env.rollout_noalloc(a, buf, r, d, 0)  # no work: returns at once
    env.close()
