"""The persistent batched run's work-queue protocol, modelled on the CPU: items
(step, phase, instance, tile) taken in order from one counter by a fixed
number of workgroups, each item waiting until its instance has finished every
item of the earlier phases and steps (the per-instance counter reaching
`need`).  Under random interleavings, with fewer workgroups than items in a
phase and with a single workgroup, every run drains, no item starts before
its predecessors have finished, and the counters end at steps x items per
instance.  With the counter updates made invisible (a wait that can never be
satisfied) the bounded waits end every workgroup.  CPU only: a model of the
decode and wait arithmetic of batch_persistent_kernel, not a run of it."""
import numpy as np
import pytest


def decode(g, per_step, phase_items, offsets):
    k, r = divmod(g, per_step)
    ph = 0
    while r >= phase_items[ph]:
        r -= phase_items[ph]
        ph += 1
    off = offsets[ph]
    pos = int(np.searchsorted(off, r, side="right") - 1)
    return k, ph, pos, r - off[pos]


def need(k, ph, items):
    return k * sum(items) + sum(items[:ph])


def run(items_per_instance, steps, workgroups, seed, spin_limit=None, visible=True):
    """items_per_instance: [count][4] item counts per phase (queue order).
    Returns (finished items, aborted)."""
    rng = np.random.default_rng(seed)
    count = len(items_per_instance)
    phase_items = [sum(it[p] for it in items_per_instance) for p in range(4)]
    offsets = [np.concatenate([[0], np.cumsum([it[p] for it in items_per_instance])])
               for p in range(4)]
    per_step = sum(phase_items)
    total = per_step * steps
    done = [0] * count
    finished = set()
    nxt = 0
    abort = False
    # workgroup state: None (free) or [item, pos, need, remaining work, spins, started]
    wg = [None] * workgroups
    live = set(range(workgroups))
    while live:
        w = int(rng.choice(sorted(live)))
        st = wg[w]
        if st is None:
            if abort or nxt >= total:
                live.discard(w)
                continue
            g = nxt
            nxt += 1
            k, ph, pos, tile = decode(g, per_step, phase_items, offsets)
            assert 0 <= pos < count and 0 <= tile < items_per_instance[pos][ph]
            wg[w] = [g, pos, need(k, ph, items_per_instance[pos]), int(rng.integers(1, 4)), 0, False]
            continue
        g, pos, nd, rem, spins, started = st
        if not started:
            seen = done[pos] if visible else 0
            if seen >= nd:
                # every earlier item of this instance has finished
                k, ph, _, _ = decode(g, per_step, phase_items, offsets)
                for h in range(g):
                    k2, ph2, pos2, _ = decode(h, per_step, phase_items, offsets)
                    if pos2 == pos and (k2, ph2) < (k, ph):
                        assert h in finished, (g, h)
                st[5] = True
            else:
                st[4] = spins + 1
                if spin_limit is not None and st[4] > spin_limit:
                    abort = True
                    wg[w] = None
                    live.discard(w)
                elif abort and st[4] % 4 == 0:
                    wg[w] = None
                    live.discard(w)
            continue
        st[3] = rem - 1
        if st[3] == 0:
            done[pos] += 1
            finished.add(g)
            wg[w] = None
    return finished, abort, done, total


SIZES = [[64, 36, 1, 136], [16, 10, 1, 36], [4, 3, 1, 10], [1, 1, 1, 3], [9, 6, 1, 15]]


@pytest.mark.parametrize("workgroups", [1, 3, 17])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_queue_drains_in_dependency_order(workgroups, seed):
    finished, aborted, done, total = run(SIZES, steps=3, workgroups=workgroups, seed=seed)
    assert not aborted and len(finished) == total
    assert done == [3 * sum(it) for it in SIZES]


def test_bounded_wait_ends_every_workgroup():
    """Counter updates never seen: the first wait past the bound sets the
    abort flag and every workgroup leaves (nothing hangs)."""
    finished, aborted, done, total = run(SIZES, steps=2, workgroups=8, seed=3, spin_limit=50,
                                         visible=False)
    assert aborted and len(finished) < total
