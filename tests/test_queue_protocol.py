"""The work-queue schedule of the block solves, modelled on the CPU.

Workers take (cycle, domain) tasks from a shared counter in the order the
GPU kernel uses (per cycle: black domains, then white), wait until every
neighbouring domain's epoch reaches the value the task depends on, "solve"
(a random delay) and publish their epoch.  Checked: the queue drains for any
number of workers (no deadlock), and every visit of a domain sees its
neighbours exactly at the visit the sequential half-sweep order gives, i.e.
the schedule is the multiplicative Schwarz order of the half-sweep launches.
"""
import random
import threading
import time

import pytest


def domain_grid(n):
    nd = n[0] * n[1] * n[2] * n[3]
    coords = []
    for d in range(nd):
        r, X = d, []
        for m in range(4):
            X.append(r % n[m])
            r //= n[m]
        coords.append(X)
    colour = [sum(X) % 2 for X in coords]

    def neighbours(d):
        out = []
        for mu in range(4):
            for step in (-1, 1):
                E = list(coords[d])
                E[mu] = (E[mu] + step) % n[mu]
                out.append(E[0] + n[0] * (E[1] + n[1] * (E[2] + n[2] * E[3])))
        return out

    order = [d for d in range(nd) if colour[d] == 0] + [d for d in range(nd) if colour[d] == 1]
    return nd, colour, neighbours, order


def run_queue(n, n_cycles, n_workers, seed, base=0):
    nd, colour, neighbours, order = domain_grid(n)
    nblack = sum(1 for c in colour if c == 0)
    ntask = n_cycles * nd
    lock = threading.Lock()
    counter = [0]
    epoch = [base] * nd
    seen = {}
    rng = random.Random(seed)
    delays = [rng.random() * 1e-4 for _ in range(ntask)]

    def worker():
        while True:
            with lock:
                t = counter[0]
                counter[0] += 1
            if t >= ntask:
                return
            s, k = divmod(t, nd)
            d = order[k]
            c = int(k >= nblack)
            need = base + s + c
            deadline = time.time() + 20
            for nb in neighbours(d):
                while epoch[nb] < need:
                    if time.time() > deadline:
                        raise RuntimeError("queue stalled")
                    time.sleep(1e-5)
            # what the visit sees: the neighbours' completed visits
            seen[(d, s)] = tuple(epoch[nb] - base for nb in neighbours(d))
            time.sleep(delays[t])
            assert epoch[d] == base + s, "a domain's visits complete in order"
            epoch[d] = base + s + 1

    threads = [threading.Thread(target=worker) for _ in range(n_workers)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert all(not th.is_alive() for th in threads)
    assert epoch == [base + n_cycles] * nd
    return seen, colour, neighbours


@pytest.mark.parametrize("n,n_cycles,workers", [((2, 2, 2, 2), 8, 128), ((2, 2, 2, 2), 8, 3),
                                                 ((2, 4, 4, 8), 4, 64), ((4, 2, 2, 2), 5, 1)])
def test_queue_drains_in_schwarz_order(n, n_cycles, workers):
    seen, colour, neighbours = run_queue(n, n_cycles, workers, seed=sum(n) + workers, base=7)
    for (d, s), eps in seen.items():
        # black at cycle s sees its white neighbours after s visits (cycles 0..s-1);
        # white at cycle s sees its black neighbours after s+1 visits (cycles 0..s).
        # A neighbour can be ahead by at most its next visit only if it does not
        # depend on d: impossible, since every neighbour's next visit waits for d.
        want = s + colour[d]
        assert all(e == want for e in eps), (d, s, eps, want)
