"""CPU emulation of the dataflow launch's protocol (no GPU).

The plan groups independent instances; each group's tiles form a queue with a ticket counter that
hands out chunks of consecutive queue tiles in order. A workgroup starts at queue b mod Q, takes
chunks (drawing the next one while the current one runs), moves to the next queue when one runs
dry and leaves after finding every queue dry. Before a tile runs, its workgroup waits for the flags
of the tiles it depends on (flags carry the launch's generation); after the tile it publishes the
tile's own flag. The last workgroup to leave resets the counters and advances the generation.

The emulation interleaves the workgroups' steps at random, lets only a few of them be resident at
once (the others start when one leaves, as a GPU dispatches them), and runs several launches back
to back on the plan's real dependency lists and groups. It checks that every tile runs once per
launch, after every tile it depends on, that no wait exhausts its bound, and that the planner's
dependencies stay inside a group and point to smaller tiles; as controls, a dependency on a later
tile or across groups (which the planner never emits) can block with few resident workgroups.
"""
import numpy as np
import pytest

from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I


class Launches:
    """Shared device state (counters, gone count, generation, flags) and one launch at a time."""

    def __init__(self, dep_ptr, dep_list, tile_group, chunk):
        self.ptr, self.lst, self.K = dep_ptr, dep_list, chunk
        self.n = len(dep_ptr) - 1
        self.Q = int(tile_group.max()) + 1 if self.n else 1
        self.queues = [[t for t in range(self.n) if tile_group[t] == g] for g in range(self.Q)]
        self.ticket = [0] * self.Q
        self.gone = self.gen_word = 0
        self.flags = [0] * max(self.n, 1)
        self.error = False

    def launch(self, grid, resident, rng, spin_limit=10_000):
        done_at = {}
        waiting = list(range(grid))      # not yet dispatched, in order
        running = {}

        def draw(q):
            k = self.ticket[q]
            self.ticket[q] += 1
            return k

        def program(w):
            gen = self.gen_word + 1
            q, tried = w % self.Q, 1
            k = draw(q)
            yield
            while True:
                while k * self.K >= len(self.queues[q]) and tried < self.Q:
                    q, tried = (q + 1) % self.Q, tried + 1
                    k = draw(q)
                    yield
                if k * self.K >= len(self.queues[q]):
                    break
                nxt = draw(q)            # drawn while the chunk runs
                yield
                for t in self.queues[q][k * self.K:(k + 1) * self.K]:
                    for u in self.lst[self.ptr[t]:self.ptr[t + 1]]:
                        spins = 0
                        while self.flags[u] != gen:
                            spins += 1
                            if spins > spin_limit:
                                self.error = True  # the kernel would go on with stale values
                                return
                            yield
                    for u in self.lst[self.ptr[t]:self.ptr[t + 1]]:
                        assert u in done_at, f"tile {t} ran before its dependency {u}"
                    assert t not in done_at, f"tile {t} ran twice"
                    done_at[t] = len(done_at)
                    yield
                    self.flags[t] = gen
                    yield
                k = nxt
            gone = self.gone
            self.gone += 1
            if gone == grid - 1:
                self.ticket, self.gone, self.gen_word = [0] * self.Q, 0, gen

        while waiting or running:
            while waiting and len(running) < resident:
                w = waiting.pop(0)
                running[w] = program(w)
            w = rng.choice(list(running))
            try:
                next(running[w])
            except StopIteration:
                del running[w]
            if self.error:
                return done_at
        return done_at


def _plans():
    return {
        "cfg1": lambda: B.Plan(B.Problem.from_ilp(I.config(1))),
        "rand": lambda: B.Plan(B.Problem.from_ilp(I.random_ilp(80, 60, kmax=9, cmax=3, seed=3))),
        "batch": lambda: B.Plan([B.Problem.from_ilp(q) for q in
                                 (I.tomography(6, seed=0), I.tracking(250, seed=1), I.config(1),
                                  I.random_ilp(30, 20, seed=5), I.tomography(5, seed=8))]),
    }


@pytest.mark.parametrize("name", list(_plans()))
@pytest.mark.parametrize("chunk", [1, 2, 5])
def test_protocol_runs_every_tile_after_its_dependencies(name, chunk):
    plan = _plans()[name]()
    rng = np.random.default_rng(chunk)
    for pass_ in (0, 1):
        ptr, lst, grp = plan.tile_deps(pass_)
        n = len(ptr) - 1
        for t in range(n):
            for q in range(ptr[t], ptr[t + 1]):
                assert lst[q] < t and grp[lst[q]] == grp[t]
        if name == "batch":
            assert plan.stats.n_groups == 5 and set(grp.tolist()) == set(range(5))
        st = Launches(ptr, lst, grp, chunk)
        for k in range(4):
            # any grid and any number of resident workgroups, down to one
            grid = int(rng.integers(1, n + 2))
            resident = int(rng.integers(1, min(grid, 6) + 1))
            done = st.launch(grid, resident, rng)
            assert not st.error, (name, pass_, k, grid, resident)
            assert sorted(done) == list(range(n))
            assert st.gen_word == k + 1 and st.ticket == [0] * st.Q and st.gone == 0


def test_a_dependency_on_a_later_tile_can_block():
    """Control: tile 0 waiting for tile 5 with one resident workgroup never sees it done."""
    ptr = np.array([0, 1, 1, 1, 1, 1, 1])
    lst = np.array([5])
    st = Launches(ptr, lst, np.zeros(6, np.int32), 1)
    st.launch(grid=6, resident=1, rng=np.random.default_rng(0), spin_limit=200)
    assert st.error


def test_a_dependency_across_groups_can_block():
    """Control: tile 2 (group 1) waits for tile 1 (group 0), tile 0 waits for tile 2. Workgroup 0
    takes tile 0 from queue 0 and waits; workgroup 1 takes tile 2 from queue 1 and waits for tile
    1, which only queue 0's next draw would take: with those two resident, nothing moves."""
    ptr = np.array([0, 1, 1, 2, 2])
    lst = np.array([2, 1])
    st = Launches(ptr, lst, np.array([0, 0, 1, 1]), 1)
    st.launch(grid=2, resident=2, rng=np.random.default_rng(2), spin_limit=300)
    assert st.error


def _two_branch_run(ptr, lst, beg, mid, bw, rng):
    """Runs the two chains of the two-branch launch in a random interleaving: chain A takes the A
    parts in wave order without waiting, chain B takes part B of wave w once chain A has finished
    wave bw[w]. Returns the order in which tiles finished."""
    W = len(mid)
    done_at, a_done = {}, -1
    a_w = b_w = 0
    while a_w < W or b_w < W:
        can_a = a_w < W
        can_b = b_w < W and bw[b_w] <= a_done
        assert can_a or can_b, "the two chains wait for each other"
        if can_a and (not can_b or rng.random() < 0.5):
            for t in range(beg[a_w], mid[a_w]):
                for u in lst[ptr[t]:ptr[t + 1]]:
                    assert u in done_at, f"A tile {t} ran before {u}"
            for t in range(beg[a_w], mid[a_w]):
                done_at[t] = len(done_at)
            a_done, a_w = a_w, a_w + 1
        else:
            for t in range(mid[b_w], beg[b_w + 1]):
                for u in lst[ptr[t]:ptr[t + 1]]:
                    assert u in done_at, f"B tile {t} ran before {u}"
            for t in range(mid[b_w], beg[b_w + 1]):
                done_at[t] = len(done_at)
            b_w += 1
    return done_at


@pytest.mark.parametrize("name", list(_plans()))
def test_two_branch_split_respects_every_dependency(name):
    """The planner's split of each wave (bddmp_plan_export_wave_split) against its own dependency
    lists: an A part reads only A tiles of earlier waves, a B part only B tiles of earlier waves or
    A tiles up to its wave's b_wait (the latest such wave exactly), A is the longest such prefix up
    to half the wave, and random interleavings of the two chains run every tile after its
    dependencies."""
    plan = _plans()[name]()
    rng = np.random.default_rng(11)
    for pass_ in (0, 1):
        ptr, lst, _ = plan.tile_deps(pass_)
        beg, mid, bw = plan.wave_split(pass_)
        W = len(mid)
        assert beg[0] == 0 and beg[-1] == len(ptr) - 1 and np.all(np.diff(beg) > 0)
        wave = np.repeat(np.arange(W), np.diff(beg))
        in_a = np.arange(len(ptr) - 1) < mid[wave]
        for w in range(W):
            n = beg[w + 1] - beg[w]
            assert beg[w] <= mid[w] <= beg[w + 1] and 2 * (mid[w] - beg[w]) <= n + 1
            latest = -1
            for t in range(beg[w], beg[w + 1]):
                d = lst[ptr[t]:ptr[t + 1]]
                assert np.all(wave[d] < w)
                if t < mid[w]:
                    assert np.all(in_a[d])
                else:
                    if np.any(in_a[d]):
                        latest = max(latest, int(wave[d][in_a[d]].max()))
            assert bw[w] == latest, (pass_, w)
            # the prefix stops at the cap or at the first tile reading a B tile
            if mid[w] < beg[w] + (n + 1) // 2:
                d = lst[ptr[mid[w]]:ptr[mid[w] + 1]]
                assert not np.all(in_a[d])
        for _ in range(5):
            done = _two_branch_run(ptr, lst, beg, mid, bw, rng)
            assert sorted(done) == list(range(len(ptr) - 1))


def test_two_branch_split_is_balanced_on_a_grid_mrf():
    """On the 128x128, 4-label Potts workload every wave's dependencies stay near the same relative
    position, so the A parts hold close to half of each pass's tiles and each B part waits only for
    the previous wave's A part."""
    plan = B.Plan(B.Problem.from_ilp(I.config(5)))
    for pass_ in (0, 1):
        beg, mid, bw = plan.wave_split(pass_)
        a = (mid - beg[:-1]).sum() / (beg[-1] - beg[0])
        assert 0.45 < a <= 0.5, (pass_, a)
        assert np.all(bw[1:] == np.arange(len(mid) - 1))


def _group_launch(ptr, lst, beg, w0, nw, slots, rng, done_at):
    """One wave-group launch (waves w0 .. w0 + nw - 1, tiles t0 .. t_end - 1 in pass order,
    workgroup b running tile t0 + b) under the hardware's dispatch: workgroup b goes to XCD b mod 8,
    each XCD dispatches its own workgroups in block order into `slots` slots; running workgroups
    advance in random order. A tile of the launch's first wave runs at once; a later one waits until
    every tile it depends on is done. Returns False on a deadlock."""
    t0, t_first, t_end = beg[w0], beg[w0 + 1], beg[w0 + nw]
    queues = [[b for b in range(t_end - t0) if b % 8 == x] for x in range(8)]
    running = [[] for _ in range(8)]
    while any(queues) or any(running):
        for x in range(8):
            while queues[x] and len(running[x]) < slots:
                running[x].append(queues[x].pop(0))
        ready = []
        for x in range(8):
            for b in running[x]:
                t = t0 + b
                if t < t_first or all(u in done_at for u in lst[ptr[t]:ptr[t + 1]]):
                    ready.append((x, b, t))
        if not ready:
            return False
        x, b, t = ready[rng.integers(len(ready))]
        assert t not in done_at
        for u in lst[ptr[t]:ptr[t + 1]]:
            assert u in done_at, f"tile {t} ran before {u}"
        done_at[t] = len(done_at)
        running[x].remove(b)
    return True


@pytest.mark.parametrize("name", ["cfg1", "rand", "batch"])
@pytest.mark.parametrize("group", [2, 3, 8, 4096])
def test_wave_group_launch_runs_every_tile_after_its_dependencies(name, group):
    """The wave-group launch's block mapping (the launch's tiles in pass order, one workgroup each)
    under per-XCD in-order dispatch with as few as one slot per XCD: every tile runs once, after
    every tile it reads from, and no launch deadlocks (the control below shows the ordering
    matters)."""
    plan = _plans()[name]()
    rng = np.random.default_rng(group)
    for pass_ in (0, 1):
        ptr, lst, _ = plan.tile_deps(pass_)
        beg, _, _ = plan.wave_split(pass_)
        W = len(beg) - 1
        for slots in (1, 3):
            done_at = {}
            for w0 in range(0, W, group):
                assert _group_launch(ptr, lst, beg, w0, min(group, W - w0), slots, rng, done_at), (pass_, w0, slots)
            assert sorted(done_at) == list(range(len(ptr) - 1))


def _pair_launch(ptr, lst, beg, w0, nw, slots, rng, done_at, split_rule=True):
    """One wave-group launch with two tiles per workgroup (launch mode 4): workgroup b takes tiles
    a = t0 + 2b and a + 1 (if inside the launch), dispatched as in _group_launch. When tile a + 1
    waits (it lies past the launch's first wave) and its last dependency is a, the workgroup runs a,
    then a + 1; otherwise both run together once every tile either of them waits for is done
    (split_rule False: always together). Returns (False on a deadlock, pairs run one after the
    other)."""
    t0, t_first, t_end = beg[w0], beg[w0 + 1], beg[w0 + nw]
    nb = (t_end - t0 + 1) // 2
    queues = [[b for b in range(nb) if b % 8 == x] for x in range(8)]
    running = [[] for _ in range(8)]
    step = {}
    seq = 0

    def ready(t):
        return t < t_first or all(u in done_at for u in lst[ptr[t]:ptr[t + 1]])

    def run(t):
        assert t not in done_at
        for u in lst[ptr[t]:ptr[t + 1]]:
            assert u in done_at, f"tile {t} ran before {u}"
        done_at[t] = len(done_at)

    while any(queues) or any(running):
        for x in range(8):
            while queues[x] and len(running[x]) < slots:
                b = queues[x].pop(0)
                a = t0 + 2 * b
                two = a + 1 < t_end
                d = lst[ptr[a + 1]:ptr[a + 2]] if two else []
                sequential = split_rule and two and a + 1 >= t_first and len(d) > 0 and d[-1] == a
                seq += sequential
                step[b] = [[a], [a + 1]] if sequential else [[a, a + 1] if two else [a]]
                running[x].append(b)
        movable = [(x, b) for x in range(8) for b in running[x] if all(ready(t) for t in step[b][0])]
        if not movable:
            return False, seq
        x, b = movable[rng.integers(len(movable))]
        for t in step[b].pop(0):
            run(t)
        if not step[b]:
            running[x].remove(b)
    return True, seq


@pytest.mark.parametrize("name", ["cfg1", "rand", "batch"])
@pytest.mark.parametrize("group", [2, 3, 8, 4096])
def test_two_tile_wave_group_launch_runs_every_tile_after_its_dependencies(name, group):
    """The two-tile mapping of the wave-group launch (consecutive tiles in pass order per workgroup,
    a pair across a wave boundary one tile after the other) under per-XCD in-order dispatch with as
    few as one slot per XCD: every tile runs once, after every tile it reads from, and no launch
    deadlocks; pairs across a wave boundary do occur."""
    plan = _plans()[name]()
    rng = np.random.default_rng(100 + group)
    n_seq = 0
    for pass_ in (0, 1):
        ptr, lst, _ = plan.tile_deps(pass_)
        beg, _, _ = plan.wave_split(pass_)
        W = len(beg) - 1
        for slots in (1, 3):
            done_at = {}
            for w0 in range(0, W, group):
                ok, seq = _pair_launch(ptr, lst, beg, w0, min(group, W - w0), slots, rng, done_at)
                assert ok, (pass_, w0, slots)
                n_seq += seq
            assert sorted(done_at) == list(range(len(ptr) - 1))
    assert n_seq > 0


def test_two_tile_control_pair_run_together_deadlocks():
    """Control: a pair whose second tile reads from its first, waiting for both tiles' dependencies
    before running either, waits for itself; the one-after-the-other rule runs it."""
    # two waves of one tile each: tile 1 depends on tile 0, both in one workgroup
    ptr, lst, beg = np.array([0, 0, 1]), np.array([0]), np.array([0, 1, 2])
    ok, _ = _pair_launch(ptr, lst, beg, 0, 2, 1, np.random.default_rng(0), {}, split_rule=False)
    assert not ok
    done_at = {}
    ok, seq = _pair_launch(ptr, lst, beg, 0, 2, 1, np.random.default_rng(0), done_at)
    assert ok and seq == 1 and done_at == {0: 0, 1: 1}


def test_wave_group_control_reversed_waves_deadlock():
    """Control: a launch whose later wave sits in lower blocks than the wave it depends on (the
    order the mapping forbids) deadlocks with one slot per XCD."""
    # two waves of 8 tiles; tile 8 + j depends on tile j; blocks 0..7 hold wave 1, 8..15 wave 0
    def launch(slots):
        queues = [[b for b in range(16) if b % 8 == x] for x in range(8)]
        running = [[] for _ in range(8)]
        done = set()
        while any(queues) or any(running):
            for x in range(8):
                while queues[x] and len(running[x]) < slots:
                    running[x].append(queues[x].pop(0))
            moved = False
            for x in range(8):
                for b in list(running[x]):
                    t = 8 + b if b < 8 else b - 8   # reversed: wave 1 first
                    if t < 8 or (t - 8) in done:
                        done.add(t)
                        running[x].remove(b)
                        moved = True
            if not moved:
                return False
        return True

    assert not launch(1)
    assert launch(2)
