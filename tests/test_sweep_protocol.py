"""A CPU model of the persistent sweep kernel's synchronisation protocol,
run under random interleavings with delayed store visibility.

The sweep kernel has no grid barrier: workgroups ("parts") talk only through
words in device memory, each of which carries its own "written" mark (an
empty word holds a pattern arithmetic never produces). This model restates
the protocol's steps as coroutines, one per role of each part (the row waves
and the wave that runs the termination test, which meet at the four block
barriers of every sweep), and runs them under a random scheduler:

* exchange words of boundary variables: m^2 words per variable and parity,
  reader-major (base + reader * m + writer); each owner publishes its partial
  sum of sweep k into the words of the other owners at the end of sweep k
  (parity k % 2), and every owner reads the m - 1 words addressed to it in
  the global update of sweep k + 1, after loading them together, then
  empties them;
* the residual sums in two levels, rings of 8 sweeps: every part's sums of
  sweep k (level 1), read and emptied by its group's leader, which stores the
  group sums (level 2); every part loads the group sums of sweep k a phase
  early (and again after the local phase if they were still empty), reads
  them at the start of sweep k + 3 and runs the test; a leader empties its
  group words of sweep k once it tests sweep k + 3;
* the aggregated residual form: boundary variables' per-owner sums go to the
  variable's first owner, which reads and empties them in the next global
  update (or after the last sweep), and the part's sums of sweep k reach
  level 1 during sweep k + 1;
* memory: a store becomes visible to other parts at a random later time, in
  any order across addresses (in program order for one address), and all of
  a role's stores are visible after its explicit waits (s_waitcnt 0: the row
  waves before barrier B4, the test wave after B2 and after B4); block
  barriers alone are not assumed to publish anything; a load issued early
  keeps what it saw (a stale non-empty value would be used as it is).

Every value carries a tag (kind, sweep, writer, ...); the model checks that
every read returns the intended sweep's value, that no store overwrites a
word that is not empty (an unread value), that every role ends (no
deadlock), and that every part stops at the same sweep.
"""
import random

import pytest

EMPTY = None


class Memory:
    def __init__(self, rng):
        self.vis = {}
        self.rng = rng
        self.errors = []

    def load(self, addr):
        return self.vis.get(addr, EMPTY)

    def make_visible(self, addr, val):
        cur = self.vis.get(addr, EMPTY)
        if val is not EMPTY and cur is not EMPTY:
            self.errors.append(f"overwrite of unread {cur} at {addr} by {val}")
        self.vis[addr] = val


class Role:
    """One coroutine with a FIFO of stores not yet visible to others."""

    def __init__(self, name, gen):
        self.name = name
        self.gen = gen
        self.pending = []
        self.done = False
        self.waiting = None  # None, ("mem", predicate), ("bar", part, gen), ("drain",)


class Part:
    def __init__(self, p):
        self.p = p
        self.bar_count = 0
        self.bar_gen = 0
        self.lds = {}


def build(P, kgroup, n_var, rng):
    """Parts own contiguous runs of variables' copies, as the planner's
    depth-first runs do: each variable is held by 1 to 3 consecutive parts."""
    owners = []
    for v in range(n_var):
        m = rng.choice([1, 1, 1, 2, 2, 3])
        p0 = rng.randrange(0, P - m + 1)
        owners.append(list(range(p0, p0 + m)))
    for p in range(P):  # every part holds at least one variable
        owners.append([p])
    base, slots = [], 0
    for own in owners:
        m = len(own)
        base.append(slots if m > 1 else -1)
        if m > 1:
            slots += m * m
    parts_vars = [[] for _ in range(P)]
    for v, own in enumerate(owners):
        for me, p in enumerate(own):
            parts_vars[p].append((v, len(own), me, base[v]))
    return parts_vars


def run_model(seed, P=10, kgroup=4, n_var=24, max_iter=30, stop_at=None, agg=False, check=True, vis_p=0.3):
    rng = random.Random(seed)
    mem = Memory(rng)
    parts_vars = build(P, kgroup, n_var, rng)
    ngroups = (P + kgroup - 1) // kgroup
    nq = 7 if agg else 5
    parts = [Part(p) for p in range(P)]
    outcome = {}

    def test_result(sweep):
        # every part adds the same words, so every part takes the same decision
        return stop_at is not None and sweep >= stop_at

    def row_role(part, role):
        p = part.p
        my = parts_vars[p]
        done = 0

        def store(addr, val):
            role.pending.append((addr, val))

        def await_(addr, snap):
            if snap is not EMPTY:
                return snap
            while True:
                val = mem.load(addr)
                if val is not EMPTY:
                    return val
                role.waiting = ("mem", lambda a=addr: mem.load(a) is not EMPTY)
                yield

        # partial sums of the starting state (tag sweep 0), published
        for v, m, me, sb in my:
            if m > 1:
                for j in range(m):
                    if j != me:
                        store(("b", 0, sb + j * m + me), ("P", v, 0, me))
        yield from barrier(part, role)
        while done < max_iter:
            bp = done & 1
            # global update: the words addressed to this part, loaded together
            for v, m, me, sb in my:
                if m > 1:
                    snaps = {j: mem.load(("b", bp, sb + me * m + j)) for j in range(m) if j != me}
                    yield
                    for j in sorted(snaps):
                        val = yield from await_(("b", bp, sb + me * m + j), snaps[j])
                        if val != ("P", v, done, j):
                            mem.errors.append(f"part {p} sweep {done + 1}: read {val} for var {v} from owner {j}")
                        store(("b", bp, sb + me * m + j), EMPTY)
                    if agg and done >= 1 and me == 0:
                        for j in range(m):
                            for q in range(2):
                                val = yield from await_(("a", bp, q, sb + j), EMPTY)
                                if val != ("A1", v, done, j, q):
                                    mem.errors.append(f"part {p}: aggregated word {val} for var {v} owner {j}")
                                store(("a", bp, q, sb + j), EMPTY)
            yield from barrier(part, role)  # B1
            if part.lds.get("stop") is not None and part.lds["stop"][0] == done:
                outcome[p] = ("stop", part.lds["stop"][1])
                return
            yield from barrier(part, role)  # B2
            yield from barrier(part, role)  # B3
            yield from drain(role)          # s_waitcnt(0) before B4
            yield from barrier(part, role)  # B4
            # publication of this sweep's partial sums (sweep done + 1)
            for v, m, me, sb in my:
                if m > 1:
                    for j in range(m):
                        if j != me:
                            store(("b", bp ^ 1, sb + j * m + me), ("P", v, done + 1, me))
                    if agg:
                        for q in range(2):
                            store(("a", bp ^ 1, q, sb + me), ("A1", v, done + 1, me, q))
            done += 1
        # max_iter: the aggregated sums of the last sweep, then the barrier
        # before the test wave stores them
        if agg and done >= 1:
            bp = done & 1
            for v, m, me, sb in my:
                if m > 1 and me == 0:
                    for j in range(m):
                        for q in range(2):
                            val = yield from await_(("a", bp, q, sb + j), EMPTY)
                            if val != ("A1", v, done, j, q):
                                mem.errors.append(f"part {p}: last aggregated word {val}")
                            store(("a", bp, q, sb + j), EMPTY)
            yield from barrier(part, role)
        outcome.setdefault(p, ("max_iter", done))
        yield from drain(role)

    def test_role(part, role):
        p = part.p
        leader = p % kgroup == 0
        grp = p // kgroup
        members = [m for m in range(p, min(p + kgroup, P))] if leader else []
        done = 0
        w1, w2 = {}, {}

        def store(addr, val):
            role.pending.append((addr, val))

        def await_(addr, snap):
            if snap is not EMPTY:
                return snap
            while True:
                val = mem.load(addr)
                if val is not EMPTY:
                    return val
                role.waiting = ("mem", lambda a=addr: mem.load(a) is not EMPTY)
                yield

        def issue_members(sweep):
            for mb in members:
                for q in range(nq):
                    w1[(mb, q)] = mem.load(("r1", sweep & 7, q, mb))

        def issue_groups(sweep):
            for g in range(ngroups):
                for q in range(nq):
                    w2[(g, q)] = mem.load(("r2", sweep & 7, q, g))

        def group_sums(sweep):
            for q in range(nq):
                for mb in members:
                    val = yield from await_(("r1", sweep & 7, q, mb), w1[(mb, q)])
                    kind = "R" if q < 5 else "A"
                    if val != (kind, sweep, q, mb):
                        mem.errors.append(f"leader {p}: member word {val}, expected sweep {sweep}")
                store(("r2", sweep & 7, q, grp), ("G", sweep, q, grp))
                for mb in members:
                    store(("r1", sweep & 7, q, mb), EMPTY)

        def totals(sweep):
            for g in range(ngroups):
                for q in range(nq):
                    val = yield from await_(("r2", sweep & 7, q, g), w2[(g, q)])
                    if val != ("G", sweep, q, g):
                        mem.errors.append(f"part {p} test of sweep {sweep}: group word {val}")
            return test_result(sweep) if check else False

        yield from barrier(part, role)
        while done < max_iter:
            stop = False
            if done >= 3:
                stop = yield from totals(done - 2)
                if leader and done >= 6:
                    for q in range(nq):
                        store(("r2", (done - 5) & 7, q, grp), EMPTY)
            if stop:  # the outcome is in LDS before B1, read by both roles after it
                part.lds["stop"] = (done, done - 2)
            yield from barrier(part, role)  # B1
            if stop:
                return
            if agg and done >= 1:
                for q in (5, 6):
                    store(("r1", done & 7, q, p), ("A", done, q, p))
            yield from barrier(part, role)  # B2
            yield from drain(role)
            if leader and done >= 1:
                issue_members(done)
            if done >= 2:
                issue_groups(done - 1)
            yield from barrier(part, role)  # B3
            yield from barrier(part, role)  # B4
            yield from drain(role)
            if done >= 2:
                for key in list(w2):
                    if w2[key] is EMPTY:
                        w2[key] = mem.load(("r2", (done - 1) & 7, key[1], key[0]))
            if leader and done >= 1:
                yield from group_sums(done)
            for q in range(5):
                store(("r1", (done + 1) & 7, q, p), ("R", done + 1, q, p))
            done += 1
        # max_iter: the last sweep's group sums, then the untested sweeps
        if agg and done >= 1:
            yield from barrier(part, role)
            for q in (5, 6):
                store(("r1", done & 7, q, p), ("A", done, q, p))
        if leader and done >= 1:
            yield from drain(role)
            issue_members(done)
            yield from group_sums(done)
        for k in range(max(done - 2, 1), done + 1):
            issue_groups(k)
            yield from totals(k)
        yield from drain(role)

    def barrier(part, role):
        part.bar_count += 1
        my_gen = part.bar_gen
        if part.bar_count == 2:
            part.bar_count = 0
            part.bar_gen += 1
            yield
            return
        role.waiting = ("bar", part, my_gen)
        yield

    def drain(role):
        role.waiting = ("drain",)
        yield

    roles = []
    for part in parts:
        r = Role(f"row{part.p}", None)
        r.gen = row_role(part, r)
        t = Role(f"test{part.p}", None)
        t.gen = test_role(part, t)
        roles += [r, t]

    def runnable(r):
        if r.done:
            return False
        w = r.waiting
        if w is None:
            return True
        if w[0] == "mem":
            return w[1]()
        if w[0] == "bar":
            return w[1].bar_gen != w[2]
        if w[0] == "drain":
            return not r.pending
        return True

    steps = 0
    while True:
        steps += 1
        assert steps < 2_000_000, "model did not finish"
        # stores become visible at random times, in any order across
        # addresses, in program order for one address
        for r in roles:
            while r.pending and rng.random() < vis_p:
                seen, firsts = set(), []
                for i, (addr, _) in enumerate(r.pending):
                    if addr not in seen:
                        seen.add(addr)
                        firsts.append(i)
                addr, val = r.pending.pop(rng.choice(firsts))
                mem.make_visible(addr, val)
        ready = [r for r in roles if runnable(r)]
        if not ready:
            if all(r.done for r in roles) and not any(r.pending for r in roles):
                break
            if any(r.pending for r in roles):
                for r in roles:
                    if r.pending:
                        addr, val = r.pending.pop(0)
                        mem.make_visible(addr, val)
                continue
            stuck = [(r.name, r.waiting[0]) for r in roles if not r.done]
            raise AssertionError(f"deadlock: {stuck[:6]}")
        r = rng.choice(ready)
        r.waiting = None
        try:
            next(r.gen)
        except StopIteration:
            r.done = True
    return mem.errors, outcome


@pytest.mark.parametrize("agg", [False, True])
@pytest.mark.parametrize("seed", range(12))
def test_protocol_stops_together(seed, agg):
    stop_at = 9 + seed % 7
    errors, outcome = run_model(seed, stop_at=stop_at, agg=agg)
    assert not errors, errors[:5]
    assert set(outcome.values()) == {("stop", stop_at)}, outcome


@pytest.mark.parametrize("agg", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_protocol_runs_to_max_iter(seed, agg):
    errors, outcome = run_model(100 + seed, max_iter=17 + seed, check=False, agg=agg)
    assert not errors, errors[:5]
    assert set(outcome.values()) == {("max_iter", 17 + seed)}, outcome


def _variant(changes):
    """run_model with steps of the protocol changed (planted on the CPU only,
    to show the model catches them)."""
    import inspect
    import textwrap
    code = textwrap.dedent(inspect.getsource(run_model))
    broken = code
    for old, new in changes:
        assert old in broken, old
        broken = broken.replace(old, new)
    ns = dict(globals())
    exec(compile(broken, "<variant>", "exec"), ns)
    return ns["run_model"]


@pytest.mark.parametrize("changes", [
    # a leader that never empties its group words: the ring's reuse after
    # 8 sweeps finds them full
    [("if leader and done >= 6:", "if False:")],
    # a leader that empties them a sweep early (group words of sweep
    # done - 4 may still be unread by some part)
    [("store((\"r2\", (done - 5) & 7, q, grp), EMPTY)", "store((\"r2\", (done - 4) & 7, q, grp), EMPTY)")],
    # row waves that publish without first waiting for their own emptying
    # stores: a late empty can erase the neighbour's next word
    [("yield from drain(role)          # s_waitcnt(0) before B4", "pass")],
    # one parity of exchange words instead of two
    [("bp = done & 1\n            # global update", "bp = 0\n            # global update"),
     ("store((\"b\", bp ^ 1, sb + j * m + me)", "store((\"b\", bp, sb + j * m + me)")],
])
def test_model_catches_planted_protocol_mistakes(changes):
    variant = _variant(changes)
    caught = 0
    for seed in range(40):
        try:
            errors, outcome = variant(seed, max_iter=30, stop_at=20, vis_p=0.05)
        except AssertionError:
            caught += 1  # deadlock
            continue
        if errors or set(outcome.values()) != {("stop", 20)}:
            caught += 1
    assert caught > 0
