"""CPU model of the device-wide look-back protocol of the scans and one-sweep sorts,
run under adversarial schedules.

The model restates the protocol of the HIP kernels (it shares no code with them):
tile t publishes its aggregate, sums the aggregates of the earlier tiles of its
group of 32, and walks back over the groups' status words, 16 per round trip,
until it meets an inclusive prefix; a group's last tile publishes the group's
aggregate and then its inclusive prefix. A status word carries flag and value
together, so a reader never sees one without the other.

The dispatch model is that of a multi-XCD GPU: workgroup t goes to XCD t mod 8,
each XCD starts its own workgroups in id order as its slots free up, and any
resident block may take the next step. The adversary picks every step at random
(dispatch or block step, and with two kernels, which kernel's next workgroup an
XCD takes).

What the tests establish:
  * one kernel alone always terminates with the exact exclusive prefix, whatever
    the schedule, the slot count or the tile count (in-order dispatch per XCD is
    enough: the lowest unfinished tile is always resident or dispatchable);
  * two look-back kernels sharing the GPU (frames prepared on concurrent streams)
    CAN deadlock: XCD a full of kernel B's blocks waiting on a B tile that belongs
    to XCD b, XCD b full of kernel A's blocks waiting on an A tile that belongs to
    XCD a. A wait bound with a sticky abort word turns every such schedule into a
    prompt error of a frame instead of a hang: all blocks finish;
  * a poll that can never see what it waits for (a stale cached copy of the
    status words), bounded per block without a sticky abort, stalls the pass for
    about one bound per generation of resident blocks (the arithmetic of a
    multi-minute silence), and for about one bound in all with it.
"""
import random

import pytest

GROUP = 32
WINDOW = 16
XCDS = 8
AGG, PREFIX = 1, 2


class Kernel:
    """One look-back pass over len(values) tiles (shared status words)."""

    def __init__(self, values, withhold=-1):
        self.vals = list(values)
        self.T = len(values)
        self.ngroups = (self.T + GROUP - 1) // GROUP
        self.tstat = [(0, 0)] * self.T
        self.gstat = [(0, 0)] * self.ngroups
        self.result = [None] * self.T
        self.next = [x for x in range(XCDS)]  # next tile each XCD dispatches
        self.abort = False
        self.withhold = withhold
        self.stale = False  # defective polls: a block sees only words published before it started
        self.clock = 0
        self.tpub = [0] * self.T
        self.gpub = [0] * self.ngroups

    def pending(self, xcd):
        return self.next[xcd] < self.T

    def take(self, xcd):
        t = self.next[xcd]
        self.next[xcd] += XCDS
        return Block(self, t)

    def set_t(self, j, word):
        self.tstat[j] = word
        self.tpub[j] = self.clock

    def set_g(self, j, word):
        self.gstat[j] = word
        self.gpub[j] = self.clock

    def done(self):
        return all(r is not None for r in self.result)


class Block:
    """Tile t's protocol as a state machine; step() makes one round (a read or a
    publication) and returns whether its state changed."""

    def __init__(self, k, t):
        self.k, self.t = k, t
        self.g = t // GROUP
        self.g0 = self.g * GROUP
        self.last = t % GROUP == GROUP - 1 or t == k.T - 1
        self.phase = "publish"
        self.E = 0
        self.X = 0
        self.b = self.g - 1
        self.waited = 0
        self.finished = False
        self.start = k.clock

    def tword(self, j):
        k = self.k
        return (0, 0) if k.stale and k.tpub[j] >= self.start else k.tstat[j]

    def gword(self, j):
        k = self.k
        return (0, 0) if k.stale and k.gpub[j] >= self.start else k.gstat[j]

    def ready_intra(self):
        return all(self.tword(j)[0] != 0 for j in range(self.g0, self.t))

    def step(self, bound=None, sticky=True):
        k = self.k
        if self.phase == "publish":
            if self.t != k.withhold:
                k.set_t(self.t, (AGG, k.vals[self.t]))
            self.phase = "intra"
            return True
        if self.phase == "intra":
            if self.ready_intra():
                self.E = sum(self.tword(j)[1] for j in range(self.g0, self.t))
                if self.last and self.t != k.withhold:
                    k.set_g(self.g, (AGG, self.E + k.vals[self.t]))
                self.phase = "walk"
                self.waited = 0
                return True
            return self._wait(bound, sticky)
        if self.phase == "walk":
            if self.b < 0:
                return self._finish()
            used, found = 0, False
            for q in range(WINDOW):
                j = self.b - q
                flag, val = (PREFIX, 0) if j < 0 else self.gword(j)
                if flag == 0:
                    break
                self.X += val
                used = q + 1
                if flag == PREFIX:
                    found = True
                    break
            if found:
                return self._finish()
            self.b -= used
            if used == WINDOW:
                return True
            if used > 0:
                self.waited = 0
                return True
            return self._wait(bound, sticky)
        return False

    def _wait(self, bound, sticky):
        k = self.k
        if sticky and k.abort:
            return self._give_up()
        if bound is None:
            return False  # an unbounded wait with nothing new to read makes no progress
        self.waited += 1  # a bounded wait advances its clock
        if self.waited > bound:
            if sticky:
                k.abort = True
            return self._give_up()
        return True

    def _give_up(self):
        self.finished = True
        self.k.result[self.t] = "aborted"
        if self.last and self.t != self.k.withhold:
            self.k.set_g(self.g, (PREFIX, 0))
        return True

    def _finish(self):
        k = self.k
        if self.last and self.t != k.withhold:
            k.set_g(self.g, (PREFIX, self.X + self.E + k.vals[self.t]))
        k.result[self.t] = self.X + self.E
        self.finished = True
        return True


def run(kernels, slots, rng, bound=None, sticky=True, max_steps=2_000_000):
    """Adversarial schedule; returns ('done', steps) or ('deadlock', steps)."""
    resident = [[] for _ in range(XCDS)]
    steps = 0
    while steps < max_steps:
        if all(k.done() for k in kernels):
            return "done", steps
        moves = []
        for x in range(XCDS):
            if len(resident[x]) < slots:
                for ki, k in enumerate(kernels):
                    if k.pending(x):
                        moves.append(("dispatch", x, ki))
            for bi in range(len(resident[x])):
                moves.append(("step", x, bi))
        progressed = False
        rng.shuffle(moves)
        for mv in moves:
            steps += 1
            if mv[0] == "dispatch":
                resident[mv[1]].append(kernels[mv[2]].take(mv[1]))
                progressed = True
                break
            blk = resident[mv[1]][mv[2]]
            if blk.step(bound, sticky):
                if blk.finished:
                    resident[mv[1]].pop(mv[2])
                progressed = True
                break
        if not progressed:
            return "deadlock", steps
    return "limit", steps


def exclusive(vals):
    out, s = [], 0
    for v in vals:
        out.append(s)
        s += v
    return out


@pytest.mark.parametrize("T,slots", [(1, 1), (17, 1), (40, 2), (70, 2), (300, 3), (700, 8)])
def test_one_kernel_always_terminates_exactly(T, slots):
    for seed in range(6):
        rng = random.Random(seed * 1000 + T)
        vals = [rng.randrange(0, 50) for _ in range(T)]
        k = Kernel(vals)
        outcome, _ = run([k], slots, rng)
        assert outcome == "done", (T, slots, seed)
        assert k.result == exclusive(vals)


def test_two_kernels_can_deadlock_without_a_bound():
    """Frames on two streams: some schedule leaves every resident block waiting on
    a tile whose XCD is full of the other kernel's waiting blocks."""
    found = 0
    for seed in range(200):
        rng = random.Random(seed)
        ka = Kernel([1] * 96)
        kb = Kernel([1] * 96)
        outcome, _ = run([ka, kb], 2, rng)
        found += outcome == "deadlock"
    print("deadlocked schedules: %d of 200" % found)
    assert found > 0


def test_a_wait_bound_with_sticky_abort_ends_every_schedule():
    aborted = 0
    for seed in range(200):
        rng = random.Random(seed)
        ka = Kernel([1] * 96)
        kb = Kernel([1] * 96)
        outcome, _ = run([ka, kb], 2, rng, bound=200)
        assert outcome == "done", seed
        for k in (ka, kb):
            if k.abort:
                aborted += 1
            else:
                assert k.result == exclusive(k.vals)
    print("kernels aborted: %d of 400" % aborted)
    assert aborted > 0


def run_rounds(kernel, slots, rng, bound, sticky):
    """Elapsed time in rounds: each round the XCDs fill their free slots, then every
    resident block takes one step."""
    resident = [[] for _ in range(XCDS)]
    rounds = 0
    while not kernel.done():
        rounds += 1
        kernel.clock = rounds
        for x in range(XCDS):
            while len(resident[x]) < slots and kernel.pending(x):
                resident[x].append(kernel.take(x))
        blocks = [(x, b) for x in range(XCDS) for b in resident[x]]
        rng.shuffle(blocks)
        for x, b in blocks:
            b.step(bound, sticky)
            if b.finished:
                resident[x].remove(b)
        assert rounds < 10 ** 6
    return rounds


def test_stale_polls_cost_one_bound_per_generation_without_a_sticky_abort():
    """A defective poll that only ever sees the status words published before its
    block started (a stale cached copy): each generation of resident blocks waits
    on tiles of its own generation that it can never see. Bounded per block, every
    generation waits out the whole bound; with the sticky abort word the pass ends
    about one bound after it starts."""
    T, slots, bound = 400, 2, 300
    generations = T // (slots * XCDS)

    def elapsed(sticky):
        k = Kernel([1] * T)
        k.stale = True
        return run_rounds(k, slots, random.Random(5), bound, sticky)

    per_block, with_abort = elapsed(False), elapsed(True)
    print("rounds: per-block bounds %d, sticky abort %d; %d generations x bound %d = %d"
          % (per_block, with_abort, generations, bound, generations * bound))
    assert per_block > 0.5 * generations * bound
    assert with_abort < 3 * bound
