"""Binomial checkpointing for reverse sweeps longer than the HBM trajectory budget.

The paper keeps periodic primal snapshots and recomputes the states in between when the
adjoint needs them ("Implementation", checkpointing).  With a fixed number of snapshot slots
the recomputation is minimised by the binomial schedule of Griewank & Walther ("Algorithm 799:
revolve", ACM TOMS 26, 2000): with s slots (the base included) and at most r forward
repetitions per step one can reverse beta(s, r) = C(s + r, s) steps, and the least number of
forward steps for l steps is  t(l, s) = r l - beta(s + 1, r - 1)  with r the smallest integer
for which beta(s, r) >= l.  The schedule below splits each segment at a point that attains this
minimum (the split cost is convex in the split point, so a ternary search finds it).

Actions (``schedule``):
  ("advance", i, j)   advance the working state from step i to step j (j - i primal steps)
  ("store", i)        copy the working state (step i) into a free slot
  ("reverse", i)      one reverse step n = i, reading state i from its slot or the working state
  ("free", i)         release the slot of step i
The first action reads the stored initial state; no action needs more than `slots` slots.
"""
from math import comb


def beta(s, r):
    return comb(s + r, s)


def repetitions(l, s):
    r = 0
    while beta(s, r) < l:
        r += 1
    return r


def min_advances(l, s):
    """Least number of forward steps to reverse l steps from a stored base with s slots."""
    if l <= 1:
        return 0
    if s <= 1:
        return l * (l - 1) // 2
    r = repetitions(l, s)
    return r * l - beta(s + 1, r - 1)


def _split(l, s):
    """A split point m (1 <= m < l) with m + t(l - m, s - 1) + t(m, s) = t(l, s)."""
    def cost(m):
        return m + min_advances(l - m, s - 1) + min_advances(m, s)

    lo, hi = 1, l - 1
    while hi - lo > 2:
        m1 = lo + (hi - lo) // 3
        m2 = hi - (hi - lo) // 3
        if cost(m1) <= cost(m2):
            hi = m2
        else:
            lo = m1
    return min(range(lo, hi + 1), key=cost)


def schedule(l, s):
    """Action list reversing steps l-1 .. 0 from the stored state 0 with s slots (s >= 1)."""
    if s < 1:
        raise ValueError("at least one slot (the initial state) is needed")
    acts = []

    def rev(a, b, slots):
        # precondition: state a is stored; reverses steps b-1 .. a
        if b - a == 1:
            acts.append(("reverse", a))
            return
        if slots == 1:
            for i in range(b - 1, a, -1):
                acts.append(("advance", a, i))
                acts.append(("reverse", i))
            acts.append(("reverse", a))
            return
        m = a + _split(b - a, slots)
        acts.append(("advance", a, m))
        acts.append(("store", m))
        rev(m, b, slots - 1)
        acts.append(("free", m))
        rev(a, m, slots)

    rev(0, l, s)
    return acts


def simulate(acts, l, s):
    """Checks an action list: every reverse sees its state, slots never exceed s, steps are
    reversed in order l-1 .. 0.  Returns the number of primal steps advanced."""
    stored = {0}
    work = None  # step of the working state
    advanced = 0
    expect = l - 1
    for act in acts:
        kind = act[0]
        if kind == "advance":
            i, j = act[1], act[2]
            if i not in stored and work != i:
                raise AssertionError(f"advance from {i}: state not available")
            advanced += j - i
            work = j
        elif kind == "store":
            if work != act[1]:
                raise AssertionError("store of a state that is not the working state")
            stored.add(act[1])
            if len(stored) > s:
                raise AssertionError("more than s slots in use")
        elif kind == "free":
            stored.discard(act[1])
        elif kind == "reverse":
            i = act[1]
            if i != expect:
                raise AssertionError(f"reverse {i}, expected {expect}")
            if i not in stored and work != i:
                raise AssertionError(f"reverse {i}: state not available")
            expect -= 1
    if expect != -1:
        raise AssertionError("not every step was reversed")
    return advanced


def slots_for_budget(state_bytes, budget_bytes, nsteps):
    """Number of snapshot slots that fit a byte budget (at least 2, at most nsteps)."""
    return int(max(2, min(nsteps, budget_bytes // max(1, state_bytes))))
