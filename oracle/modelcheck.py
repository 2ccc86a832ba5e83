"""Exhaustive-interleaving model checker for the synchronization algorithms.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the GPU library).

Every algorithm is written as a per-agent state machine whose transitions are single
atomic memory steps (a load, a store, an exchange, a compare-and-swap or a
fetch-and-add).  ``explore`` enumerates every interleaving of 2-3 agents under
sequential consistency and checks, on every reachable state:

* the safety property of Section 5's definition of the primitive (barrier: no agent
  reads a round's data before every agent published it, nor after it was overwritten;
  mutex: at most one agent inside; semaphore: at most K inside; ticket locks: admission
  in ticket order),
* a final-state property once every agent is done (exact counters and the algorithm's
  quiescent state),
* that from every reachable state a state with every agent done is still reachable
  (no deadlock, no livelock without an escape).

Backoff only delays steps, so it does not change the set of interleavings and is not
modelled.  The ``mutant`` options plant known-wrong variants; the test-suite requires
the checker to find a violation in each of them.
"""

from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class Result:
    states: int
    violation: str | None = None
    trace: list = field(default_factory=list)
    deadlock: bool = False

    @property
    def ok(self) -> bool:
        return self.violation is None and not self.deadlock


def explore(model, limit: int = 4_000_000) -> Result:
    """Depth-first enumeration of all interleavings of ``model``."""
    init = model.init()
    index = {init: 0}
    states = [init]
    parent = [-1]
    succ: list[list[int]] = [[]]
    stack = [0]
    n = model.n

    def trace_of(i):
        out = []
        while i >= 0:
            out.append(states[i])
            i = parent[i]
        return out[::-1]

    while stack:
        i = stack.pop()
        sh, los = states[i]
        msg = model.check(sh, los)
        if msg:
            return Result(len(states), msg, trace_of(i))
        active = False
        for a in range(n):
            if model.done(los[a]):
                continue
            active = True
            sh2, lo2 = model.step(a, sh, los[a])
            nxt = (sh2, los[:a] + (lo2,) + los[a + 1:])
            j = index.get(nxt)
            if j is None:
                j = len(states)
                if j >= limit:
                    raise RuntimeError(f"state limit {limit} exceeded")
                index[nxt] = j
                states.append(nxt)
                parent.append(i)
                succ.append([])
                stack.append(j)
            succ[i].append(j)
        if not active:
            msg = model.final_check(sh, los)
            if msg:
                return Result(len(states), msg, trace_of(i))

    # Liveness: every state must be able to reach a terminal (all agents done) state.
    pred: list[list[int]] = [[] for _ in states]
    for i, ss in enumerate(succ):
        for j in ss:
            pred[j].append(i)
    good = [False] * len(states)
    work = [i for i, (sh, los) in enumerate(states) if all(model.done(lo) for lo in los)]
    for i in work:
        good[i] = True
    while work:
        j = work.pop()
        for i in pred[j]:
            if not good[i]:
                good[i] = True
                work.append(i)
    if not all(good):
        bad = good.index(False)
        return Result(len(states), "deadlock: no way to finish", trace_of(bad), deadlock=True)
    return Result(len(states))


# ------------------------------------------------------------------------------------
# Mutexes.  Each agent acquires the single lock `ops` times; the critical section is a
# non-atomic increment of `data` (a load step then a store step).
# shared = (lock, ticket, turn, data, inside, entries)
# local  = (pc, j, tmp, my)
# ------------------------------------------------------------------------------------

class MutexModel:
    """kind: 'spin_cas'   -- compare-and-swap 0 -> 1 until it succeeds;
             'spin_exch'  -- exchange with 1 until the old value is 0 (Algorithms 1, 2);
             'ticket'     -- fetch-and-add a ticket, poll turn, unlock by a plain
                             load and store of turn + 1 (Algorithm 3);
             'sleep'      -- poll the word with loads until it reads 0, then one
                             compare-and-swap (test-and-test-and-set).
       mutant: 'check_then_set' -- 'sleep' with the compare-and-swap replaced by a plain
                             store of 1 (test, then set, as two separate steps);
               'skip_release'   -- unlock does nothing (must be reported as a deadlock)."""

    ACQ, POLL, TEST, TRY, CS_IN, CS_LD, CS_ST, CS_OUT, REL, REL2, DONE = range(11)

    def __init__(self, kind: str, n: int = 3, ops: int = 2, mutant: str | None = None):
        self.kind, self.n, self.ops, self.mutant = kind, n, ops, mutant

    def init(self):
        return (0, 0, 0, 0, 0, 0), tuple((self.ACQ, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    def step(self, a, sh, lo):
        lock, ticket, turn, data, inside, entries = sh
        pc, j, tmp, my = lo
        k = self.kind
        if pc == self.ACQ:
            if k == "spin_cas":
                if lock == 0:
                    return (1, ticket, turn, data, inside, entries), (self.CS_IN, j, tmp, my)
                return sh, lo
            if k == "spin_exch":
                old = lock
                sh = (1, ticket, turn, data, inside, entries)
                return sh, ((self.CS_IN if old == 0 else self.ACQ), j, tmp, my)
            if k == "ticket":
                return (lock, ticket + 1, turn, data, inside, entries), (self.POLL, j, tmp, ticket)
            return sh, (self.TEST, j, tmp, my)  # sleep
        if pc == self.POLL:  # ticket: wait until turn equals my ticket
            return sh, ((self.CS_IN if turn == my else self.POLL), j, tmp, my)
        if pc == self.TEST:  # sleep: load until the word reads free
            return sh, ((self.TRY if lock == 0 else self.TEST), j, tmp, my)
        if pc == self.TRY:
            if self.mutant == "check_then_set":
                return (1, ticket, turn, data, inside, entries), (self.CS_IN, j, tmp, my)
            if lock == 0:
                return (1, ticket, turn, data, inside, entries), (self.CS_IN, j, tmp, my)
            return sh, (self.TEST, j, tmp, my)
        if pc == self.CS_IN:
            return (lock, ticket, turn, data, inside + 1, entries), (self.CS_LD, j, tmp, my)
        if pc == self.CS_LD:
            return sh, (self.CS_ST, j, data, my)
        if pc == self.CS_ST:
            return (lock, ticket, turn, tmp + 1, inside, entries), (self.CS_OUT, j, tmp, my)
        if pc == self.CS_OUT:
            return (lock, ticket, turn, data, inside - 1, entries + 1), (self.REL, j, tmp, my)
        nxt = self.ACQ if j + 1 < self.ops else self.DONE
        if pc == self.REL:
            if self.mutant == "skip_release":
                return sh, (nxt, j + 1, tmp, my)
            if k == "ticket":  # only the holder writes turn: a plain load ...
                return sh, (self.REL2, j, turn, my)
            return (0, ticket, turn, data, inside, entries), (nxt, j + 1, tmp, my)
        if pc == self.REL2:  # ... then a plain store of turn + 1
            return (lock, ticket, tmp + 1, data, inside, entries), (nxt, j + 1, tmp, my)
        raise AssertionError(pc)

    def check(self, sh, los):
        inside, entries = sh[4], sh[5]
        if inside > 1:
            return f"mutual exclusion violated: {inside} inside"
        if self.kind == "ticket":
            for pc, j, tmp, my in los:
                if pc == self.CS_LD and my != entries:
                    return f"ticket order violated: ticket {my} entered after {entries} entries"
        return None

    def final_check(self, sh, los):
        total = self.n * self.ops
        if sh[3] != total:
            return f"lost update: data {sh[3]} != {total}"
        if self.mutant == "skip_release":
            return None
        if self.kind == "ticket" and not (sh[1] == sh[2] == total):
            return f"ticket/turn {sh[1]}/{sh[2]} != {total}"
        if self.kind != "ticket" and sh[0] != 0:
            return "lock left held"
        return None


class QueueLockModel:
    """Queue mutexes over a ring of Q slots; tail draws tickets, FIFO by construction.
    kind: 'ring'  -- Section 5's ring-buffer mutex: an arriving agent draws ticket t,
                     writes its id (t + 1) into slot t mod Q, then polls head and the
                     slot head points at until that slot holds its id; unlock stores
                     head = t + 1;
          'array' -- every agent polls only its own slot t mod Q until it holds t;
                     unlock grants slot (t + 1) mod Q the value t + 1.
    mutant: 'small_ring' -- Q = n - 1, fewer slots than contenders (the ring needs one
                            slot per contender: an id can be overwritten before its
                            owner reaches the head);
            'skip_write' -- ring without writing one's own id;
            'grant_self' -- array unlock writes t + 1 into its own slot t mod Q."""

    ACQ, WRITE, POLL_H, POLL_R, POLL, CS_IN, CS_LD, CS_ST, CS_OUT, REL, DONE = range(11)

    def __init__(self, kind: str, n: int = 3, ops: int = 2, Q: int | None = None,
                 mutant: str | None = None):
        self.kind, self.n, self.ops, self.mutant = kind, n, ops, mutant
        self.Q = (n - 1 if mutant == "small_ring" else n) if Q is None else Q

    def init(self):
        # shared = (tail, head, slots, data, inside, entries); local = (pc, j, tmp, t)
        return (0, 0, (0,) * self.Q, 0, 0, 0), tuple((self.ACQ, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    def _slot(self, slots, i, v):
        return slots[:i] + (v,) + slots[i + 1:]

    def step(self, a, sh, lo):
        tail, head, slots, data, inside, entries = sh
        pc, j, tmp, t = lo
        Q = self.Q
        if pc == self.ACQ:
            sh = (tail + 1, head, slots, data, inside, entries)
            return sh, ((self.WRITE if self.kind == "ring" else self.POLL), j, tmp, tail)
        if pc == self.WRITE:
            if self.mutant != "skip_write":
                slots = self._slot(slots, t % Q, t + 1)
            return (tail, head, slots, data, inside, entries), (self.POLL_H, j, tmp, t)
        if pc == self.POLL_H:
            return sh, (self.POLL_R, j, head, t)
        if pc == self.POLL_R:
            return sh, ((self.CS_IN if slots[tmp % Q] == t + 1 else self.POLL_H), j, tmp, t)
        if pc == self.POLL:
            return sh, ((self.CS_IN if slots[t % Q] == t else self.POLL), j, tmp, t)
        if pc == self.CS_IN:
            return (tail, head, slots, data, inside + 1, entries), (self.CS_LD, j, tmp, t)
        if pc == self.CS_LD:
            return sh, (self.CS_ST, j, data, t)
        if pc == self.CS_ST:
            return (tail, head, slots, tmp + 1, inside, entries), (self.CS_OUT, j, tmp, t)
        if pc == self.CS_OUT:
            return (tail, head, slots, data, inside - 1, entries + 1), (self.REL, j, tmp, t)
        if pc == self.REL:
            nxt = self.ACQ if j + 1 < self.ops else self.DONE
            if self.kind == "ring":
                return (tail, t + 1, slots, data, inside, entries), (nxt, j + 1, tmp, t)
            at = t % Q if self.mutant == "grant_self" else (t + 1) % Q
            slots = self._slot(slots, at, t + 1)
            return (tail, head, slots, data, inside, entries), (nxt, j + 1, tmp, t)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[4] > 1:
            return f"mutual exclusion violated: {sh[4]} inside"
        for pc, j, tmp, t in los:
            if pc == self.CS_LD and t != sh[5]:
                return f"queue order violated: ticket {t} entered after {sh[5]} entries"
        return None

    def final_check(self, sh, los):
        total = self.n * self.ops
        if sh[3] != total or sh[0] != total:
            return f"final data {sh[3]} tail {sh[0]} != {total}"
        if self.kind == "ring" and sh[1] != total:
            return f"final head {sh[1]} != {total}"
        return None


class CohortLockModel:
    """XCD-cohort lock: a local ticket lock per cohort (agent a belongs to cohort a mod C)
    in front of a global ticket lock.  Each cohort has G grant slots; local ticket t polls
    slot t mod G, which holds the local turn and the session together (one store writes
    both, one load reads both): session 0 says the cohort does not hold the global lock,
    k > 0 that it does and k holders have passed it on.  A local holder that reads
    session 0 takes the global lock.  Unlock (by the holder of local ticket t) writes slot
    (t + 1) mod G: when a local waiter exists (local tickets drawn beyond one's own) and
    k + 1 < B, grant (t + 1, k + 1) -- the global lock stays with the cohort; else release
    the global lock, then grant (t + 1, 0).  G = 1 is the single grant word; with G > 1
    tickets t and t + G share a slot, which is rewritten only after t has entered.
    mutant 'keep_session': a global release grants (turn + 1, k + 1);
    mutant 'no_waiter_check': pass locally even when nobody of the cohort waits;
    mutant 'skip_global_wait': a holder reading session 0 takes a global ticket but
    enters without waiting for its turn;
    mutant 'own_slot': the grant goes into the holder's own slot t mod G."""

    (ACQ, POLL_L, G_ACQ, POLL_G, CS_IN, CS_LD, CS_ST, CS_OUT, REL, REL_G, REL_L,
     DONE) = range(12)

    def __init__(self, n: int = 4, ops: int = 2, C: int = 2, B: int = 2,
                 mutant: str | None = None, G: int = 1):
        self.n, self.ops, self.C, self.B, self.mutant, self.G = n, ops, C, B, mutant, G

    def init(self):
        C, G = self.C, self.G
        # shared = (gticket, gturn, lticket, slots (C x G of (turn, session)), data,
        #           inside, entries)
        # local  = (pc, j, tmp, t, s)
        sh = (0, 0, (0,) * C, tuple(((0, 0),) * G for _ in range(C)), 0, 0, 0)
        return sh, tuple((self.ACQ, 0, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(tup, i, v):
        return tup[:i] + (v,) + tup[i + 1:]

    def _grant(self, slots, c, t, turn, sess):
        i = (t if self.mutant == "own_slot" else t + 1) % self.G
        return self._set(slots, c, self._set(slots[c], i, (turn, sess)))

    def step(self, a, sh, lo):
        gt, gturn, lt, slots, data, inside, entries = sh
        pc, j, tmp, t, s = lo
        c = a % self.C
        nxt = self.ACQ if j + 1 < self.ops else self.DONE
        if pc == self.ACQ:
            return (gt, gturn, self._set(lt, c, lt[c] + 1), slots, data, inside,
                    entries), (self.POLL_L, j, tmp, lt[c], s)
        if pc == self.POLL_L:  # reads turn and session in one load
            turn, sess = slots[c][t % self.G]
            if turn != t:
                return sh, (self.POLL_L, j, tmp, t, s)
            return sh, ((self.G_ACQ if sess == 0 else self.CS_IN), j, tmp, t, sess)
        if pc == self.G_ACQ:
            after = self.CS_IN if self.mutant == "skip_global_wait" else self.POLL_G
            return (gt + 1, gturn, lt, slots, data, inside, entries), (after, j, gt, t, s)
        if pc == self.POLL_G:
            return sh, ((self.CS_IN if gturn == tmp else self.POLL_G), j, tmp, t, s)
        if pc == self.CS_IN:
            return (gt, gturn, lt, slots, data, inside + 1, entries), (self.CS_LD, j, tmp, t, s)
        if pc == self.CS_LD:
            return sh, (self.CS_ST, j, data, t, s)
        if pc == self.CS_ST:
            return (gt, gturn, lt, slots, tmp + 1, inside, entries), (self.CS_OUT, j, tmp, t, s)
        if pc == self.CS_OUT:
            return (gt, gturn, lt, slots, data, inside - 1, entries + 1), (self.REL, j, tmp, t, s)
        if pc == self.REL:
            waiter = lt[c] > t + 1 or self.mutant == "no_waiter_check"
            if waiter and s + 1 < self.B:  # pass: one store of the grant
                return (gt, gturn, lt, self._grant(slots, c, t, t + 1, s + 1),
                        data, inside, entries), (nxt, j + 1, tmp, t, s)
            return sh, (self.REL_G, j, tmp, t, s)
        if pc == self.REL_G:
            return (gt, gturn + 1, lt, slots, data, inside, entries), (self.REL_L, j, tmp, t, s)
        if pc == self.REL_L:
            k = s + 1 if self.mutant == "keep_session" else 0
            return (gt, gturn, lt, self._grant(slots, c, t, t + 1, k), data, inside,
                    entries), (nxt, j + 1, tmp, t, s)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[5] > 1:
            return f"mutual exclusion violated: {sh[5]} inside"
        return None

    def final_check(self, sh, los):
        gt, gturn, lt, slots, data, inside, entries = sh
        total = self.n * self.ops
        if data != total or entries != total:
            return f"final data {data} entries {entries} != {total}"
        # each cohort's next ticket finds its turn with session 0
        if gt != gturn or any(slots[c][lt[c] % self.G] != (lt[c], 0) for c in range(self.C)):
            return f"final state gticket {gt} gturn {gturn} local {lt} slots {slots}"
        return None


class MCSLockModel:
    """MCS queue lock (a linked queue of per-waiter nodes; each waiter polls a word of its
    own node).  Node a+1 belongs to agent a; 0 is "none".  tail is the lock word.
    lock:   my.next = 0; my.locked = 1; prev = exchange(tail, me);
            if prev: prev.next = me, then poll my.locked until 0.
    unlock: if my.next == 0: if compare-and-swap(tail, me -> 0) succeeds, done;
            otherwise poll my.next until it is set; then successor.locked = 0.
    mutant 'no_wait_for_next': a failed compare-and-swap returns without handing over;
    mutant 'link_before_init': my.locked = 1 is stored after linking into prev.next;
    mutant 'store_tail': unlock clears tail with a plain store instead of the
    compare-and-swap when next reads 0;
    mutant 'no_spin': a waiter with a predecessor enters once it has linked in."""

    (INIT_N, INIT_L, XCHG, LINK, SPIN, CS_IN, CS_LD, CS_ST, CS_OUT, REL_RD, REL_CAS,
     REL_WAIT, REL_GO, LATE_L, DONE) = range(15)

    def __init__(self, n: int = 3, ops: int = 2, mutant: str | None = None):
        self.n, self.ops, self.mutant = n, ops, mutant

    def init(self):
        # shared = (tail, next (n), locked (n), data, inside, entries); local = (pc, j, tmp, prev)
        n = self.n
        return (0, (0,) * n, (0,) * n, 0, 0, 0), tuple((self.INIT_N, 0, 0, 0) for _ in range(n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(tup, i, v):
        return tup[:i] + (v,) + tup[i + 1:]

    def step(self, a, sh, lo):
        tail, nxt, locked, data, inside, entries = sh
        pc, j, tmp, prev = lo
        me = a + 1
        fin = self.INIT_N if j + 1 < self.ops else self.DONE
        if pc == self.INIT_N:
            after = self.XCHG if self.mutant == "link_before_init" else self.INIT_L
            return (tail, self._set(nxt, a, 0), locked, data, inside, entries), (after, j, tmp, prev)
        if pc == self.INIT_L:
            return (tail, nxt, self._set(locked, a, 1), data, inside, entries), (self.XCHG, j, tmp, prev)
        if pc == self.XCHG:
            sh = (me, nxt, locked, data, inside, entries)
            if tail == 0:
                return sh, (self.CS_IN, j, tmp, 0)
            return sh, (self.LINK, j, tmp, tail)
        if pc == self.LINK:
            sh = (tail, self._set(nxt, prev - 1, me), locked, data, inside, entries)
            after = self.LATE_L if self.mutant == "link_before_init" else self.SPIN
            if self.mutant == "no_spin":
                after = self.CS_IN
            return sh, (after, j, tmp, prev)
        if pc == self.LATE_L:
            return (tail, nxt, self._set(locked, a, 1), data, inside, entries), (self.SPIN, j, tmp, prev)
        if pc == self.SPIN:
            return sh, ((self.CS_IN if locked[a] == 0 else self.SPIN), j, tmp, prev)
        if pc == self.CS_IN:
            return (tail, nxt, locked, data, inside + 1, entries), (self.CS_LD, j, tmp, prev)
        if pc == self.CS_LD:
            return sh, (self.CS_ST, j, data, prev)
        if pc == self.CS_ST:
            return (tail, nxt, locked, tmp + 1, inside, entries), (self.CS_OUT, j, tmp, prev)
        if pc == self.CS_OUT:
            return (tail, nxt, locked, data, inside - 1, entries + 1), (self.REL_RD, j, tmp, prev)
        if pc == self.REL_RD:
            if nxt[a] != 0:
                return sh, (self.REL_GO, j, nxt[a], prev)
            return sh, (self.REL_CAS, j, tmp, prev)
        if pc == self.REL_CAS:
            if self.mutant == "store_tail":
                return (0, nxt, locked, data, inside, entries), (fin, j + 1, tmp, prev)
            if tail == me:
                return (0, nxt, locked, data, inside, entries), (fin, j + 1, tmp, prev)
            if self.mutant == "no_wait_for_next":
                return sh, (fin, j + 1, tmp, prev)
            return sh, (self.REL_WAIT, j, tmp, prev)
        if pc == self.REL_WAIT:
            if nxt[a] != 0:
                return sh, (self.REL_GO, j, nxt[a], prev)
            return sh, lo
        if pc == self.REL_GO:
            return (tail, nxt, self._set(locked, tmp - 1, 0), data, inside, entries), (fin, j + 1, tmp, prev)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[4] > 1:
            return f"mutual exclusion violated: {sh[4]} inside"
        return None

    def final_check(self, sh, los):
        total = self.n * self.ops
        if sh[3] != total or sh[5] != total:
            return f"final data {sh[3]} entries {sh[5]} != {total}"
        if sh[0] != 0:
            return f"lock left with tail {sh[0]}"
        return None


class CondModel:
    """Bounded buffer on a mutex and two condition variables (Mesa semantics).
    The mutex is one atomic test-and-set word.  A condition variable is two counters:
    wait(c): t = waiters[c]++ (while holding the mutex); unlock; poll until
    signals[c] > t; lock again.  signal(c): if signals[c] < waiters[c], signals[c] += 1
    (one compare-and-swap step).  Producers put `items` values each into a buffer of
    capacity C (while count == C: wait(not_full); put; signal(not_empty)); consumers take
    their quota (while count == 0: wait(not_empty); take; signal(not_full)).
    Checks: 0 <= count <= C, mutual exclusion, every item consumed, no deadlock.
    mutant 'late_register': wait draws its ticket after unlocking (a lost wakeup);
    mutant 'if_not_while': the predicate is tested once, not re-tested after waking;
    mutant 'no_signal': producers do not signal."""

    # local program counters
    (LOCK, CHECK, REG, UNLOCK_W, POLL, RELOCK, ACT, SIGNAL, UNLOCK, DONE) = range(10)

    def __init__(self, producers: int = 1, consumers: int = 2, items: int = 2, C: int = 1,
                 mutant: str | None = None):
        self.P, self.Cn, self.items, self.C, self.mutant = producers, consumers, items, C, mutant
        self.n = producers + consumers
        total = producers * items
        self.quota = [items] * producers + [total // consumers + (1 if i < total % consumers
                                                                  else 0)
                                            for i in range(consumers)]

    def init(self):
        # shared = (mutex, count, inside, waiters(2), signals(2)); cv 0 = not_full, 1 = not_empty
        return (0, 0, 0, (0, 0), (0, 0)), tuple((self.LOCK, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    def step(self, a, sh, lo):
        mutex, count, inside, W, S = sh
        pc, j, t = lo
        prod = a < self.P
        cv_wait = 0 if prod else 1     # producers wait on not_full, consumers on not_empty
        cv_sig = 1 if prod else 0
        if pc == self.LOCK:
            if mutex:
                return sh, lo
            return (1, count, inside + 1, W, S), (self.CHECK, j, t)
        if pc == self.CHECK:  # predicate test while holding the mutex
            blocked = count == self.C if prod else count == 0
            if blocked:
                return sh, (self.REG if self.mutant != "late_register" else self.UNLOCK_W, j, t)
            return sh, (self.ACT, j, t)
        if pc == self.REG:  # register with the condition variable (mutex held)
            W2 = tuple(w + (1 if i == cv_wait else 0) for i, w in enumerate(W))
            nxt = self.UNLOCK_W if self.mutant != "late_register" else self.POLL
            return (mutex, count, inside, W2, S), (nxt, j, W[cv_wait])
        if pc == self.UNLOCK_W:
            nxt = self.POLL if self.mutant != "late_register" else self.REG
            return (0, count, inside - 1, W, S), (nxt, j, t)
        if pc == self.POLL:
            return sh, ((self.RELOCK if S[cv_wait] > t else self.POLL), j, t)
        if pc == self.RELOCK:
            if mutex:
                return sh, lo
            nxt = self.ACT if self.mutant == "if_not_while" else self.CHECK
            return (1, count, inside + 1, W, S), (nxt, j, t)
        if pc == self.ACT:
            count2 = count + 1 if prod else count - 1
            return (mutex, count2, inside, W, S), (self.SIGNAL, j, t)
        if pc == self.SIGNAL:
            if self.mutant == "no_signal" and prod:
                return sh, (self.UNLOCK, j, t)
            if S[cv_sig] < W[cv_sig]:
                S = tuple(x + (1 if i == cv_sig else 0) for i, x in enumerate(S))
            return (mutex, count, inside, W, S), (self.UNLOCK, j, t)
        if pc == self.UNLOCK:
            nxt = self.LOCK if j + 1 < self.quota[a] else self.DONE
            return (0, count, inside - 1, W, S), (nxt, j + 1, t)
        raise AssertionError(pc)

    def check(self, sh, los):
        mutex, count, inside, W, S = sh
        if inside > 1:
            return f"mutual exclusion violated: {inside} inside"
        if not 0 <= count <= self.C:
            return f"buffer count {count} outside [0, {self.C}]"
        return None

    def final_check(self, sh, los):
        if sh[1] != 0:
            return f"items left in the buffer: {sh[1]}"
        return None


# ------------------------------------------------------------------------------------
# Semaphores with initial value K.  Each agent performs `ops` wait/post pairs with an
# occupancy counter incremented on entry and decremented on exit.
# Algorithm 4 shared = (S, inside);            local = (pc, j, v)
# Algorithm 5 shared = (count, ticket, turn, inside); local = (pc, j, idx)
# ------------------------------------------------------------------------------------

class SpinSemModel:
    """Algorithm 4: S starts at K + 1; 0 means another agent is updating it.
    wait: exchange S with 0 -> v; v > 1: store v - 1 and enter; v == 1: store 1 back
    (at capacity) and retry; v == 0: retry.  post: exchange S with 0 -> v; v > 0: store
    v + 1 and leave; v == 0: retry.
    mutant 'enter_at_one': a waiter that reads v == 1 enters (an off-by-one in the
    K + 1 encoding)."""

    W0, W_TAKE, W_RESTORE, CS_IN, CS_OUT, P0, P_GIVE, DONE = range(8)

    def __init__(self, K: int, n: int = 3, ops: int = 2, mutant: str | None = None):
        self.K, self.n, self.ops, self.mutant = K, n, ops, mutant

    def init(self):
        return (self.K + 1, 0), tuple((self.W0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    def step(self, a, sh, lo):
        S, inside = sh
        pc, j, v = lo
        if pc == self.W0:
            v = S
            sh = (0, inside)
            if v > 1 or (v == 1 and self.mutant == "enter_at_one"):
                return sh, (self.W_TAKE, j, v)
            if v == 1:
                return sh, (self.W_RESTORE, j, v)
            return sh, (self.W0, j, v)
        if pc == self.W_TAKE:
            return (v - 1, inside), (self.CS_IN, j, v)
        if pc == self.W_RESTORE:
            return (1, inside), (self.W0, j, v)
        if pc == self.CS_IN:
            return (S, inside + 1), (self.CS_OUT, j, v)
        if pc == self.CS_OUT:
            return (S, inside - 1), (self.P0, j, v)
        if pc == self.P0:
            v = S
            sh = (0, inside)
            return sh, ((self.P_GIVE if v > 0 else self.P0), j, v)
        if pc == self.P_GIVE:
            nxt = self.W0 if j + 1 < self.ops else self.DONE
            return (v + 1, inside), (nxt, j + 1, 0)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[1] > self.K:
            return f"occupancy {sh[1]} > K={self.K}"
        return None

    def final_check(self, sh, los):
        if sh[0] != self.K + 1:
            return f"final S {sh[0]} != K+1"
        return None



class FASemModel:
    """Algorithm 5: count, ticket and turn start at 0.
    wait: old = fetch-and-add(count, 1); old < K: enter; otherwise idx =
    fetch-and-add(ticket, 1) and poll until turn > idx.
    post: old = fetch-and-add(count, -1); old > K: fetch-and-add(turn, 1).
    mutant 'geq': the waiter proceeds once turn >= idx (the prose wording with 0-based
    tickets).  mutant 'always_bump': post increments turn unconditionally."""

    W0, W_TICKET, W_POLL, CS_IN, CS_OUT, P0, P_BUMP, DONE = range(8)

    def __init__(self, K: int, n: int = 3, ops: int = 2, mutant: str | None = None):
        self.K, self.n, self.ops, self.mutant = K, n, ops, mutant

    def init(self):
        return (0, 0, 0, 0), tuple((self.W0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    def step(self, a, sh, lo):
        count, ticket, turn, inside = sh
        pc, j, idx = lo
        if pc == self.W0:
            old = count
            sh = (count + 1, ticket, turn, inside)
            return sh, ((self.CS_IN if old < self.K else self.W_TICKET), j, idx)
        if pc == self.W_TICKET:
            return (count, ticket + 1, turn, inside), (self.W_POLL, j, ticket)
        if pc == self.W_POLL:
            go = turn >= idx if self.mutant == "geq" else turn > idx
            return sh, ((self.CS_IN if go else self.W_POLL), j, idx)
        if pc == self.CS_IN:
            return (count, ticket, turn, inside + 1), (self.CS_OUT, j, idx)
        if pc == self.CS_OUT:
            return (count, ticket, turn, inside - 1), (self.P0, j, idx)
        nxt = self.W0 if j + 1 < self.ops else self.DONE
        if pc == self.P0:
            old = count
            sh = (count - 1, ticket, turn, inside)
            if old > self.K or self.mutant == "always_bump":
                return sh, (self.P_BUMP, j, idx)
            return sh, (nxt, j + 1, 0)
        if pc == self.P_BUMP:
            return (count, ticket, turn + 1, inside), (nxt, j + 1, 0)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[3] > self.K:
            return f"occupancy {sh[3]} > K={self.K}"
        return None

    def final_check(self, sh, los):
        count, ticket, turn, _ = sh
        if count != 0 or ticket != turn:
            return f"final count={count} ticket={ticket} turn={turn}"
        if self.K >= self.n and ticket != 0:
            return f"an agent queued although K={self.K} >= {self.n} agents"
        return None


class CohortSemModel:
    """Algorithm 5 with per-XCD queues and local hand-over of units.

    count (global) counts workgroups inside or waiting, as in Algorithm 5.  wait:
    old = fetch-and-add(count, 1); old < K: enter with a fresh unit; otherwise draw a
    local ticket lt of one's own XCD's queue and poll grant slot lt mod Q of that queue
    until it holds lt + 1, with the number of local passes k of the unit it receives.
    post: c = load(count).  K = 1 and c > 1: the poster holds the only unit, so no other
    post lowers count before its own decrement, which is sure to find a waiter
    ("hand-over mode"): decrement count, then, if k + 1 < B and one's own XCD has an
    unserved ticket (claimed with a compare-and-swap on its served counter), grant it
    with k + 1 and no L2 writeback (both workgroups use the same L2); otherwise write the
    L2 back and grant the first XCD after one's own that has an unserved ticket, with
    k = 0.  Otherwise (and always for K >= 2): write back first, then decrement;
    old > K: grant a waiter of any XCD (preferring one's own); else the unit returns to
    the free count.
    Units: free (K - inside - waiting, when positive) + held + in transit = K throughout;
    the B bound sends every unit to another XCD after at most B local hand-overs.

    placement: XCD of each agent.  Data: one word updated in every critical section with
    a plain load and store through the agent's XCD's L2 (per XCD: empty, or (value,
    dirty)); a writeback copies a dirty value to memory; the waiter's acquire drops a
    clean copy.  With K = 1 the final value must count every admission.  A grant slot is
    reused (Q slots per XCD): a post writes a grant only into an empty slot, and the
    admitted waiter empties its slot as it takes the grant.
    small_q: Q = 1 slot per XCD (the reuse path on every grant).
    mutant 'no_remote_writeback': a hand-over to another XCD skips the writeback;
    mutant 'no_acquire': the admitted waiter does not invalidate;
    mutant 'claim_unchecked': a post claims the next local slot even when no ticket for
    it has been drawn;
    mutant 'predict_2k': hand-over mode for any K whenever the loaded count exceeds 2K
    (the other K - 1 units can change hands before the decrement lands, so the post may
    find no waiter left: reported as a deadlock)."""

    (W_CNT, W_LT, W_POLL, ACQ, CS_LD, CS_ST, P_PRED, P_DEC_H, P_LOCAL, P_WB_R, P_REMOTE,
     P_WB_S, P_DEC_S, P_ANY, P_GRANT, DONE) = range(16)

    def __init__(self, K: int, placement: tuple, ops: int = 2, B: int = 2,
                 mutant: str | None = None, small_q: bool = False):
        self.K, self.pl, self.ops, self.B, self.mutant = K, tuple(placement), ops, B, mutant
        self.n = len(self.pl)
        self.X = 1 + max(self.pl)
        self.Q = 1 if small_q else self.n

    # shared = (count, ltick, lserved, grant (X tuples of Q (ticket+1, k)), l2 (X), mem,
    #           inside)
    # local  = (pc, j, lt, k, tmp, gx, gs)
    def init(self):
        X, Q = self.X, self.Q
        sh = (0, (0,) * X, (0,) * X, tuple(((0, 0),) * Q for _ in range(X)), (None,) * X, 0, 0)
        return sh, tuple((self.W_CNT, 0, 0, 0, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(t, i, v):
        return t[:i] + (v,) + t[i + 1:]

    def _wb(self, l2, mem, x):
        if l2[x] is not None and l2[x][1]:
            return self._set(l2, x, (l2[x][0], False)), l2[x][0]
        return l2, mem

    def _claim(self, ltick, lserved, y):
        """Compare-and-swap claim of XCD y's next unserved ticket; None if none."""
        if lserved[y] < ltick[y] or self.mutant == "claim_unchecked":
            return self._set(lserved, y, lserved[y] + 1), lserved[y]
        return None

    def step(self, a, sh, lo):
        count, ltick, lserved, grant, l2, mem, inside = sh
        pc, j, lt, k, tmp, gx, gs = lo
        x, K, X, Q = self.pl[a], self.K, self.X, self.Q
        fin = self.W_CNT if j + 1 < self.ops else self.DONE

        def S(**kw):
            d = dict(count=count, ltick=ltick, lserved=lserved, grant=grant, l2=l2, mem=mem,
                     inside=inside)
            d.update(kw)
            return (d["count"], d["ltick"], d["lserved"], d["grant"], d["l2"], d["mem"],
                    d["inside"])

        if pc == self.W_CNT:
            if count < K:
                return S(count=count + 1), (self.ACQ, j, 0, 0, tmp, gx, gs)
            return S(count=count + 1), (self.W_LT, j, 0, 0, tmp, gx, gs)
        if pc == self.W_LT:
            return S(ltick=self._set(ltick, x, ltick[x] + 1)), (self.W_POLL, j, ltick[x], 0, tmp, gx, gs)
        if pc == self.W_POLL:  # take the grant and empty the slot in one step
            t1, kk = grant[x][lt % Q]
            if t1 == lt + 1:
                g = self._set(grant, x, self._set(grant[x], lt % Q, (0, 0)))
                return S(grant=g), (self.ACQ, j, lt, kk, tmp, gx, gs)
            return sh, lo
        if pc == self.ACQ:
            if self.mutant != "no_acquire" and l2[x] is not None and not l2[x][1]:
                l2 = self._set(l2, x, None)
            return S(l2=l2, inside=inside + 1), (self.CS_LD, j, lt, k, tmp, gx, gs)
        if pc == self.CS_LD:
            if l2[x] is None:
                l2 = self._set(l2, x, (mem, False))
            return S(l2=l2), (self.CS_ST, j, lt, k, l2[x][0], gx, gs)
        if pc == self.CS_ST:
            return S(l2=self._set(l2, x, (tmp + 1, True))), (self.P_PRED, j, lt, k, tmp, gx, gs)
        if pc == self.P_PRED:  # leaving the critical section; predict from count
            if self.mutant == "predict_2k":
                nxt = self.P_DEC_H if count > 2 * K else self.P_WB_S
            else:
                nxt = self.P_DEC_H if (K == 1 and count > 1) else self.P_WB_S
            return S(inside=inside - 1), (nxt, j, lt, k, tmp, gx, gs)
        if pc == self.P_DEC_H:
            nxt = self.P_LOCAL if k + 1 < self.B else self.P_WB_R
            return S(count=count - 1), (nxt, j, lt, k, tmp, gx, gs)
        if pc == self.P_LOCAL:
            c = self._claim(ltick, lserved, x)
            if c is None:
                return sh, (self.P_WB_R, j, lt, k, tmp, gx, gs)
            return S(lserved=c[0]), (self.P_GRANT, j, lt, k + 1, tmp, x, c[1])
        if pc == self.P_WB_R:
            if self.mutant != "no_remote_writeback":
                l2, mem = self._wb(l2, mem, x)
            return S(l2=l2, mem=mem), (self.P_REMOTE, j, lt, k, tmp, gx, gs)
        if pc in (self.P_REMOTE, self.P_ANY):
            first = x if (pc == self.P_ANY and k + 1 < self.B) else x + 1
            for y in [(first + d) % X for d in range(X)]:
                c = self._claim(ltick, lserved, y)
                if c is not None:
                    kk = k + 1 if (pc == self.P_ANY and y == x) else 0
                    return S(lserved=c[0]), (self.P_GRANT, j, lt, kk, tmp, y, c[1])
            return sh, lo  # the waiter that counted itself has not drawn its ticket yet
        if pc == self.P_WB_S:
            l2, mem = self._wb(l2, mem, x)
            return S(l2=l2, mem=mem), (self.P_DEC_S, j, lt, k, tmp, gx, gs)
        if pc == self.P_DEC_S:
            if count > K:
                return S(count=count - 1), (self.P_ANY, j, lt, k, tmp, gx, gs)
            return S(count=count - 1), (fin, j + 1, 0, 0, tmp, gx, gs)
        if pc == self.P_GRANT:  # once the slot's previous ticket has taken its grant
            if grant[gx][gs % Q][0] != 0:
                return sh, lo
            g = self._set(grant, gx, self._set(grant[gx], gs % Q, (gs + 1, k)))
            return S(grant=g), (fin, j + 1, 0, 0, tmp, gx, gs)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[6] > self.K:
            return f"occupancy {sh[6]} > K={self.K}"
        return None

    def final_check(self, sh, los):
        count, ltick, lserved, grant, l2, mem, inside = sh
        if count != 0 or inside != 0 or ltick != lserved:
            return f"final count={count} inside={inside} tickets={ltick} served={lserved}"
        if self.K == 1:
            total = self.n * self.ops
            vals = [e[0] for e in l2 if e is not None and e[1]]
            final = vals[0] if vals else mem
            if final != total:
                return f"lost update: data {final} != {total}"
        return None


class ArraySemModel:
    """Two monotone counters with a grant slot per ticket (the array semaphore).

    tickets, posts and the M grant slots start at 0.  wait: t = fetch-and-add(tickets,
    1); t < K: enter; otherwise poll slot t mod M until it holds at least t + 1.  post:
    write the L2 back, p = fetch-and-add(posts, 1), then raise slot (p + K) mod M to
    p + K + 1 with an atomic maximum.  The admission rule is the two-counter one (enter
    once posts + K > t); the slots only tell each waiter when.  M below the number of
    tickets makes several tickets share a slot, and grants for one slot may land in any
    order.

    placement: XCD of each agent.  Data as in CohortSemModel: one word updated in every
    critical section with a plain load and store through the agent's XCD's L2 (per XCD:
    empty, or (value, dirty)); a writeback copies a dirty value to memory; the admitted
    waiter's acquire drops a clean copy.  With K = 1 every load must see every earlier
    update and the final value must count every admission.
    mutant 'enter_at_k': tickets t <= K enter at once (an off-by-one);
    mutant 'poll_eq': the waiter enters only on exactly t + 1 (a later grant of the same
    slot hides its own);
    mutant 'grant_next': the post grants ticket p + K + 1;
    mutant 'store': the grant is a plain store (a late earlier grant can lower a slot);
    mutant 'no_writeback': the post skips the writeback;
    mutant 'no_acquire': the admitted waiter does not invalidate.

    rule 'chain' (the chain semaphore): the post keeps the ticket t its own wait drew,
    counts itself in posts, and stores t + K + 1 into slot (t + K) mod M -- a plain
    store, correct when M is a multiple of K (with any other M a later chain's store can
    admit a waiter early: the bound breaks)."""

    W_TICKET, W_POLL, ACQ, CS_LD, CS_ST, P_WB, P_DRAW, P_GRANT, DONE = range(9)

    def __init__(self, K: int, placement: tuple, M: int, ops: int = 2,
                 mutant: str | None = None, rule: str = "posts"):
        self.K, self.pl, self.M, self.ops, self.mutant = K, tuple(placement), M, ops, mutant
        self.rule = rule
        self.n = len(self.pl)
        self.X = 1 + max(self.pl)

    # shared = (tickets, posts, slots (M), l2 (X), mem, inside, done_cs)
    # local  = (pc, j, t, tmp)
    def init(self):
        sh = (0, 0, (0,) * self.M, (None,) * self.X, 0, 0, 0)
        return sh, tuple((self.W_TICKET, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(t, i, v):
        return t[:i] + (v,) + t[i + 1:]

    def step(self, a, sh, lo):
        tickets, posts, slots, l2, mem, inside, done_cs = sh
        pc, j, t, tmp = lo
        x = self.pl[a]
        if pc == self.W_TICKET:
            t = tickets
            go = t <= self.K if self.mutant == "enter_at_k" else t < self.K
            return ((tickets + 1, posts, slots, l2, mem, inside, done_cs),
                    (self.ACQ if go else self.W_POLL, j, t, 0))
        if pc == self.W_POLL:
            v = slots[t % self.M]
            go = v == t + 1 if self.mutant == "poll_eq" else v >= t + 1
            return sh, (self.ACQ if go else self.W_POLL, j, t, 0)
        if pc == self.ACQ:
            if self.mutant != "no_acquire" and l2[x] is not None and not l2[x][1]:
                l2 = self._set(l2, x, None)
            return (tickets, posts, slots, l2, mem, inside + 1, done_cs), (self.CS_LD, j, t, 0)
        if pc == self.CS_LD:
            if l2[x] is None:
                l2 = self._set(l2, x, (mem, False))
            return (tickets, posts, slots, l2, mem, inside, done_cs), (self.CS_ST, j, t, l2[x][0])
        if pc == self.CS_ST:
            if self.K == 1 and tmp != done_cs:
                # a stale load: report it through the occupancy check's channel
                inside = self.K + 100
            l2 = self._set(l2, x, (tmp + 1, True))
            return ((tickets, posts, slots, l2, mem, inside - 1, done_cs + 1),
                    (self.P_WB, j, t, 0))
        if pc == self.P_WB:
            if self.mutant != "no_writeback" and l2[x] is not None and l2[x][1]:
                mem = l2[x][0]
                l2 = self._set(l2, x, (mem, False))
            return (tickets, posts, slots, l2, mem, inside, done_cs), (self.P_DRAW, j, t, 0)
        if pc == self.P_DRAW:
            q = (t if self.rule == "chain" else posts) + self.K
            q += 1 if self.mutant == "grant_next" else 0
            return ((tickets, posts + 1, slots, l2, mem, inside, done_cs),
                    (self.P_GRANT, j, t, q))
        if pc == self.P_GRANT:
            i = tmp % self.M
            plain = self.mutant == "store" or self.rule == "chain"
            v = tmp + 1 if plain else max(slots[i], tmp + 1)
            nxt = self.W_TICKET if j + 1 < self.ops else self.DONE
            return ((tickets, posts, self._set(slots, i, v), l2, mem, inside, done_cs),
                    (nxt, j + 1, 0, 0))
        raise AssertionError(pc)

    def check(self, sh, los):
        inside = sh[5]
        if inside > self.K + 50:
            return "a holder loaded the data word without an earlier holder's update"
        if inside > self.K:
            return f"occupancy {inside} > K={self.K}"
        return None

    def final_check(self, sh, los):
        tickets, posts, slots, l2, mem, inside, done_cs = sh
        total = self.n * self.ops
        if tickets != total or posts != total or inside != 0:
            return f"final tickets={tickets} posts={posts} inside={inside}"
        if self.K == 1 and mem != total:
            return f"final data {mem} != {total} admissions"
        return None


class CuCohortLockModel:
    """CU-cohort lock, with caches: a ticket lock per CU group in front of the XCD-cohort
    lock (a ticket lock per XCD in front of a global ticket lock); one lock, one data word.

    placement: per agent (xcd, cu), CU ids global; the group of an agent is its CU.  Each
    group has a ticket counter, an announcement word (the count of tickets drawn as the
    last announcer saw it: drawing and announcing are separate steps, so announcements can
    lag and land out of order), a grant (turn, session) and a record of the XCD lock its
    session holds (local ticket, session); each XCD a local ticket counter and a grant
    (turn, session); the global lock a ticket and a turn.  Lock: draw and announce a group
    ticket, wait for its grant; session k > 0: read the record and enter with no cache
    maintenance; session 0: take the XCD lock (and the global one when the XCD grant says
    session 0), acquire (the CU's L1 and the XCD's clean L2 lines dropped), write the
    record.  Unlock: when an announcement shows a later group ticket and k + 1 < B, grant
    (turn + 1, k + 1) within the group; else hand the XCD lock on (within the XCD when a
    later local ticket was drawn and its session may grow, without a writeback; else write
    the XCD's L2 back and advance the global turn), then grant (turn + 1, 0).  Caches: an
    L1 per CU, shared by the CU's agents (a load goes L1 -> L2 -> memory, a store updates
    the CU's L1 and dirties the XCD's L2), an L2 per XCD.
    mutant 'no_acquire': the holder that took the XCD lock keeps its caches;
    mutant 'group_by_xcd': the groups are the XCDs (a CU id read wrongly), so a pass
    within a group can cross CUs without an acquire;
    mutant 'no_waiter_check': pass within the group with no later ticket announced."""

    (DRAW_C, ANN, POLL_C, DRAW_X, POLL_X, DRAW_G, POLL_G, ACQ, CS_LD, CS_ST, REL,
     DONE) = range(12)

    def __init__(self, placement: tuple, ops: int = 2, B: int = 2, mutant: str | None = None):
        self.pl, self.ops, self.B, self.mutant = tuple(placement), ops, B, mutant
        self.n = len(self.pl)
        self.X = 1 + max(x for x, _ in self.pl)
        self.NC = 1 + max(c for _, c in self.pl)
        self.grp = tuple((x if mutant == "group_by_xcd" else c) for x, c in self.pl)
        self.NG = 1 + max(max(self.grp), self.NC - 1)

    # shared = (gt, gturn, xt (X), xg (X of (turn, session)), ct (NG), ann (NG),
    #           cg (NG of (turn, session)), rec (NG of (ticket, session)),
    #           l1 (NC: value or None), l2 (X: (value, dirty) or None), mem,
    #           inside, done_cs, bad)
    # local  = (pc, j, tc, kc, tx, kx, tmp)
    def init(self):
        X, NG, NC = self.X, self.NG, self.NC
        sh = (0, 0, (0,) * X, ((0, 0),) * X, (0,) * NG, (0,) * NG, ((0, 0),) * NG,
              ((0, 0),) * NG, (None,) * NC, (None,) * X, 0, 0, 0, None)
        return sh, tuple((self.DRAW_C, 0, 0, 0, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(t, i, v):
        return t[:i] + (v,) + t[i + 1:]

    def step(self, a, sh, lo):
        gt, gturn, xt, xg, ct, ann, cg, rec, l1, l2, mem, inside, done_cs, bad = sh
        pc, j, tc, kc, tx, kx, tmp = lo
        x, cu = self.pl[a]
        g = self.grp[a]
        S = self._set

        def out(pc2, **kw):
            v = dict(gt=gt, gturn=gturn, xt=xt, xg=xg, ct=ct, ann=ann, cg=cg, rec=rec, l1=l1,
                     l2=l2, mem=mem, inside=inside, done_cs=done_cs, bad=bad, tc=tc, kc=kc,
                     tx=tx, kx=kx, tmp=tmp, j=j)
            v.update(kw)
            return ((v["gt"], v["gturn"], v["xt"], v["xg"], v["ct"], v["ann"], v["cg"],
                     v["rec"], v["l1"], v["l2"], v["mem"], v["inside"], v["done_cs"], v["bad"]),
                    (pc2, v["j"], v["tc"], v["kc"], v["tx"], v["kx"], v["tmp"]))

        if pc == self.DRAW_C:
            return out(self.ANN, ct=S(ct, g, ct[g] + 1), tc=ct[g])
        if pc == self.ANN:
            return out(self.POLL_C, ann=S(ann, g, tc + 1))
        if pc == self.POLL_C:
            turn, sess = cg[g]
            if turn != tc:
                return sh, lo
            if sess > 0:
                rt, rk = rec[g]
                return out(self.CS_LD, kc=sess, tx=rt, kx=rk)
            return out(self.DRAW_X, kc=0)
        if pc == self.DRAW_X:
            return out(self.POLL_X, xt=S(xt, x, xt[x] + 1), tx=xt[x])
        if pc == self.POLL_X:
            turn, sess = xg[x]
            if turn != tx:
                return sh, lo
            return out(self.ACQ if sess > 0 else self.DRAW_G, kx=sess)
        if pc == self.DRAW_G:
            return out(self.POLL_G, gt=gt + 1, tmp=gt)
        if pc == self.POLL_G:
            return out(self.ACQ) if gturn == tmp else (sh, lo)
        if pc == self.ACQ:
            if self.mutant != "no_acquire":
                l1 = S(l1, cu, None)
                l2 = S(l2, x, l2[x] if l2[x] is not None and l2[x][1] else None)
            return out(self.CS_LD, l1=l1, l2=l2, rec=S(rec, g, (tx, kx)))
        if pc == self.CS_LD:
            v = l1[cu]
            if v is None:
                if l2[x] is None:
                    l2 = S(l2, x, (mem, False))
                v = l2[x][0]
                l1 = S(l1, cu, v)
            return out(self.CS_ST, l1=l1, l2=l2, tmp=v, inside=inside + 1)
        if pc == self.CS_ST:
            if inside > 1:
                bad = bad or "two holders inside"
            elif tmp != done_cs:
                bad = bad or f"stale read: {tmp} after {done_cs} sections"
            return out(self.REL, l1=S(l1, cu, tmp + 1), l2=S(l2, x, (tmp + 1, True)),
                       inside=inside - 1, done_cs=done_cs + 1, bad=bad)
        if pc == self.REL:
            waiter = ann[g] > tc + 1 or self.mutant == "no_waiter_check"
            nxt = self.DRAW_C if j + 1 < self.ops else self.DONE
            if waiter and kc + 1 < self.B:
                return out(nxt, cg=S(cg, g, (tc + 1, kc + 1)), j=j + 1)
            if xt[x] > tx + 1 and kx + 1 < self.B:
                xg = S(xg, x, (tx + 1, kx + 1))
            else:
                if l2[x] is not None and l2[x][1]:
                    mem = l2[x][0]
                    l2 = S(l2, x, (mem, False))
                gturn = gturn + 1
                xg = S(xg, x, (tx + 1, 0))
            return out(nxt, xg=xg, l2=l2, mem=mem, gturn=gturn, cg=S(cg, g, (tc + 1, 0)), j=j + 1)
        raise AssertionError(pc)

    def check(self, sh, los):
        return sh[13]

    def final_check(self, sh, los):
        gt, gturn, xt, xg, ct, ann, cg = sh[:7]
        if sh[12] != self.n * self.ops:
            return f"{sh[12]} sections of {self.n * self.ops}"
        if gturn != gt or any(xg[x][0] != xt[x] for x in range(self.X)) or \
                any(cg[i][0] != ct[i] for i in range(self.NG)):
            return "a lock level not released at the end"
        return None


class XcdChainSemModel:
    """The chain semaphore with its units split over per-XCD queues.

    Queue q (agent a uses queue placement[a] mod Q) owns K_q = K / Q units (the first
    K mod Q queues one more) and runs the chain rule alone: tickets drawn per queue,
    ticket t >= K_q waits for slot t mod M_q to hold t + 1, which the holder of ticket
    t - K_q stores when it posts (M_q a multiple of K_q).  Each queue guards a data word
    of its own (with K_q = 1 its holders exclude each other).  Caches: a per-agent L1
    (clean copies; each agent runs on a CU of its own) and a per-XCD L2 ((value, dirty));
    a load goes L1 -> L2 -> memory, a store writes through the L1 into the L2 (dirty); the
    admitted waiter's acquire drops its L1 and its XCD's clean L2 lines; a writeback
    copies the XCD's dirty lines to memory.  The post skips the writeback when every
    queue holds one XCD's agents (Q >= number of XCDs), since the chain's next holder
    reads through the same L2; otherwise it writes back.
    mutant 'skip_when_shared': the post skips the writeback although XCDs share a queue;
    mutant 'no_acquire': the admitted waiter keeps its L1;
    mutant 'enter_at_k': tickets t <= K_q enter at once."""

    W_TICKET, W_POLL, ACQ, CS_LD, CS_ST, P_WB, P_GRANT, DONE = range(8)

    def __init__(self, K: int, placement: tuple, Q: int, M: int = 2, ops: int = 2,
                 mutant: str | None = None):
        self.K, self.pl, self.Q, self.ops, self.mutant = K, tuple(placement), Q, ops, mutant
        self.n = len(self.pl)
        self.X = 1 + max(self.pl)
        self.Kq = tuple(K // Q + (1 if q < K % Q else 0) for q in range(Q))
        assert min(self.Kq) >= 1
        self.Mq = tuple(max(1, M // k) * k for k in self.Kq)
        self.local = Q >= self.X

    # shared = (tickets (Q), slots (Q x M_q), l1 (n x Q: value or None),
    #           l2 (X x Q: (value, dirty) or None), mem (Q), inside (Q), done_cs (Q))
    # local  = (pc, j, t, tmp)
    def init(self):
        Q, X, n = self.Q, self.X, self.n
        sh = ((0,) * Q, tuple((0,) * self.Mq[q] for q in range(Q)),
              tuple((None,) * Q for _ in range(n)), tuple((None,) * Q for _ in range(X)),
              (0,) * Q, (0,) * Q, (0,) * Q)
        return sh, tuple((self.W_TICKET, 0, 0, 0) for _ in range(n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(t, i, v):
        return t[:i] + (v,) + t[i + 1:]

    def step(self, a, sh, lo):
        tickets, slots, l1, l2, mem, inside, done_cs = sh
        pc, j, t, tmp = lo
        x, q = self.pl[a], self.pl[a] % self.Q
        kq, mq = self.Kq[q], self.Mq[q]
        if pc == self.W_TICKET:
            t = tickets[q]
            go = t <= kq if self.mutant == "enter_at_k" else t < kq
            return ((self._set(tickets, q, t + 1), slots, l1, l2, mem, inside, done_cs),
                    (self.ACQ if go else self.W_POLL, j, t, 0))
        if pc == self.W_POLL:
            return sh, (self.ACQ if slots[q][t % mq] >= t + 1 else self.W_POLL, j, t, 0)
        if pc == self.ACQ:
            if self.mutant != "no_acquire":
                l1 = self._set(l1, a, (None,) * self.Q)
                l2 = self._set(l2, x, tuple(e if e is not None and e[1] else None for e in l2[x]))
            return ((tickets, slots, l1, l2, mem, self._set(inside, q, inside[q] + 1), done_cs),
                    (self.CS_LD, j, t, 0))
        if pc == self.CS_LD:
            v = l1[a][q]
            if v is None:
                if l2[x][q] is None:
                    l2 = self._set(l2, x, self._set(l2[x], q, (mem[q], False)))
                v = l2[x][q][0]
                l1 = self._set(l1, a, self._set(l1[a], q, v))
            return (tickets, slots, l1, l2, mem, inside, done_cs), (self.CS_ST, j, t, v)
        if pc == self.CS_ST:
            if kq == 1 and tmp != done_cs[q]:
                inside = self._set(inside, q, kq + 100)  # reported by check()
            l1 = self._set(l1, a, self._set(l1[a], q, tmp + 1))
            l2 = self._set(l2, x, self._set(l2[x], q, (tmp + 1, True)))
            return ((tickets, slots, l1, l2, mem, self._set(inside, q, inside[q] - 1),
                     self._set(done_cs, q, done_cs[q] + 1)), (self.P_WB, j, t, 0))
        if pc == self.P_WB:
            skip = self.local or self.mutant == "skip_when_shared"
            if not skip:
                m = list(mem)
                for i, e in enumerate(l2[x]):
                    if e is not None and e[1]:
                        m[i] = e[0]
                mem = tuple(m)
                l2 = self._set(l2, x, tuple(None if e is None else (e[0], False) for e in l2[x]))
            return (tickets, slots, l1, l2, mem, inside, done_cs), (self.P_GRANT, j, t, 0)
        if pc == self.P_GRANT:
            g = t + kq
            slots = self._set(slots, q, self._set(slots[q], g % mq, g + 1))
            nxt = self.W_TICKET if j + 1 < self.ops else self.DONE
            return (tickets, slots, l1, l2, mem, inside, done_cs), (nxt, j + 1, 0, 0)
        raise AssertionError(pc)

    def check(self, sh, los):
        inside = sh[5]
        for q in range(self.Q):
            if inside[q] > self.Kq[q] + 50:
                return "a holder loaded its queue's word without an earlier holder's update"
            if inside[q] > self.Kq[q]:
                return f"occupancy {inside[q]} > K_q={self.Kq[q]} in queue {q}"
        if sum(inside) > self.K:
            return f"occupancy {sum(inside)} > K={self.K}"
        return None

    def final_check(self, sh, los):
        tickets, slots, l1, l2, mem, inside, done_cs = sh
        for q in range(self.Q):
            want = self.ops * sum(1 for p in self.pl if p % self.Q == q)
            if tickets[q] != want or done_cs[q] != want or inside[q] != 0:
                return f"queue {q}: tickets {tickets[q]} done {done_cs[q]} != {want}"
        return None


class WeightedSemModel:
    """Fetch-and-add semaphore with weighted requests, the admission rule of the serving
    queue (Algorithm 5 with u tickets drawn at once).  issued and released start at 0.
    wait(u): end = fetch-and-add(issued, u) + u; poll until released + K >= end.
    post(u): fetch-and-add(released, u).
    Agent a asks for weights[a] units on each of its `ops` requests.
    mutant 'ignore_weight': admit once released + K >= end - u (the first ticket only).
    mutant 'strict': admit once released + K > end.
    mutant 'post_one': post returns one unit instead of u."""

    W_TICKET, W_POLL, CS_IN, CS_OUT, POST, DONE = range(6)

    def __init__(self, K: int, weights: tuple, ops: int = 2, mutant: str | None = None):
        self.K, self.weights, self.n, self.ops, self.mutant = K, tuple(weights), len(weights), ops, mutant

    def init(self):
        return (0, 0, 0), tuple((self.W_TICKET, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    def _admit(self, released, end, u):
        if self.mutant == "ignore_weight":
            return released + self.K >= end - u
        if self.mutant == "strict":
            return released + self.K > end
        return released + self.K >= end

    def step(self, a, sh, lo):
        issued, released, inside = sh
        pc, j, end = lo
        u = self.weights[a]
        if pc == self.W_TICKET:
            return (issued + u, released, inside), (self.W_POLL, j, issued + u)
        if pc == self.W_POLL:
            return sh, ((self.CS_IN if self._admit(released, end, u) else self.W_POLL), j, end)
        if pc == self.CS_IN:
            return (issued, released, inside + u), (self.CS_OUT, j, end)
        if pc == self.CS_OUT:
            return (issued, released, inside - u), (self.POST, j, end)
        if pc == self.POST:
            back = 1 if self.mutant == "post_one" else u
            nxt = self.W_TICKET if j + 1 < self.ops else self.DONE
            return (issued, released + back, inside), (nxt, j + 1, 0)
        raise AssertionError(pc)

    def check(self, sh, los):
        issued, released, inside = sh
        if inside > self.K:
            return f"units in use {inside} > K={self.K}"
        # FIFO: while a waiter cannot be admitted, nobody with a later ticket is inside
        for lo in los:
            if lo[0] == self.W_POLL and not released + self.K >= lo[2]:
                for lo2 in los:
                    if lo2[0] in (self.CS_IN, self.CS_OUT) and lo2[2] > lo[2]:
                        return "a later ticket was admitted before an earlier one"
        return None

    def final_check(self, sh, los):
        issued, released, inside = sh
        total = self.ops * sum(self.weights)
        if issued != total or released != total or inside != 0:
            return f"final issued={issued} released={released} inside={inside}"
        return None


# ------------------------------------------------------------------------------------
# Barriers running the hash-exchange workload: in round r agent b stores the round
# number into slot[r & 1][b], passes the barrier, then reads slot[r & 1][(b + r) % N],
# which must hold r (published by that agent in this round and not yet overwritten).
# Counters and flags are monotone (compared with >=), never reset.
# ------------------------------------------------------------------------------------

class BarrierModel:
    """kind: 'central' -- one counter; an agent arrives with fetch-and-add and waits
                          until the counter reaches N * (r + 1);
             'split'   -- the same counter; the agent whose fetch-and-add returns
                          N * (r + 1) - 1 (the last arriver) stores r + 1 into a separate
                          release word, which the others poll;
             'tree'    -- agents split into G groups (b mod G); the last arriver of a
                          group adds one to a top counter; the last group publishes a
                          top generation word; each group's last arriver copies it into
                          its group's generation word, which the others poll;
             'flag'    -- decentralized: agent b stores r + 1 into arrive[b]; agent 0
                          (master) waits for every arrive flag, then stores r + 1 into
                          every release flag; the others poll their release flag.
       mutant: 'single_buffer' -- one slot array for every round;
               'no_wait'       -- arrive but never wait (central, split, flag);
               'split_off_by_one' -- split: the agent that sees N * (r + 1) - 2 publishes;
               'no_top_wait'   -- tree: a group's last arriver releases its group without
                                  waiting for the other groups."""

    WRITE, ARRIVE, POLL, TOP, TOP_POLL, TOP_REL, GROUP_REL, SCAN, RELEASE, READ, DONE = range(11)

    def __init__(self, kind: str, n: int = 3, rounds: int = 3, groups: int = 2,
                 mutant: str | None = None):
        self.kind, self.n, self.R, self.mutant = kind, n, rounds, mutant
        self.G = min(groups, n)
        self.members = [sum(1 for b in range(n) if b % self.G == g) for g in range(self.G)]

    # shared = (slots (2N tuple), cnt, gcnt (G), ggen (G), top, topgen, arrive (N), release (N))
    def init(self):
        N, G = self.n, self.G
        sh = ((-1,) * (2 * N), 0, (0,) * G, (0,) * G, 0, 0, (0,) * N, (0,) * N)
        return sh, tuple((self.WRITE, 0, 0, 0) for _ in range(N))  # (pc, r, i, bad)

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(t, i, v):
        return t[:i] + (v,) + t[i + 1:]

    def _slot(self, r, b):
        return (0 if self.mutant == "single_buffer" else (r & 1)) * self.n + b

    def step(self, a, sh, lo):
        slots, cnt, gcnt, ggen, top, topgen, arrive, release = sh
        pc, r, i, bad = lo
        N, G, stamp = self.n, self.G, r + 1
        if pc == self.WRITE:
            slots = self._set(slots, self._slot(r, a), r)
            return (slots, cnt, gcnt, ggen, top, topgen, arrive, release), (self.ARRIVE, r, 0, bad)
        if pc == self.ARRIVE:
            if self.kind == "central":
                sh = (slots, cnt + 1, gcnt, ggen, top, topgen, arrive, release)
                return sh, (self.READ if self.mutant == "no_wait" else self.POLL, r, 0, bad)
            if self.kind == "split":
                old = cnt
                sh = (slots, cnt + 1, gcnt, ggen, top, topgen, arrive, release)
                last = N * stamp - (2 if self.mutant == "split_off_by_one" else 1)
                if old == last:
                    return sh, (self.TOP_REL, r, 0, bad)
                return sh, (self.READ if self.mutant == "no_wait" else self.POLL, r, 0, bad)
            if self.kind == "tree":
                g = a % G
                old = gcnt[g]
                sh = (slots, cnt, self._set(gcnt, g, old + 1), ggen, top, topgen, arrive, release)
                last = old == self.members[g] * stamp - 1
                return sh, ((self.TOP if last else self.POLL), r, 0, bad)
            arrive = self._set(arrive, a, stamp)
            sh = (slots, cnt, gcnt, ggen, top, topgen, arrive, release)
            if self.mutant == "no_wait":
                return sh, (self.READ, r, 0, bad)
            return sh, ((self.SCAN if a == 0 else self.POLL), r, 0, bad)
        if pc == self.POLL:
            if self.kind == "central":
                ok = cnt >= N * stamp
            elif self.kind == "split":
                ok = topgen >= stamp
            elif self.kind == "tree":
                ok = ggen[a % G] >= stamp
            else:
                ok = release[a] >= stamp
            return sh, ((self.READ if ok else self.POLL), r, i, bad)
        if pc == self.TOP:  # tree: last of the group arrives at the top counter
            t = top
            sh = (slots, cnt, gcnt, ggen, top + 1, topgen, arrive, release)
            if self.mutant == "no_top_wait":
                return sh, (self.GROUP_REL, r, 0, bad)
            return sh, ((self.TOP_REL if t == G * stamp - 1 else self.TOP_POLL), r, 0, bad)
        if pc == self.TOP_POLL:
            return sh, ((self.GROUP_REL if topgen >= stamp else self.TOP_POLL), r, 0, bad)
        if pc == self.TOP_REL:
            sh = (slots, cnt, gcnt, ggen, top, stamp, arrive, release)
            return sh, ((self.READ if self.kind == "split" else self.GROUP_REL), r, 0, bad)
        if pc == self.GROUP_REL:
            ggen = self._set(ggen, a % G, stamp)
            return (slots, cnt, gcnt, ggen, top, topgen, arrive, release), (self.READ, r, 0, bad)
        if pc == self.SCAN:  # flag master: wait for arrive[i], i = 0 .. N-1
            if arrive[i] >= stamp:
                return sh, ((self.SCAN if i + 1 < N else self.RELEASE), r, (i + 1) % N, bad)
            return sh, lo
        if pc == self.RELEASE:
            release = self._set(release, i, stamp)
            sh = (slots, cnt, gcnt, ggen, top, topgen, arrive, release)
            return sh, ((self.RELEASE if i + 1 < N else self.READ), r, (i + 1) % N, bad)
        if pc == self.READ:
            v = slots[self._slot(r, (a + r) % N)]
            bad = bad or (v != r)
            return sh, ((self.WRITE if r + 1 < self.R else self.DONE), r + 1, 0, bad)
        raise AssertionError(pc)

    def check(self, sh, los):
        for b, (pc, r, i, bad) in enumerate(los):
            if bad:
                return f"phase violated: agent {b} read stale or overwritten data"
        return None

    def final_check(self, sh, los):
        return None


# ------------------------------------------------------------------------------------
# The per-XCD barrier as the library runs it, with the caches it has to maintain.
#
# Memory model of the data (the exchanged slots; every flag, stamp and counter is an
# agent-scope atomic and is modelled as a plain shared variable under sequential
# consistency).  All 2N slots share one cache line, so a read fills every slot:
#   * each CU has an L1 holding the whole line or nothing; a load hits it if present,
#     otherwise fills it from its XCD's L2;
#   * each XCD has an L2 holding, per slot, nothing or (value, dirty); a load or a store
#     that misses fills the missing slots from memory (write-allocate); a store marks its
#     slot dirty and updates the storing CU's L1 copy, not the other CUs' copies;
#   * a release (L2 writeback) copies the XCD's dirty slots to memory and marks them
#     clean; with l2_coherent it also drops those slots from every other XCD's L2 (the
#     L2s are then kept coherent by the hardware), otherwise other L2s keep stale copies;
#   * an agent-scope acquire empties the CU's L1 and drops the clean slots of its XCD's
#     L2; a workgroup-scope invalidate empties the CU's L1 only;
#   * a plain store is issued first and completes into the L2 in a later step: the wait
#     for outstanding stores is the agent's own step sequence.
# ------------------------------------------------------------------------------------

class XcdBarrierModel:
    """Per-XCD barrier, hash-exchange workload (round r: agent a stores r into slot
    (r & 1, a), passes the barrier, reads slot (r & 1, (a + r) mod n), which must hold r).

    placement: per agent (xcd, cu); CU ids are global.  Registration: member k of an XCD
    in agent order (k = 0 is the XCD's master), CU leader = first agent of its CU, rank of
    a CU = order of its first agent among its XCD's CUs.  With register=True, round 0
    computes these with fetch-and-adds exactly as the library does (XCD count, CU count,
    CU rank of each CU's first agent), then passes a fenced counter barrier (release,
    arrive, poll, acquire) and reads the registration; an XCD with more than `block`
    members or more than `cu_lines` CUs makes every agent fall back to the counter barrier
    in the later rounds.

    Later rounds, mode 'plain' (data with plain accesses; coherent_cs = 0):
      members: the slot store completes, then the arrival flag is stored;
      the master: the store completes, it scans its members' flags, writes its XCD's L2
        back, publishes its XCD's stamp into each of `copies` copies;
      CU leaders: poll the populated XCDs' stamps in copy (x + X * rank) mod copies,
        acquire for the CU, store the CU's release line;
      other agents: poll their CU's release line.
    mode 'l1only': as 'plain', but every agent polls the stamps and invalidates its CU's
      L1 only (no release line).
    mode 'coherent': slots are stored and loaded with atomics (no caches); every agent
      polls the stamps; no writeback, no acquire.

    mutant: 'early_publish' -- the master skips its last member's flag;
            'early_release' -- a CU leader polls only its own XCD's stamp;
            'skip_copy'     -- XCD 0's master does not write the last copy;
            'no_writeback'  -- masters do not write the L2 back;
            'no_invalidate' -- CU leaders do not acquire;
            'no_cu_wait'    -- agents that are not CU leaders poll the stamps themselves and
                               read without their CU's invalidation;
            'flag_before_store' -- a member stores its arrival flag before its slot store
                               has completed into the L2;
            'rank_after_arrival' -- (register=True) a CU's first agent stores its CU's rank
                               after arriving at the registration barrier, so another agent
                               of the CU can read the rank before it is written (and poll
                               another CU's release line).
    The release lines are indexed by (XCD, rank of the CU), as in the library.  Flags are
    words every reader sees once stored; for the release line, which only its CU's agents
    read, that holds at workgroup scope too (they share the CU's L1), which is how the
    library stores and polls it."""

    (WRITE, COMPLETE, ARRIVE, SCAN, WB, PUB, POLL, ACQ, REL, WAIT_REL, INV_L1, READ,
     REG_X, REG_CU, REG_RANK, REG_RANKST, REG_WB, REG_ARRIVE, REG_POLL, REG_ACQ, REG_READ,
     FB_WB, FB_ARRIVE, FB_POLL, FB_ACQ, LATE, DONE) = range(27)

    def __init__(self, placement, rounds: int = 3, copies: int = 2, mode: str = "plain",
                 register: bool = False, block: int = 8, cu_lines: int = 8,
                 l2_coherent: bool = False, mutant: str | None = None):
        self.pl = tuple(placement)
        self.n = len(self.pl)
        self.R, self.C, self.mode, self.register = rounds, copies, mode, register
        self.block, self.cu_lines, self.l2c, self.mutant = block, cu_lines, l2_coherent, mutant
        self.X = 1 + max(x for x, _ in self.pl)
        self.ncu = 1 + max(c for _, c in self.pl)
        # static registration (also what register=True must reproduce when it fits)
        self.k, self.slot, self.rank = [], [], []
        ranks, cus_of = {}, {}
        for a, (x, c) in enumerate(self.pl):
            self.k.append(sum(1 for b in range(a) if self.pl[b][0] == x))
            self.slot.append(sum(1 for b in range(a) if self.pl[b][1] == c))
            if c not in ranks:
                ranks[c] = cus_of.get(x, 0)
                cus_of[x] = ranks[c] + 1
            self.rank.append(ranks[c])
        self.members = [sum(1 for x2, _ in self.pl if x2 == x) for x in range(self.X)]
        self.xmask = tuple(x for x in range(self.X) if self.members[x])

    # shared = (mem, l1, l2, arrive, mail, rel, reg) where reg = (xcount, cucount, xcu,
    #          curank, overflow, cnt)
    # local  = (pc, r, i, bad, pend, k, slot, rank, use)
    def init(self):
        S = 2 * self.n
        reg = ((0,) * self.X, (0,) * self.ncu, (0,) * self.X, (0,) * self.ncu, 0, 0)
        sh = ((-1,) * S, (None,) * self.ncu, (None,) * self.X, (0,) * self.n,
              tuple((0,) * self.X for _ in range(self.C)), (0,) * (self.X * self.cu_lines), reg)
        los = []
        for a in range(self.n):
            if self.register:
                los.append((self.WRITE, 0, 0, False, None, -1, -1, -1, True))
            else:
                los.append((self.WRITE, 0, 0, False, None, self.k[a], self.slot[a],
                            self.rank[a], True))
        return sh, tuple(los)

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(t, i, v):
        return t[:i] + (v,) + t[i + 1:]

    # ---- caches --------------------------------------------------------------------
    def _fill(self, mem, line2):
        return tuple((mem[j], False) if line2 is None or line2[j] is None else line2[j]
                     for j in range(len(mem)))

    def _load(self, sh, a, i):
        mem, l1, l2 = sh[0], sh[1], sh[2]
        x, c = self.pl[a]
        if self.mode == "coherent":
            return sh, mem[i]
        if l1[c] is not None:
            return sh, l1[c][i]
        line2 = self._fill(mem, l2[x])
        vals = tuple(v for v, _ in line2)
        sh = (mem, self._set(l1, c, vals), self._set(l2, x, line2)) + sh[3:]
        return sh, vals[i]

    def _store_complete(self, sh, a, i, v):
        mem, l1, l2 = sh[0], sh[1], sh[2]
        x, c = self.pl[a]
        line2 = self._set(self._fill(mem, l2[x]), i, (v, True))
        if l1[c] is not None:
            l1 = self._set(l1, c, self._set(l1[c], i, v))
        return (mem, l1, self._set(l2, x, line2)) + sh[3:]

    def _writeback(self, sh, x):
        mem, l1, l2 = sh[0], sh[1], sh[2]
        line2 = l2[x]
        if line2 is None:
            return sh
        dirty = [j for j, e in enumerate(line2) if e is not None and e[1]]
        for j in dirty:
            mem = self._set(mem, j, line2[j][0])
        l2 = self._set(l2, x, tuple(None if e is None else (e[0], False) for e in line2))
        if self.l2c:
            for y in range(self.X):
                if y != x and l2[y] is not None:
                    l2 = self._set(l2, y, tuple(None if j in dirty else e
                                                for j, e in enumerate(l2[y])))
        return (mem, l1, l2) + sh[3:]

    def _acquire(self, sh, a):
        mem, l1, l2 = sh[0], sh[1], sh[2]
        x, c = self.pl[a]
        l1 = self._set(l1, c, None)
        if l2[x] is not None:
            l2 = self._set(l2, x, tuple(e if e is not None and e[1] else None for e in l2[x]))
        return (mem, l1, l2) + sh[3:]

    def _inv_l1(self, sh, a):
        return (sh[0], self._set(sh[1], self.pl[a][1], None)) + sh[2:]

    # ---- protocol ----------------------------------------------------------------------
    def _slot_index(self, r, b):
        return (r & 1) * self.n + b

    def _scan_list(self, a):
        x = self.pl[a][0]
        mem = [b for b in range(self.n) if self.pl[b][0] == x and b != a]
        if self.mutant == "early_publish" and mem:
            mem = mem[:-1]
        return mem

    def _poll_list(self, a):
        if self.mutant == "early_release":
            return [self.pl[a][0]]
        return list(self.xmask)

    def _after_arrival(self, lo):
        pc, r, i, bad, pend, k, slot, rank, use = lo
        if self.mode == "plain" and slot != 0 and self.mutant != "no_cu_wait":
            return (self.WAIT_REL, r, 0, bad, pend, k, slot, rank, use)
        return (self.POLL, r, 0, bad, pend, k, slot, rank, use)

    def step(self, a, sh, lo):
        pc, r, i, bad, pend, k, slot, rank, use = lo
        mem, l1, l2, arrive, mail, rel, reg = sh
        x, c = self.pl[a]
        stamp = r + 1
        if pc == self.WRITE:
            idx = self._slot_index(r, a)
            if self.mode == "coherent":
                sh = (self._set(mem, idx, r),) + sh[1:]
                nxt = self.REG_X if (self.register and r == 0) else (
                    self.FB_WB if not use else (self.SCAN if k == 0 else self.ARRIVE))
                return sh, (nxt, r, 0, bad, None, k, slot, rank, use)
            nxt = self.COMPLETE
            if (self.mutant == "flag_before_store" and use and k != 0
                    and not (self.register and r == 0)):
                nxt = self.ARRIVE
            return sh, (nxt, r, 0, bad, (idx, r), k, slot, rank, use)
        if pc == self.COMPLETE:
            sh = self._store_complete(sh, a, pend[0], pend[1])
            lo = (pc, r, 0, bad, None, k, slot, rank, use)
            if self.register and r == 0:
                return sh, (self.REG_X,) + lo[1:]
            if not use:
                return sh, (self.FB_WB,) + lo[1:]
            if self.mutant == "flag_before_store" and k != 0:  # flag already stored
                return sh, self._after_arrival(lo)
            return sh, ((self.SCAN if k == 0 else self.ARRIVE),) + lo[1:]
        if pc == self.ARRIVE:
            sh = (mem, l1, l2, self._set(arrive, a, stamp), mail, rel, reg)
            lo2 = (pc, r, 0, bad, pend, k, slot, rank, use)
            if pend is not None:  # flag_before_store: the slot store completes later
                return sh, (self.COMPLETE,) + lo2[1:]
            return sh, self._after_arrival(lo2)
        if pc == self.SCAN:
            lst = self._scan_list(a)
            if i < len(lst):
                if arrive[lst[i]] >= stamp:
                    return sh, (self.SCAN, r, i + 1, bad, pend, k, slot, rank, use)
                return sh, lo
            nxt = self.PUB if (self.mode == "coherent" or self.mutant == "no_writeback") else self.WB
            return sh, (nxt, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.WB:
            return self._writeback(sh, x), (self.PUB, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.PUB:
            if not (self.mutant == "skip_copy" and x == 0 and i == self.C - 1):
                mail = self._set(mail, i, self._set(mail[i], x, stamp))
            sh = (mem, l1, l2, arrive, mail, rel, reg)
            if i + 1 < self.C:
                return sh, (self.PUB, r, i + 1, bad, pend, k, slot, rank, use)
            return sh, self._after_arrival(lo)
        if pc == self.POLL:
            lst = self._poll_list(a)
            copy = (x + self.X * rank) % self.C
            if i < len(lst):
                if mail[copy][lst[i]] >= stamp:
                    return sh, (self.POLL, r, i + 1, bad, pend, k, slot, rank, use)
                return sh, lo
            if self.mode == "coherent" or (self.mutant == "no_cu_wait" and slot != 0):
                nxt = self.READ
            elif self.mode == "l1only":
                nxt = self.INV_L1
            else:
                nxt = self.REL if self.mutant == "no_invalidate" else self.ACQ
            return sh, (nxt, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.ACQ:
            return self._acquire(sh, a), (self.REL, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.REL:
            sh = (mem, l1, l2, arrive, mail, self._set(rel, x * self.cu_lines + rank, stamp), reg)
            return sh, (self.READ, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.WAIT_REL:
            if rel[x * self.cu_lines + rank] >= stamp:
                return sh, (self.READ, r, 0, bad, pend, k, slot, rank, use)
            return sh, lo
        if pc == self.INV_L1:
            return self._inv_l1(sh, a), (self.READ, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.READ:
            sh, v = self._load(sh, a, self._slot_index(r, (a + r) % self.n))
            bad = bad or v != r
            nxt = self.WRITE if r + 1 < self.R else self.DONE
            return sh, (nxt, r + 1, 0, bad, pend, k, slot, rank, use)
        # ---- round 0 with registration -------------------------------------------------
        xcount, cucount, xcu, curank, overflow, cnt = reg
        if pc == self.REG_X:
            k = xcount[x]
            overflow += 1 if k >= self.block else 0
            reg = (self._set(xcount, x, k + 1), cucount, xcu, curank, overflow, cnt)
            return (mem, l1, l2, arrive, mail, rel, reg), (self.REG_CU, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.REG_CU:
            slot = cucount[c]
            reg = (xcount, self._set(cucount, c, slot + 1), xcu, curank, overflow, cnt)
            nxt = self.REG_RANK if slot == 0 else self.REG_WB
            return (mem, l1, l2, arrive, mail, rel, reg), (nxt, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.LATE:  # rank_after_arrival: the CU leader stores its rank only now
            reg = (xcount, cucount, xcu, self._set(curank, c, i), overflow, cnt)
            return (mem, l1, l2, arrive, mail, rel, reg), (self.REG_POLL, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.REG_RANK:
            rk = xcu[x]
            overflow += 1 if rk >= self.cu_lines else 0
            reg = (xcount, cucount, self._set(xcu, x, rk + 1), curank, overflow, cnt)
            return (mem, l1, l2, arrive, mail, rel, reg), (self.REG_RANKST, r, rk, bad, pend, k, slot, rank, use)
        if pc == self.REG_RANKST:
            if self.mutant == "rank_after_arrival":
                return sh, (self.REG_WB, r, i, bad, pend, k, slot, rank, use)
            reg = (xcount, cucount, xcu, self._set(curank, c, i), overflow, cnt)
            return (mem, l1, l2, arrive, mail, rel, reg), (self.REG_WB, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.REG_WB:
            sh = sh if self.mode == "coherent" else self._writeback(sh, x)
            return sh, (self.REG_ARRIVE, r, i, bad, pend, k, slot, rank, use)
        if pc == self.REG_ARRIVE:
            reg = (xcount, cucount, xcu, curank, overflow, cnt + 1)
            late = self.mutant == "rank_after_arrival" and slot == 0
            return (mem, l1, l2, arrive, mail, rel, reg), (
                (self.LATE if late else self.REG_POLL), r, i if late else 0, bad, pend, k, slot,
                rank, use)
        if pc == self.REG_POLL:
            if cnt >= self.n:
                return sh, (self.REG_ACQ, r, 0, bad, pend, k, slot, rank, use)
            return sh, lo
        if pc == self.REG_ACQ:
            sh = sh if self.mode == "coherent" else self._acquire(sh, a)
            return sh, (self.REG_READ, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.REG_READ:
            rank = curank[c]
            use = overflow == 0
            return sh, (self.READ, r, 0, bad, pend, k, slot, rank, use)
        # ---- fallback: a fenced counter barrier (round r's target is n * r; round 0's
        # registration barrier counted n) ----------------------------------------------------
        if pc == self.FB_WB:
            sh = sh if self.mode == "coherent" else self._writeback(sh, x)
            return sh, (self.FB_ARRIVE, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.FB_ARRIVE:
            reg = (xcount, cucount, xcu, curank, overflow, cnt + 1)
            return (mem, l1, l2, arrive, mail, rel, reg), (self.FB_POLL, r, 0, bad, pend, k, slot, rank, use)
        if pc == self.FB_POLL:
            if cnt >= self.n * (r + 1):
                return sh, (self.FB_ACQ, r, 0, bad, pend, k, slot, rank, use)
            return sh, lo
        if pc == self.FB_ACQ:
            sh = sh if self.mode == "coherent" else self._acquire(sh, a)
            return sh, (self.READ, r, 0, bad, pend, k, slot, rank, use)
        raise AssertionError(pc)

    def check(self, sh, los):
        for b, lo in enumerate(los):
            if lo[3]:
                return f"phase violated: agent {b} read stale or overwritten data"
        return None

    def final_check(self, sh, los):
        if not self.register:
            return None
        fits = all(m <= self.block for m in self.members) and all(
            len({c for x2, c in self.pl if x2 == x}) <= self.cu_lines for x in range(self.X))
        if any(lo[8] != fits for lo in los):
            return f"per-XCD path taken {[lo[8] for lo in los]}, registration fits: {fits}"
        for x in self.xmask:
            on = [a for a in range(self.n) if self.pl[a][0] == x]
            if sorted(los[a][5] for a in on) != list(range(len(on))):
                return f"XCD {x}: member numbers {[los[a][5] for a in on]}"
            cus = sorted({self.pl[a][1] for a in on})
            if sorted({los[a][7] for a in on}) != list(range(len(cus))) or any(
                    los[a][7] != los[b][7] for a in on for b in on
                    if self.pl[a][1] == self.pl[b][1]):
                return f"XCD {x}: CU ranks {[los[a][7] for a in on]}"
            for cu in cus:
                if sorted(los[a][6] for a in on if self.pl[a][1] == cu) != list(
                        range(sum(1 for a in on if self.pl[a][1] == cu))):
                    return f"CU {cu}: registration order {[los[a][6] for a in on]}"
        return None
