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
    in front of a global ticket lock.  The cohort's grant word holds the local turn and
    the session together (one store writes both, one load reads both): session 0 says
    the cohort does not hold the global lock, k > 0 that it does and k holders have
    passed it on.  A local holder that reads session 0 takes the global lock.  Unlock:
    when a local waiter exists (local tickets drawn beyond one's own) and k + 1 < B,
    grant (turn + 1, k + 1) -- the global lock stays with the cohort; else release the
    global lock, then grant (turn + 1, 0).
    mutant 'keep_session': a global release grants (turn + 1, k + 1);
    mutant 'no_waiter_check': pass locally even when nobody of the cohort waits;
    mutant 'skip_global_wait': a holder reading session 0 takes a global ticket but
    enters without waiting for its turn."""

    (ACQ, POLL_L, G_ACQ, POLL_G, CS_IN, CS_LD, CS_ST, CS_OUT, REL, REL_G, REL_L,
     DONE) = range(12)

    def __init__(self, n: int = 4, ops: int = 2, C: int = 2, B: int = 2,
                 mutant: str | None = None):
        self.n, self.ops, self.C, self.B, self.mutant = n, ops, C, B, mutant

    def init(self):
        C = self.C
        # shared = (gticket, gturn, lticket, lturn, sess, data, inside, entries)
        # local  = (pc, j, tmp, t, s)
        sh = (0, 0, (0,) * C, (0,) * C, (0,) * C, 0, 0, 0)
        return sh, tuple((self.ACQ, 0, 0, 0, 0) for _ in range(self.n))

    def done(self, lo):
        return lo[0] == self.DONE

    @staticmethod
    def _set(tup, i, v):
        return tup[:i] + (v,) + tup[i + 1:]

    def step(self, a, sh, lo):
        gt, gturn, lt, ltn, sess, data, inside, entries = sh
        pc, j, tmp, t, s = lo
        c = a % self.C
        nxt = self.ACQ if j + 1 < self.ops else self.DONE
        if pc == self.ACQ:
            return (gt, gturn, self._set(lt, c, lt[c] + 1), ltn, sess, data, inside,
                    entries), (self.POLL_L, j, tmp, lt[c], s)
        if pc == self.POLL_L:  # reads turn and session in one load
            if ltn[c] != t:
                return sh, (self.POLL_L, j, tmp, t, s)
            return sh, ((self.G_ACQ if sess[c] == 0 else self.CS_IN), j, tmp, t, sess[c])
        if pc == self.G_ACQ:
            after = self.CS_IN if self.mutant == "skip_global_wait" else self.POLL_G
            return (gt + 1, gturn, lt, ltn, sess, data, inside, entries), (after, j, gt, t, s)
        if pc == self.POLL_G:
            return sh, ((self.CS_IN if gturn == tmp else self.POLL_G), j, tmp, t, s)
        if pc == self.CS_IN:
            return (gt, gturn, lt, ltn, sess, data, inside + 1, entries), (self.CS_LD, j, tmp, t, s)
        if pc == self.CS_LD:
            return sh, (self.CS_ST, j, data, t, s)
        if pc == self.CS_ST:
            return (gt, gturn, lt, ltn, sess, tmp + 1, inside, entries), (self.CS_OUT, j, tmp, t, s)
        if pc == self.CS_OUT:
            return (gt, gturn, lt, ltn, sess, data, inside - 1, entries + 1), (self.REL, j, tmp, t, s)
        if pc == self.REL:
            waiter = lt[c] > t + 1 or self.mutant == "no_waiter_check"
            if waiter and s + 1 < self.B:  # pass: one store of the grant word
                return (gt, gturn, lt, self._set(ltn, c, t + 1), self._set(sess, c, s + 1),
                        data, inside, entries), (nxt, j + 1, tmp, t, s)
            return sh, (self.REL_G, j, tmp, t, s)
        if pc == self.REL_G:
            return (gt, gturn + 1, lt, ltn, sess, data, inside, entries), (self.REL_L, j, tmp, t, s)
        if pc == self.REL_L:
            k = s + 1 if self.mutant == "keep_session" else 0
            return (gt, gturn, lt, self._set(ltn, c, t + 1), self._set(sess, c, k), data, inside,
                    entries), (nxt, j + 1, tmp, t, s)
        raise AssertionError(pc)

    def check(self, sh, los):
        if sh[6] > 1:
            return f"mutual exclusion violated: {sh[6]} inside"
        return None

    def final_check(self, sh, los):
        gt, gturn, lt, ltn, sess, data, inside, entries = sh
        total = self.n * self.ops
        if data != total or entries != total:
            return f"final data {data} entries {entries} != {total}"
        if gt != gturn or lt != ltn or any(sess):
            return f"final state gticket {gt} gturn {gturn} local {lt} {ltn} sess {sess}"
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
             'xcd'     -- agents split into G groups (b mod G); the last arriver of a
                          group adds one to a top counter; the last group publishes a
                          top generation word; each group's last arriver copies it into
                          its group's generation word, which the others poll;
             'flag'    -- decentralized: agent b stores r + 1 into arrive[b]; agent 0
                          (master) waits for every arrive flag, then stores r + 1 into
                          every release flag; the others poll their release flag.
       mutant: 'single_buffer' -- one slot array for every round;
               'no_wait'       -- arrive but never wait (central, flag);
               'no_top_wait'   -- xcd: a group's last arriver releases its group without
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
            if self.kind == "xcd":
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
            elif self.kind == "xcd":
                ok = ggen[a % G] >= stamp
            else:
                ok = release[a] >= stamp
            return sh, ((self.READ if ok else self.POLL), r, i, bad)
        if pc == self.TOP:  # xcd: last of the group arrives at the top counter
            t = top
            sh = (slots, cnt, gcnt, ggen, top + 1, topgen, arrive, release)
            if self.mutant == "no_top_wait":
                return sh, (self.GROUP_REL, r, 0, bad)
            return sh, ((self.TOP_REL if t == G * stamp - 1 else self.TOP_POLL), r, 0, bad)
        if pc == self.TOP_POLL:
            return sh, ((self.GROUP_REL if topgen >= stamp else self.TOP_POLL), r, 0, bad)
        if pc == self.TOP_REL:
            return (slots, cnt, gcnt, ggen, top, stamp, arrive, release), (self.GROUP_REL, r, 0, bad)
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
