// CPU oracle for the inter-workgroup synchronization primitives of
// Stuart & Owens, "Efficient Synchronization Primitives for GPUs" (2011).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
// CPU-baseline leg of the benchmark may load or call this library.  It shares no code,
// header, table or constant with the GPU library: everything here is written from the
// paper and from the plain definitions of the synthetic workloads.
//
// Two independent parts:
//   (O1) closed forms -- sequential, single-threaded definitions of every workload's
//        output.  These are the bit-exact expected values.
//   (O2) threaded reference -- one std::thread per agent (an agent is one workgroup
//        acting with "block semantics", Section 3), shared words are
//        std::atomic<uint32_t>, and each primitive follows Section 5 and the appendix
//        algorithms.  It must reproduce (O1) and hold the invariants of Section 5's
//        definitions (barrier phase, mutual exclusion, at most n inside a semaphore).
//
// Critical-section "non-atomic" updates are written as a relaxed load followed by a
// relaxed store on std::atomic: a lost update (a mutual-exclusion bug) still shows up
// in the counts, but the program has no data race in the C++ sense.
//
// Every function returns 0 on success or a negative code on a detected violation.

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

extern "C" {

// ------------------------------------------------------------------------------------
// Counter-based hash used by all synthetic workloads.
//
// The paper defines no hash; the workloads use "splitmix32", read here as the 32-bit
// golden-ratio increment (floor(2^32 / phi) = 0x9E3779B9) followed by the 32-bit
// MurmurHash3 finalizer (fmix32).
// ------------------------------------------------------------------------------------
uint32_t or_fmix32(uint32_t z) {
  z ^= z >> 16;
  z *= 0x85EBCA6Bu;
  z ^= z >> 13;
  z *= 0xC2B2AE35u;
  z ^= z >> 16;
  return z;
}

uint32_t or_sm32(uint32_t x) { return or_fmix32(x + 0x9E3779B9u); }

// Per-(agent, operation, stream) key for the mutex and semaphore schedules:
// key(b, j, s) = sm32(sm32(sm32(seed ^ s) ^ b) ^ j).
uint32_t or_key(uint32_t seed, uint32_t b, uint32_t j, uint32_t s) {
  return or_sm32(or_sm32(or_sm32(seed ^ s) ^ b) ^ j);
}

// Hash chain of the serving workload: h_0 = x, h_{i+1} = sm32(h_i), result h_L.
uint32_t or_chain(uint32_t x, uint32_t L) {
  uint32_t h = x;
  for (uint32_t i = 0; i < L; ++i) h = or_sm32(h);
  return h;
}

void or_chain_batch(uint32_t seed, const uint32_t* L, uint32_t n, uint32_t* out) {
  for (uint32_t r = 0; r < n; ++r) out[r] = or_chain(seed ^ r, L[r]);
}

// Number of operations agent b performs when `total` operations are split over nwg
// agents: total / nwg each, and the first (total mod nwg) agents do one more.
uint64_t or_ops_for_agent(uint32_t nwg, uint64_t total, uint32_t b) {
  uint64_t base = total / nwg;
  uint64_t extra = total % nwg;
  return base + (b < extra ? 1 : 0);
}

// ------------------------------------------------------------------------------------
// (O1) Closed forms
// ------------------------------------------------------------------------------------

// Hash-exchange barrier workload.  In round r agent b publishes
// sm32(seed ^ (b << 16) ^ r), everyone passes the barrier, then agent b XORs the
// value published by agent (b + r) mod N in the same round into its checksum.
void or_barrier_closed(uint32_t seed, uint32_t N, uint32_t R, uint32_t* chk) {
  for (uint32_t b = 0; b < N; ++b) {
    uint32_t c = 0;
    for (uint32_t r = 0; r < R; ++r) {
      uint32_t src = (uint32_t)(((uint64_t)b + r) % N);
      c ^= or_sm32(seed ^ (src << 16) ^ r);
    }
    chk[b] = c;
  }
}

// Mutex workload: agent b's j-th acquisition takes lock key(b,j,1) mod L and adds one
// to each of that lock's W words.  Final word value = number of acquisitions of the
// lock.  words has L*W entries, lock-major.
void or_mutex_closed(uint32_t seed, uint32_t nwg, uint64_t total, uint32_t L, uint32_t W,
                     uint32_t* words) {
  std::memset(words, 0, sizeof(uint32_t) * (size_t)L * W);
  for (uint32_t b = 0; b < nwg; ++b) {
    uint64_t A = or_ops_for_agent(nwg, total, b);
    for (uint64_t j = 0; j < A; ++j) {
      uint32_t lock = or_key(seed, b, (uint32_t)j, 1) % L;
      for (uint32_t w = 0; w < W; ++w) words[(size_t)lock * W + w] += 1;
    }
  }
}

// Semaphore workload: agent b's admission checksum XOR_j sm32(seed ^ (b << 16) ^ j)
// over its own wait/post pairs j.
void or_sem_closed(uint32_t seed, uint32_t nwg, uint64_t total, uint32_t* chk) {
  for (uint32_t b = 0; b < nwg; ++b) {
    uint64_t A = or_ops_for_agent(nwg, total, b);
    uint32_t c = 0;
    for (uint64_t j = 0; j < A; ++j) c ^= or_sm32(seed ^ (b << 16) ^ (uint32_t)j);
    chk[b] = c;
  }
}

// Memory-system microbenchmark schedule: issuer u (u < U) performs operation i
// (i < n) on position (u + i) mod T of the permutation perm, i.e. on word perm[...].
// counts[t] = number of operations that target word t.
void or_bench_counts(uint32_t U, uint64_t n, uint32_t T, const uint32_t* perm,
                     uint64_t* counts) {
  std::memset(counts, 0, sizeof(uint64_t) * T);
  for (uint32_t u = 0; u < U; ++u)
    for (uint64_t i = 0; i < n; ++i) counts[perm[(u + i) % T]] += 1;
}

// Same count for a single word: the number of (u, i) with (u + i) mod T == p, where p
// is the word's position in the permutation.  For each issuer the hits are the i in
// [0, n) congruent to (p - u) mod T.
uint64_t or_bench_count_one(uint32_t U, uint64_t n, uint32_t T, uint32_t p) {
  uint64_t c = 0;
  for (uint32_t u = 0; u < U; ++u) {
    uint64_t first = ((uint64_t)p + T - (u % T)) % T;  // smallest i with (u+i)%T == p
    if (first < n) c += (n - 1 - first) / T + 1;
  }
  return c;
}

// Sum of (v mod 2^32) over the integers v in [a, a + c): the total of the values an
// atomic increment returns when a word starting at a receives c increments.
// Uses S(m) = sum of (v mod 2^32) for v in [0, m): full 2^32 cycles contribute
// 2^31 * (2^32 - 1) each, the remainder q contributes q (q - 1) / 2.  Result mod 2^64.
static uint64_t sum_mod32_prefix(unsigned __int128 m) {
  const unsigned __int128 P = (unsigned __int128)1 << 32;
  unsigned __int128 cycles = m / P, rem = m % P;
  unsigned __int128 s = cycles * ((P * (P - 1)) / 2);
  if (rem > 0) s += (rem * (rem - 1)) / 2;
  return (uint64_t)s;
}
uint64_t or_sum_increments(uint32_t a, uint64_t c) {
  unsigned __int128 lo = a, hi = (unsigned __int128)a + c;
  return sum_mod32_prefix(hi) - sum_mod32_prefix(lo);
}

// Value written by issuer u's i-th exchange: sm32(sm32(seed ^ u) ^ i).
uint32_t or_exch_value(uint32_t seed, uint32_t u, uint32_t i) {
  return or_sm32(or_sm32(seed ^ u) ^ i);
}

// Prefill of word t for the load / store / exchange benchmarks: sm32(seed ^ t).
uint32_t or_prefill(uint32_t seed, uint32_t t) { return or_sm32(seed ^ t); }

// Closed forms of the microbenchmark outputs (op: 0 ADD, 1 CAS-increment, 2 EXCH,
// 3 LD, 4 ST).  finals[t] is the final word value; *sum is the uint64 sum (mod 2^64)
// of every value the operations returned.  For EXCH the final values are not unique
// and the function returns instead, in *sum, the conserved quantity
// sum(initial) + sum(written), which must equal sum(returned) + sum(final).
int or_bench_closed(int op, uint32_t seed, uint32_t U, uint64_t n, uint32_t T,
                    const uint32_t* perm, uint32_t* finals, uint64_t* sum) {
  std::vector<uint64_t> counts(T);
  or_bench_counts(U, n, T, perm, counts.data());
  uint64_t s = 0;
  switch (op) {
    case 0:
    case 1:  // words start at 0; each receives counts[t] increments
      for (uint32_t t = 0; t < T; ++t) {
        finals[t] = (uint32_t)counts[t];
        s += or_sum_increments(0, counts[t]);
      }
      break;
    case 2:  // exchange: conservation of the multiset of values
      for (uint32_t t = 0; t < T; ++t) {
        finals[t] = 0;  // not unique
        s += or_prefill(seed, t);
      }
      for (uint32_t u = 0; u < U; ++u)
        for (uint64_t i = 0; i < n; ++i) s += or_exch_value(seed, u, (uint32_t)i);
      break;
    case 3:  // load: words keep their prefill; each load returns it
      for (uint32_t t = 0; t < T; ++t) {
        finals[t] = or_prefill(seed, t);
        s += counts[t] * (uint64_t)finals[t];
      }
      break;
    case 4:  // store: words start at 0; every store to word t writes sm32(seed ^ t)
      for (uint32_t t = 0; t < T; ++t) finals[t] = counts[t] ? or_prefill(seed, t) : 0u;
      break;
    default:
      return -1;
  }
  *sum = s;
  return 0;
}

// Exchange finals are not unique (last writer wins), but each final word must be its
// initial value sm32(seed ^ t) or one of the values written to that word.  Returns the
// number of words for which neither holds (0 for a valid outcome).
uint64_t or_exch_finals_invalid(uint32_t seed, uint32_t U, uint64_t n, uint32_t T,
                                const uint32_t* perm, const uint32_t* finals) {
  std::vector<char> ok(T, 0);
  for (uint32_t t = 0; t < T; ++t) ok[t] = finals[t] == or_prefill(seed, t);
  for (uint32_t u = 0; u < U; ++u)
    for (uint64_t i = 0; i < n; ++i) {
      const uint32_t t = perm[(u + i) % T];
      if (!ok[t] && finals[t] == or_exch_value(seed, u, (uint32_t)i)) ok[t] = 1;
    }
  uint64_t bad = 0;
  for (uint32_t t = 0; t < T; ++t) bad += ok[t] ? 0 : 1;
  return bad;
}

// Multiset of the values the bounded buffer's producers put, in producer order: producer
// w's j-th value is sm32(seed ^ (w << 16) ^ j); shares split as or_ops_for_agent.
void or_bb_values(uint32_t seed, uint32_t P, uint64_t items, uint32_t* out) {
  uint64_t k = 0;
  for (uint32_t w = 0; w < P; ++w) {
    const uint64_t A = or_ops_for_agent(P, items, w);
    for (uint64_t j = 0; j < A; ++j) out[k++] = or_sm32(seed ^ (w << 16) ^ (uint32_t)j);
  }
}

// ------------------------------------------------------------------------------------
// (O2) Threaded reference
// ------------------------------------------------------------------------------------

unsigned or_hardware_threads(void) { return std::thread::hardware_concurrency(); }

}  // extern "C"

namespace {

using Word = std::atomic<uint32_t>;

// Wrap-safe "a has reached b" for monotone 32-bit counters.
inline bool reached(uint32_t a, uint32_t b) { return (int32_t)(a - b) >= 0; }

// Waits yield the core: agents (threads) outnumber host cores.
inline void relax() { std::this_thread::yield(); }

// Backoff of Section 5 (mutex): a counter I runs from Imin; after every failed attempt
// the agent waits I units and increments I, and wraps to Imin once I exceeds Imax.  One
// unit is one uncontended load.
struct Backoff {
  uint32_t imin, imax, i;
  Word private_word{0};
  Backoff(uint32_t lo, uint32_t hi) : imin(lo), imax(hi), i(lo) {}
  void operator()() {
    for (uint32_t k = 0; k < i; ++k) (void)private_word.load(std::memory_order_relaxed);
    relax();
    i += 1;
    if (i > imax) i = imin;
  }
};

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double seconds() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

template <class F>
double run_agents(uint32_t n, F&& body) {
  std::vector<std::thread> threads;
  threads.reserve(n);
  std::atomic<uint32_t> ready{0};
  std::atomic<bool> go{false};
  for (uint32_t b = 0; b < n; ++b)
    threads.emplace_back([&, b] {
      ready.fetch_add(1);
      while (!go.load(std::memory_order_acquire)) relax();
      body(b);
    });
  while (ready.load() != n) relax();
  Timer t;
  go.store(true, std::memory_order_release);
  for (auto& th : threads) th.join();
  return t.seconds();
}

}  // namespace

extern "C" {

// Barrier kinds: 0 centralized counter, 1 hierarchical (groups of agents, then a top
// counter), 2 decentralized flag barrier with a master agent (the "XF" barrier of
// Section 5), 3 the per-XCD flag protocol (below), 4 centralized counter whose last
// arriver publishes a separate release word.  The workload is the hash exchange of
// or_barrier_closed; the published values live in two slot arrays selected by round
// parity, so that a round-(r+1) store can never overwrite a round-r value that has not
// been read yet.
//
// Kind 3 groups the agents as a GPU groups workgroups: agent b sits in group (XCD)
// b mod G and in "CU" (b / G) mod 4 of that group.  Round 0 registers every agent with
// fetch-and-adds -- its member number in its group (member 0 is the group's master), its
// order on its CU (0 = the CU's leader), and for a CU's leader the rank of the CU among
// its group's CUs -- then passes a counter barrier and reads the registration.  Later
// rounds: a member stores its arrival stamp in its group's flag block; the master checks
// every member's flag, then stores the group's stamp into each of 2G copies; each CU
// leader waits until every populated group's stamp is in copy (group + G * rank) mod 2G,
// then stores its CU's release line; the other agents of the CU wait on that line.
// Returns 0, or -2 if the phase check failed (an agent read a slot that did not hold
// the value of the round it is in).
int or_barrier_threaded(int kind, uint32_t seed, uint32_t N, uint32_t R, uint32_t groups,
                        uint32_t* chk, double* seconds) {
  if (N == 0 || kind < 0 || kind > 4) return -1;
  if (groups == 0) groups = 1;
  std::vector<Word> slot(2 * (size_t)N);
  for (auto& s : slot) s.store(0);
  Word cnt{0};
  // hierarchical state
  uint32_t G = groups < N ? groups : N;
  std::vector<Word> gcnt(G), ggen(G);
  for (uint32_t g = 0; g < G; ++g) gcnt[g].store(0), ggen[g].store(0);
  Word top{0}, topgen{0};
  // flag state
  std::vector<Word> arrive(N), release(N);
  for (uint32_t b = 0; b < N; ++b) arrive[b].store(0), release[b].store(0);
  std::atomic<int> bad{0};
  // split state
  Word gen{0};
  // per-XCD state (kind 3): G groups, kCus CUs per group, C = 2G copies of the stamps
  constexpr uint32_t kCus = 4;
  const uint32_t C = 2 * G;
  const uint32_t block = (N + G - 1) / G;
  std::vector<Word> xcount(G), xcu(G), cucount((size_t)G * kCus), currank((size_t)G * kCus);
  std::vector<Word> larrive((size_t)G * block), mail((size_t)C * G), rel((size_t)G * kCus);
  for (auto* v : {&xcount, &xcu, &cucount, &currank, &larrive, &mail, &rel})
    for (auto& w : *v) w.store(0);
  struct Reg {
    uint32_t x, k, members, slot, rank, copy;
    uint32_t xmask;
  };
  std::vector<Reg> reg(N);

  auto members = [&](uint32_t g) { return (N - g + G - 1) / G; };  // agents b with b%G==g

  auto wait_reached = [&](const Word& w, uint32_t stamp) {
    while (!reached(w.load(std::memory_order_acquire), stamp)) relax();
  };

  // Round 0 of kind 3: registration, then a counter barrier, then read it back.
  auto xcd_register = [&](uint32_t b) {
    Reg& g = reg[b];
    g.x = b % G;
    const uint32_t cu = g.x * kCus + (b / G) % kCus;
    g.k = xcount[g.x].fetch_add(1, std::memory_order_relaxed);
    g.slot = cucount[cu].fetch_add(1, std::memory_order_relaxed);
    if (g.slot == 0)
      currank[cu].store(xcu[g.x].fetch_add(1, std::memory_order_relaxed),
                        std::memory_order_relaxed);
    cnt.fetch_add(1, std::memory_order_acq_rel);
    wait_reached(cnt, N);
    g.members = xcount[g.x].load(std::memory_order_relaxed);
    g.rank = currank[cu].load(std::memory_order_relaxed);
    g.copy = (g.x + G * g.rank) % C;
    g.xmask = 0;
    for (uint32_t i = 0; i < G; ++i)
      if (xcount[i].load(std::memory_order_relaxed) != 0) g.xmask |= 1u << i;
  };
  auto xcd_round = [&](uint32_t b, uint32_t stamp) {
    const Reg& g = reg[b];
    Word* blk = &larrive[(size_t)g.x * block];
    if (g.k == 0) {
      for (uint32_t m = 1; m < g.members; ++m) wait_reached(blk[m], stamp);
      for (uint32_t c = 0; c < C; ++c)
        mail[(size_t)c * G + g.x].store(stamp, std::memory_order_release);
    } else {
      blk[g.k].store(stamp, std::memory_order_release);
    }
    Word& line = rel[(size_t)g.x * kCus + g.rank];
    if (g.slot == 0) {
      for (uint32_t i = 0; i < G; ++i)
        if ((g.xmask >> i) & 1) wait_reached(mail[(size_t)g.copy * G + i], stamp);
      line.store(stamp, std::memory_order_release);
    } else {
      wait_reached(line, stamp);
    }
  };

  auto barrier = [&](uint32_t b, uint32_t r) {
    const uint32_t stamp = r + 1;
    if (kind == 3) {
      if (r == 0) xcd_register(b);
      else xcd_round(b, stamp);
    } else if (kind == 4) {
      const uint32_t old = cnt.fetch_add(1, std::memory_order_acq_rel);
      if (old == N * stamp - 1) gen.store(stamp, std::memory_order_release);
      else wait_reached(gen, stamp);
    } else if (kind == 0) {
      cnt.fetch_add(1, std::memory_order_acq_rel);
      const uint32_t target = N * stamp;
      while (!reached(cnt.load(std::memory_order_acquire), target)) relax();
    } else if (kind == 1) {
      const uint32_t g = b % G, m = members(g);
      uint32_t old = gcnt[g].fetch_add(1, std::memory_order_acq_rel);
      if (old == m * stamp - 1) {  // last agent of its group
        uint32_t t = top.fetch_add(1, std::memory_order_acq_rel);
        if (t == G * stamp - 1)
          topgen.store(stamp, std::memory_order_release);
        else
          while (!reached(topgen.load(std::memory_order_acquire), stamp)) relax();
        ggen[g].store(stamp, std::memory_order_release);
      } else {
        while (!reached(ggen[g].load(std::memory_order_acquire), stamp)) relax();
      }
    } else {
      arrive[b].store(stamp, std::memory_order_release);
      if (b == 0) {
        for (uint32_t i = 0; i < N; ++i)
          while (!reached(arrive[i].load(std::memory_order_acquire), stamp)) relax();
        for (uint32_t i = 0; i < N; ++i) release[i].store(stamp, std::memory_order_release);
      } else {
        while (!reached(release[b].load(std::memory_order_acquire), stamp)) relax();
      }
    }
  };

  double t = run_agents(N, [&](uint32_t b) {
    uint32_t c = 0;
    for (uint32_t r = 0; r < R; ++r) {
      slot[(size_t)(r & 1) * N + b].store(or_sm32(seed ^ (b << 16) ^ r),
                                          std::memory_order_relaxed);
      barrier(b, r);
      uint32_t src = (uint32_t)(((uint64_t)b + r) % N);
      uint32_t v = slot[(size_t)(r & 1) * N + src].load(std::memory_order_relaxed);
      if (v != or_sm32(seed ^ (src << 16) ^ r)) bad.store(1);
      c ^= v;
    }
    chk[b] = c;
  });
  if (seconds) *seconds = t;
  return bad.load() ? -2 : 0;
}

// Mutex kinds: 0 spin lock by compare-and-swap, 1 spin lock by exchange (Algorithm 1),
// 2 spin lock with the Section 5 backoff (Algorithm 2), 3 fetch-and-add ticket mutex
// with backoff while polling (Algorithm 3), 4 polling mutex: wait with plain loads until
// the word reads free, then one compare-and-swap, 5 ring-buffer mutex (Section 5's design
// alternative: enqueue one's id, wait until the head's entry is one's own), 6 array queue
// lock (wait on one's own slot, unlock grants the next), 7 ticket mutex waiting in
// proportion to the distance from the head, 8 cohort lock, 9 MCS queue lock (a linked
// queue of per-agent nodes: lock exchanges the tail with one's node and, behind a
// predecessor, links in and waits on one's own node; unlock hands over to the successor
// or, when none has linked in, swings the tail back to empty with a compare-and-swap),
// 10 CU-cohort lock (kind 8 with a ticket lock per CU group in front of each cohort's).
// Workload: see or_mutex_closed.  An owner word checks mutual exclusion inside every
// critical section.  Returns 0, or -2 on a mutual-exclusion violation.
int or_mutex_threaded(int kind, uint32_t seed, uint32_t nwg, uint64_t total, uint32_t L,
                      uint32_t W, uint32_t imin, uint32_t imax, uint32_t* words,
                      double* seconds) {
  if (nwg == 0 || L == 0 || W == 0 || kind < 0 || kind > 10) return -1;
  std::vector<Word> lockw(L), ticket(L), turn(L), owner(L);
  for (uint32_t l = 0; l < L; ++l) lockw[l] = 0, ticket[l] = 0, turn[l] = 0, owner[l] = 0;
  // kinds 5 (ring) and 6 (array): Q slots per lock, Q a power of two >= agents
  uint32_t Q = 1;
  while (Q < nwg) Q <<= 1;
  std::vector<Word> slots(kind >= 5 ? (size_t)L * Q : 0);
  for (auto& w : slots) w.store(0);
  std::vector<Word> cs((size_t)L * W);
  for (auto& w : cs) w.store(0);
  std::atomic<int> bad{0};
  // kind 8 (cohort): agent b belongs to cohort b mod kCoh; per lock and cohort a local
  // ticket counter and kGrants grant slots, local ticket t polling slot t mod kGrants for
  // local turn t | session << 32 (session 0 = the cohort does not hold the global lock,
  // k > 0 = it does and k holders passed it on); at most kPasses holders in a row.
  constexpr uint32_t kCoh = 8, kPasses = 4, kGrants = 4;
  // kind 9 (MCS): per lock and agent a node {next (agent + 1, 0 = none), locked}; the
  // lock's tail is lockw (agent + 1, 0 = free)
  std::vector<Word> mnext(kind == 9 ? (size_t)L * nwg : 0), mlocked(mnext.size());
  for (size_t i = 0; i < mnext.size(); ++i) mnext[i] = 0, mlocked[i] = 0;
  std::vector<Word> lt(kind == 8 || kind == 10 ? (size_t)L * kCoh : 0);
  std::vector<std::atomic<uint64_t>> grant(lt.size() * kGrants);
  for (size_t i = 0; i < lt.size(); ++i) lt[i] = 0;
  for (auto& g : grant) g = 0;
  // kind 10 (CU cohort): agent b of cohort b mod kCoh sits in CU group (b / kCoh) mod kCu
  // of it; per lock and CU group a ticket counter, a grant word (CU turn | CU session <<
  // 32), the record of the cohort lock the group's session holds (what kind 8's lock
  // returned) and the announcement of the tickets drawn (a lower bound, stores in any
  // order); at most kPasses holders of a group in a row.  cu_hold keeps each agent's CU
  // ticket | CU session << 32 while it holds a lock.
  constexpr uint32_t kCu = 4;
  const size_t ncu = kind == 10 ? (size_t)L * kCoh * kCu : 0;
  std::vector<Word> cut(ncu), cann(ncu);
  std::vector<std::atomic<uint64_t>> cgrant(ncu), crec(ncu);
  for (size_t i = 0; i < ncu; ++i) cut[i] = 0, cann[i] = 0, cgrant[i] = 0, crec[i] = 0;
  std::vector<uint64_t> cu_hold(kind == 10 ? nwg : 0);

  // kind 8's two levels: the cohort's local ticket lock, then the global one unless the
  // grant says the cohort holds it; returns the local ticket | session read << 32
  auto cohort_lock = [&](uint32_t l, uint32_t b) -> uint64_t {
    const size_t c = (size_t)l * kCoh + b % kCoh;
    const uint32_t my = lt[c].fetch_add(1, std::memory_order_relaxed);
    uint64_t v;
    auto& slot = grant[c * kGrants + my % kGrants];
    while ((uint32_t)(v = slot.load(std::memory_order_acquire)) != my) relax();
    const uint32_t k = (uint32_t)(v >> 32);
    if (k == 0) {
      const uint32_t g = ticket[l].fetch_add(1, std::memory_order_relaxed);
      while (turn[l].load(std::memory_order_acquire) != g) relax();
    }
    return ((uint64_t)k << 32) | my;
  };
  auto cohort_unlock = [&](uint32_t l, uint32_t b, uint64_t held) {
    const size_t c = (size_t)l * kCoh + b % kCoh;
    const uint32_t my = (uint32_t)held, k = (uint32_t)(held >> 32) + 1;
    const bool waiter = (int32_t)(lt[c].load(std::memory_order_relaxed) - (my + 1)) > 0;
    auto& next = grant[c * kGrants + (my + 1) % kGrants];  // the next local ticket's slot
    if (waiter && k < kPasses) {  // pass the global lock with the local one
      next.store(((uint64_t)k << 32) | (my + 1), std::memory_order_release);
    } else {
      const uint32_t t = turn[l].load(std::memory_order_relaxed);  // only the holder writes
      turn[l].store(t + 1, std::memory_order_release);
      next.store(my + 1, std::memory_order_release);  // session 0
    }
  };
  auto cu_of = [&](uint32_t l, uint32_t b) -> size_t {
    return ((size_t)l * kCoh + b % kCoh) * kCu + (b / kCoh) % kCu;
  };

  // returns the ticket the lock was taken with (ticket, ring and array kinds); cohort:
  // the local ticket, and the session it read in the upper 32 bits
  auto lock = [&](uint32_t l, uint32_t b, Backoff& bo) -> uint64_t {
    switch (kind) {
      case 0:
        for (;;) {
          uint32_t e = 0;
          if (lockw[l].compare_exchange_strong(e, 1, std::memory_order_acquire,
                                               std::memory_order_relaxed))
            return 0;
          relax();
        }
      case 1:
        while (lockw[l].exchange(1, std::memory_order_acquire) != 0) relax();
        return 0;
      case 2:
        bo.i = bo.imin;
        while (lockw[l].exchange(1, std::memory_order_acquire) != 0) bo();
        return 0;
      case 3: {
        uint32_t my = ticket[l].fetch_add(1, std::memory_order_relaxed);
        bo.i = bo.imin;
        while (turn[l].load(std::memory_order_acquire) != my) bo();
        return my;
      }
      case 7: {  // ticket lock, waiting in proportion to the distance from the head
        uint32_t my = ticket[l].fetch_add(1, std::memory_order_relaxed);
        for (;;) {
          const uint32_t cur = turn[l].load(std::memory_order_acquire);
          if (cur == my) return my;
          for (uint32_t k = 1; k < my - cur && k < 64; ++k) relax();
          relax();
        }
      }
      case 5: {  // ring: enqueue one's id, wait until the head's entry is one's own
        uint32_t my = ticket[l].fetch_add(1, std::memory_order_relaxed);
        Word* ring = &slots[(size_t)l * Q];
        ring[my & (Q - 1)].store(my + 1, std::memory_order_relaxed);
        for (;;) {
          uint32_t h = turn[l].load(std::memory_order_acquire);
          if (ring[h & (Q - 1)].load(std::memory_order_acquire) == my + 1) return my;
          relax();
        }
      }
      case 6: {  // array: wait on one's own slot
        uint32_t my = ticket[l].fetch_add(1, std::memory_order_relaxed);
        Word& slot = slots[(size_t)l * Q + (my & (Q - 1))];
        while (slot.load(std::memory_order_acquire) != my) relax();
        return my;
      }
      case 9: {  // MCS
        const size_t me = (size_t)l * nwg + b;
        mnext[me].store(0, std::memory_order_relaxed);
        mlocked[me].store(1, std::memory_order_relaxed);
        const uint32_t prev = lockw[l].exchange(b + 1, std::memory_order_acq_rel);
        if (prev != 0) {
          mnext[(size_t)l * nwg + (prev - 1)].store(b + 1, std::memory_order_release);
          while (mlocked[me].load(std::memory_order_acquire) != 0) relax();
        }
        return 0;
      }
      case 8:
        return cohort_lock(l, b);
      case 10: {  // the CU group's ticket lock, then kind 8's unless the group holds it
        const size_t u = cu_of(l, b);
        const uint32_t tc = cut[u].fetch_add(1, std::memory_order_relaxed);
        cann[u].store(tc + 1, std::memory_order_relaxed);
        uint64_t v;
        while ((uint32_t)(v = cgrant[u].load(std::memory_order_acquire)) != tc) relax();
        const uint32_t kc = (uint32_t)(v >> 32);
        cu_hold[b] = ((uint64_t)kc << 32) | tc;
        if (kc > 0) return crec[u].load(std::memory_order_relaxed);
        const uint64_t held = cohort_lock(l, b);
        crec[u].store(held, std::memory_order_relaxed);  // for the group's later holders
        return held;
      }
      default:
        for (;;) {
          while (lockw[l].load(std::memory_order_relaxed) != 0) relax();
          uint32_t e = 0;
          if (lockw[l].compare_exchange_strong(e, 1, std::memory_order_acquire,
                                               std::memory_order_relaxed))
            return 0;
        }
    }
  };
  auto unlock = [&](uint32_t l, uint32_t b, uint64_t held) {
    const uint32_t my = (uint32_t)held;
    if (kind == 9) {
      const size_t me = (size_t)l * nwg + b;
      uint32_t nx = mnext[me].load(std::memory_order_acquire);
      if (nx == 0) {
        uint32_t expect = b + 1;
        if (lockw[l].compare_exchange_strong(expect, 0, std::memory_order_acq_rel,
                                             std::memory_order_relaxed))
          return;
        while ((nx = mnext[me].load(std::memory_order_acquire)) == 0) relax();
      }
      mlocked[(size_t)l * nwg + (nx - 1)].store(0, std::memory_order_release);
      return;
    }
    if (kind == 8) {
      cohort_unlock(l, b, held);
      return;
    }
    if (kind == 10) {
      const size_t u = cu_of(l, b);
      const uint32_t tc = (uint32_t)cu_hold[b], kc = (uint32_t)(cu_hold[b] >> 32) + 1;
      const bool waiter = (int32_t)(cann[u].load(std::memory_order_relaxed) - (tc + 1)) > 0;
      if (waiter && kc < kPasses) {  // the group's next holder keeps the cohort lock
        cgrant[u].store(((uint64_t)kc << 32) | (tc + 1), std::memory_order_release);
      } else {
        cohort_unlock(l, b, held);
        cgrant[u].store(tc + 1, std::memory_order_release);  // session 0
      }
      return;
    }
    if (kind == 3 || kind == 7) {
      uint32_t t = turn[l].load(std::memory_order_relaxed);  // only the holder writes turn
      turn[l].store(t + 1, std::memory_order_release);
    } else if (kind == 5) {
      turn[l].store(my + 1, std::memory_order_release);  // advance the ring's head
    } else if (kind == 6) {
      slots[(size_t)l * Q + ((my + 1) & (Q - 1))].store(my + 1, std::memory_order_release);
    } else {
      lockw[l].store(0, std::memory_order_release);
    }
  };

  double t = run_agents(nwg, [&](uint32_t b) {
    Backoff bo(imin ? imin : 1, imax ? imax : 1);
    uint64_t A = or_ops_for_agent(nwg, total, b);
    for (uint64_t j = 0; j < A; ++j) {
      uint32_t l = or_key(seed, b, (uint32_t)j, 1) % L;
      const uint64_t my = lock(l, b, bo);
      if (owner[l].exchange(b + 1, std::memory_order_relaxed) != 0) bad.store(1);
      for (uint32_t w = 0; w < W; ++w) {
        Word& x = cs[(size_t)l * W + w];
        x.store(x.load(std::memory_order_relaxed) + 1, std::memory_order_relaxed);
      }
      if (owner[l].exchange(0, std::memory_order_relaxed) != b + 1) bad.store(1);
      unlock(l, b, my);
    }
  });
  for (size_t i = 0; i < cs.size(); ++i) words[i] = cs[i].load();
  if (seconds) *seconds = t;
  return bad.load() ? -2 : 0;
}

static uint64_t sum64(const std::vector<std::atomic<uint64_t>>& v) {
  uint64_t t = 0;
  for (auto& x : v) t += x.load();
  return t;
}

// Semaphore kinds: 0 spin semaphore (Algorithm 4), 1 spin semaphore with backoff in
// both loops (Algorithm 4, UseBackoff), 2 fetch-and-add semaphore (Algorithm 5),
// 3 fetch-and-add semaphore whose queued waiters yield between polls.
// Initial value K.  Algorithm 4 keeps S = K + 1 (zero means "held"); Algorithm 5 keeps
// count, ticket and turn starting at 0, and a queued waiter proceeds once turn is
// strictly greater than the ticket it drew (0-based).
// kind: 0 Algorithm 4, 1 Algorithm 4 with backoff in both loops (the listing), 2
// Algorithm 5, 3 Algorithm 5 with yielding polls, 4 two monotone counters (ticket t
// enters once posts + K > t), 5 the same admission rule with proportional waiting (a
// waiter d posts short of admission yields (d - 1) / 4 extra times per poll), 6 Algorithm
// 4 with backoff in wait only (Section 5's prose: post proceeds aggressively), 7 Algorithm
// 5's count with a queue per group of agents (agent b in group b mod 8): a post
// decrements count and hands its unit over only if a waiter is counted beyond K, to the
// oldest waiter of its own group (at most 4 times in a row for one unit), else to the
// first other group with a waiter; for K = 1 a post that reads count above 1 knows
// before its decrement that a waiter exists; 8 two 64-bit monotone counters with a grant
// slot per ticket (16 slots, so tickets share them): ticket t >= K waits until slot
// t mod 16 holds at least t + 1, and the post that draws p raises slot (p + K) mod 16
// to p + K + 1 (a maximum: grants for one slot may land in any order); 9 K chains of
// tickets: ticket t >= K waits until slot t mod M holds t + 1, which the holder of ticket
// t - K stores when it posts (M = K x max(1, 16 / K), a multiple of K); 10 kind 9 once
// per group of agents (agent b in group b mod 8; group g owns K / 8 units, the first
// K mod 8 groups one more; K >= 8).
// Each pair: wait, occupancy tracking, checksum update, admission count, post.
// out: chk[nwg]; *maxocc; state[4] = {S or count, ticket, turn, admissions}; for the
// Algorithm 4 kinds ticket and turn are unused and state[1] / state[2] report instead the
// failed exchanges of wait / of post (attempts that found S held or the semaphore full).
// Returns 0, -2 if occupancy ever exceeded K.
int or_sem_threaded(int kind, uint32_t K, uint32_t seed, uint32_t nwg, uint64_t total,
                    uint32_t imin, uint32_t imax, uint32_t* chk, uint32_t* maxocc,
                    uint32_t* state, double* seconds) {
  if (nwg == 0 || K == 0 || kind < 0 || kind > 10) return -1;
  if (kind == 10 && K < 8) return -1;
  Word S{K + 1}, count{0}, ticket{0}, turn{0}, occ{0}, maxo{0}, adm{0};
  // kind 7: per group a queue of Q slots {ticket + 1, passes} after (drawn, served)
  constexpr uint32_t kGroups = 8, kBound = 4;
  uint32_t Q = 1;
  while (Q < nwg) Q <<= 1;
  std::vector<Word> drawn(kind == 7 ? kGroups : 0), served(drawn.size());
  std::vector<std::atomic<uint64_t>> slots(kind == 7 ? (size_t)kGroups * Q : 0);
  for (size_t i = 0; i < drawn.size(); ++i) drawn[i] = 0, served[i] = 0;
  for (auto& w : slots) w.store(0);
  // kind 8: 64-bit tickets drawn and posts made, and the grant slots
  constexpr uint32_t kGrantSlots = 16;
  std::atomic<uint64_t> tickets64{0}, posts64{0};
  const uint32_t chain_len = K * std::max<uint32_t>(1, kGrantSlots / K);
  std::vector<std::atomic<uint64_t>> grants(kind == 8 ? kGrantSlots : kind == 9 ? chain_len : 0);
  for (auto& w : grants) w.store(0);
  std::vector<uint64_t> my_ticket(kind >= 9 ? nwg : 0);  // kinds 9, 10: the ticket held
  // kind 10: per group its units, tickets, posts and chain slots
  constexpr uint32_t kChainGroups = 8;
  auto group_units = [&](uint32_t g) { return K / kChainGroups + (g < K % kChainGroups ? 1u : 0u); };
  std::vector<std::atomic<uint64_t>> gtickets(kind == 10 ? kChainGroups : 0),
      gposts(gtickets.size());
  std::vector<std::vector<std::atomic<uint64_t>>> gslots(gtickets.size());
  for (uint32_t g = 0; g < gtickets.size(); ++g) {
    gtickets[g] = 0;
    gposts[g] = 0;
    const uint32_t kg = group_units(g);
    gslots[g] = std::vector<std::atomic<uint64_t>>(kg * std::max<uint32_t>(1, kGrantSlots / kg));
    for (auto& w : gslots[g]) w.store(0);
  }
  auto claim = [&](uint32_t g, uint32_t* t) {
    uint32_t v = served[g].load(std::memory_order_relaxed);
    while ((int32_t)(drawn[g].load(std::memory_order_relaxed) - v) > 0)
      if (served[g].compare_exchange_weak(v, v + 1, std::memory_order_acq_rel)) {
        *t = v;
        return true;
      }
    return false;
  };
  auto grant = [&](uint32_t g, uint32_t t, uint32_t k) {
    // into an empty slot only, atomically: the slot's previous ticket (t - Q) may be
    // granted by another poster at the same moment
    auto& slot = slots[(size_t)g * Q + (t & (Q - 1))];
    const uint64_t v = ((uint64_t)k << 32) | (t + 1);
    for (uint64_t e = 0; !slot.compare_exchange_weak(e, v, std::memory_order_acq_rel); e = 0)
      relax();
  };
  auto claim_from = [&](uint32_t first, uint32_t* g, uint32_t* t) {
    for (;;) {
      for (uint32_t d = 0; d < kGroups; ++d)
        if (claim((first + d) % kGroups, t)) {
          *g = (first + d) % kGroups;
          return;
        }
      relax();
    }
  };
  std::vector<uint32_t> pass(kind == 7 ? nwg : 0, 0);
  const bool alg4 = kind <= 1 || kind == 6, backoff = kind == 1 || kind == 6;
  const bool post_backoff = kind == 1;
  std::atomic<uint64_t> wait_fail{0}, post_fail{0};

  auto wait = [&](Backoff& bo, uint32_t b) {
    if (kind == 10) {
      const uint32_t g = b % kChainGroups, kg = group_units(g);
      const uint64_t t = gtickets[g].fetch_add(1, std::memory_order_acq_rel);
      my_ticket[b] = t;
      if (t >= kg)
        while (gslots[g][t % gslots[g].size()].load(std::memory_order_acquire) != t + 1) relax();
      return;
    }
    if (kind == 9) {
      const uint64_t t = tickets64.fetch_add(1, std::memory_order_acq_rel);
      my_ticket[b] = t;
      if (t >= K)
        while (grants[t % chain_len].load(std::memory_order_acquire) != t + 1) relax();
      return;
    }
    if (kind == 8) {
      const uint64_t t = tickets64.fetch_add(1, std::memory_order_acq_rel);
      if (t >= K)
        while (grants[t % kGrantSlots].load(std::memory_order_acquire) <= t) relax();
      return;
    }
    if (kind == 7) {
      uint32_t k = 0;
      if (count.fetch_add(1, std::memory_order_acq_rel) >= K) {
        const uint32_t g = b % kGroups;
        const uint32_t t = drawn[g].fetch_add(1, std::memory_order_acq_rel);
        auto& slot = slots[(size_t)g * Q + (t & (Q - 1))];
        uint64_t v;
        while ((uint32_t)(v = slot.load(std::memory_order_acquire)) != t + 1) relax();
        k = (uint32_t)(v >> 32);
        slot.store(0, std::memory_order_release);
      }
      pass[b] = k;
      return;
    }
    if (alg4) {
      bo.i = bo.imin;
      for (;;) {
        uint32_t v = S.exchange(0, std::memory_order_acquire);
        if (v > 1) {
          S.exchange(v - 1, std::memory_order_release);
          return;
        }
        if (v == 1) S.exchange(1, std::memory_order_release);
        wait_fail.fetch_add(1, std::memory_order_relaxed);
        if (backoff) bo(); else relax();
      }
    } else if (kind == 4 || kind == 5) {
      // two monotone counters: ticket t enters once posts + K > t
      const uint32_t t = ticket.fetch_add(1, std::memory_order_acq_rel);
      for (;;) {
        const uint32_t posts = turn.load(std::memory_order_acquire);
        if ((int32_t)(posts + K - t) > 0) break;
        if (kind == 5)
          for (uint32_t k = 0, d = t - (posts + K) + 1; k < (d - 1) / 4; ++k) relax();
        relax();
      }
    } else {
      uint32_t old = count.fetch_add(1, std::memory_order_acq_rel);
      if (old < K) return;
      uint32_t idx = ticket.fetch_add(1, std::memory_order_acq_rel);
      while (!((int32_t)(turn.load(std::memory_order_acquire) - idx) > 0)) relax();
    }
  };
  auto post = [&](Backoff& bo, uint32_t b) {
    if (kind == 10) {
      const uint32_t g = b % kChainGroups;
      const uint64_t q = my_ticket[b] + group_units(g);
      gslots[g][q % gslots[g].size()].store(q + 1, std::memory_order_release);
      gposts[g].fetch_add(1, std::memory_order_relaxed);
      return;
    }
    if (kind == 9) {
      const uint64_t q = my_ticket[b] + K;
      grants[q % chain_len].store(q + 1, std::memory_order_release);
      posts64.fetch_add(1, std::memory_order_relaxed);
      return;
    }
    if (kind == 8) {
      const uint64_t q = posts64.fetch_add(1, std::memory_order_acq_rel) + K;
      auto& g = grants[q % kGrantSlots];
      uint64_t v = g.load(std::memory_order_relaxed);
      while (v < q + 1 && !g.compare_exchange_weak(v, q + 1, std::memory_order_acq_rel)) {
      }
      return;
    }
    if (kind == 7) {
      const uint32_t g = b % kGroups, k = pass[b];
      const bool stay = k + 1 < kBound;
      uint32_t y = 0, t = 0;
      // K = 1 only: the poster holds the only unit, so a loaded count above 1 is still
      // above 1 when its own decrement lands (a waiter exists)
      if (K == 1 && count.load(std::memory_order_acquire) > 1) {
        count.fetch_sub(1, std::memory_order_acq_rel);
        if (stay && claim(g, &t)) {
          grant(g, t, k + 1);
        } else {
          claim_from(g + 1, &y, &t);
          grant(y, t, 0);
        }
      } else if (count.fetch_sub(1, std::memory_order_acq_rel) > K) {
        claim_from(stay ? g : g + 1, &y, &t);
        grant(y, t, y == g ? k + 1 : 0);
      }
      return;
    }
    if (alg4) {
      bo.i = bo.imin;
      for (;;) {
        uint32_t v = S.exchange(0, std::memory_order_acquire);
        if (v > 0) {
          S.exchange(v + 1, std::memory_order_release);
          return;
        }
        post_fail.fetch_add(1, std::memory_order_relaxed);
        if (post_backoff) bo(); else relax();
      }
    } else if (kind == 4 || kind == 5) {
      turn.fetch_add(1, std::memory_order_acq_rel);
    } else {
      uint32_t old = count.fetch_sub(1, std::memory_order_acq_rel);
      if (old > K) turn.fetch_add(1, std::memory_order_acq_rel);
    }
  };

  double t = run_agents(nwg, [&](uint32_t b) {
    Backoff bo(imin ? imin : 1, imax ? imax : 1);
    uint64_t A = or_ops_for_agent(nwg, total, b);
    uint32_t c = 0;
    for (uint64_t j = 0; j < A; ++j) {
      wait(bo, b);
      uint32_t o = occ.fetch_add(1) + 1;
      uint32_t m = maxo.load();
      while (o > m && !maxo.compare_exchange_weak(m, o)) {
      }
      c ^= or_sm32(seed ^ (b << 16) ^ (uint32_t)j);
      adm.fetch_add(1);
      occ.fetch_sub(1);
      post(bo, b);
    }
    chk[b] = c;
  });
  *maxocc = maxo.load();
  if (kind == 7) {  // every local ticket served, every slot taken
    for (uint32_t g = 0; g < kGroups; ++g)
      if (drawn[g].load() != served[g].load()) return -3;
    for (auto& w : slots)
      if (w.load() != 0) return -3;
  }
  state[0] = alg4 ? S.load() : count.load();
  state[1] = alg4 ? (uint32_t)std::min<uint64_t>(wait_fail.load(), 0xFFFFFFFFu)
                  : kind == 10 ? (uint32_t)sum64(gtickets)
                  : kind >= 8 ? (uint32_t)tickets64.load() : ticket.load();
  state[2] = alg4 ? (uint32_t)std::min<uint64_t>(post_fail.load(), 0xFFFFFFFFu)
                  : kind == 10 ? (uint32_t)sum64(gposts)
                  : kind >= 8 ? (uint32_t)posts64.load() : turn.load();
  state[3] = adm.load();
  if (seconds) *seconds = t;
  return *maxocc > K ? -2 : 0;
}

// Threaded microbenchmark: `threads` host threads share the U issuers round-robin and
// perform the schedule of or_bench_counts with real atomics on a T-word array.
// finals[T]; *sum = uint64 sum of returned values (for EXCH: returned + final).
int or_bench_threaded(int op, uint32_t seed, uint32_t U, uint64_t n, uint32_t T,
                      const uint32_t* perm, uint32_t threads, uint32_t* finals,
                      uint64_t* sum, double* seconds) {
  if (T == 0 || op < 0 || op > 4) return -1;
  if (threads == 0) threads = 1;
  std::vector<Word> m(T);
  // ADD, CAS and ST start from zero; EXCH and LD start from the prefill.
  for (uint32_t t = 0; t < T; ++t) m[t].store((op == 2 || op == 3) ? or_prefill(seed, t) : 0u);
  std::atomic<uint64_t> total{0};
  double secs = run_agents(threads, [&](uint32_t th) {
    uint64_t s = 0;
    for (uint32_t u = th; u < U; u += threads)
      for (uint64_t i = 0; i < n; ++i) {
        uint32_t t = perm[(u + i) % T];
        switch (op) {
          case 0: s += m[t].fetch_add(1, std::memory_order_relaxed); break;
          case 1: {
            uint32_t o = m[t].load(std::memory_order_relaxed);
            while (!m[t].compare_exchange_weak(o, o + 1, std::memory_order_relaxed)) {
            }
            s += o;
            break;
          }
          case 2: s += m[t].exchange(or_exch_value(seed, u, (uint32_t)i), std::memory_order_relaxed); break;
          case 3: s += m[t].load(std::memory_order_relaxed); break;
          default: m[t].store(or_prefill(seed, t), std::memory_order_relaxed); break;
        }
      }
    total.fetch_add(s);
  });
  uint64_t s = total.load();
  for (uint32_t t = 0; t < T; ++t) {
    finals[t] = m[t].load();
    if (op == 2) s += finals[t];
  }
  *sum = s;
  if (seconds) *seconds = secs;
  return 0;
}

// Threaded serving queue: `agents` threads take requests in order from a shared counter
// (every request has already arrived), admit each against a budget of K units with the
// weighted fetch-and-add rule (draw u tickets, wait until units returned + K cover the
// last one), compute the request's hash chain, return the units.  out[n] = results;
// *maxuse = most units held at once; counters = {tickets drawn, units returned}.
// Returns 0, -1 on bad arguments, -2 if the units held ever exceeded K.
int or_serve_threaded(uint32_t seed, const uint32_t* L, const uint32_t* units, uint32_t n,
                      uint32_t K, uint32_t agents, uint32_t* out, uint32_t* maxuse,
                      uint64_t* counters, double* seconds) {
  if (agents == 0 || K == 0) return -1;
  for (uint32_t r = 0; r < n; ++r)
    if (units[r] > K) return -1;
  Word head{0}, issued{0}, released{0}, inuse{0}, maxu{0};
  double t = run_agents(agents, [&](uint32_t) {
    for (;;) {
      const uint32_t r = head.fetch_add(1, std::memory_order_relaxed);
      if (r >= n) return;
      const uint32_t u = units[r];
      const uint32_t end = issued.fetch_add(u, std::memory_order_acq_rel) + u;
      while (!((int32_t)(released.load(std::memory_order_acquire) + K - end) >= 0)) relax();
      const uint32_t now = inuse.fetch_add(u) + u;
      uint32_t m = maxu.load();
      while (now > m && !maxu.compare_exchange_weak(m, now)) {
      }
      out[r] = or_chain(seed ^ r, L[r]);
      inuse.fetch_sub(u);
      released.fetch_add(u, std::memory_order_acq_rel);
    }
  });
  *maxuse = maxu.load();
  counters[0] = issued.load();
  counters[1] = released.load();
  if (seconds) *seconds = t;
  return *maxuse > K ? -2 : 0;
}

// Bounded buffer (condition variables).  Producer w < P puts its share of `items`
// values, the j-th being sm32(seed ^ (w << 16) ^ j); shares split as or_ops_for_agent.
// Closed form of what the consumers take in total: out[0] = xor, out[1] = sum (uint64).
void or_bb_closed(uint32_t seed, uint32_t P, uint64_t items, uint64_t* out) {
  uint32_t x = 0;
  uint64_t s = 0;
  for (uint32_t w = 0; w < P; ++w) {
    const uint64_t A = or_ops_for_agent(P, items, w);
    for (uint64_t j = 0; j < A; ++j) {
      const uint32_t v = or_sm32(seed ^ (w << 16) ^ (uint32_t)j);
      x ^= v;
      s += v;
    }
  }
  out[0] = x;
  out[1] = s;
}

// Threaded bounded buffer on std::mutex and std::condition_variable: P producer and C
// consumer threads share a ring of `capacity` values.  out: {xor, sum, taken, put,
// most values in the ring at once, values left}.  Returns 0, or -2 if the ring ever
// held more than capacity or fewer than 0 values.
int or_bb_threaded(uint32_t seed, uint32_t P, uint32_t C, uint64_t items, uint32_t capacity,
                   uint64_t* out, double* seconds) {
  if (P == 0 || C == 0 || capacity == 0) return -1;
  std::mutex mu;
  std::condition_variable not_full, not_empty;
  std::vector<uint32_t> ring(capacity);
  uint64_t head = 0, tail = 0, count = 0, maxc = 0, put = 0, taken = 0, sum = 0;
  uint32_t x = 0;
  int bad = 0;
  double t = run_agents(P + C, [&](uint32_t a) {
    if (a < P) {
      const uint64_t A = or_ops_for_agent(P, items, a);
      for (uint64_t j = 0; j < A; ++j) {
        const uint32_t v = or_sm32(seed ^ (a << 16) ^ (uint32_t)j);
        std::unique_lock<std::mutex> lk(mu);
        not_full.wait(lk, [&] { return count < capacity; });
        ring[tail++ % capacity] = v;
        ++count;
        ++put;
        if (count > maxc) maxc = count;
        if (count > capacity) bad = 1;
        not_empty.notify_one();
      }
    } else {
      const uint64_t A = or_ops_for_agent(C, items, a - P);
      uint32_t lx = 0;
      uint64_t ls = 0;
      for (uint64_t j = 0; j < A; ++j) {
        std::unique_lock<std::mutex> lk(mu);
        not_empty.wait(lk, [&] { return count > 0; });
        const uint32_t v = ring[head++ % capacity];
        --count;
        ++taken;
        not_full.notify_one();
        lk.unlock();
        lx ^= v;
        ls += v;
      }
      std::lock_guard<std::mutex> g(mu);
      x ^= lx;
      sum += ls;
    }
  });
  out[0] = x;
  out[1] = sum;
  out[2] = taken;
  out[3] = put;
  out[4] = maxc;
  out[5] = count;
  if (seconds) *seconds = t;
  return bad ? -2 : 0;
}

}  // extern "C"
