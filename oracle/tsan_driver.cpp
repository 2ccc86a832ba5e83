// Runs every threaded reference of the oracle on small inputs and checks each against
// the closed forms.  Test infrastructure only: the test-suite builds it with
// -fsanitize=thread, so that a data race in the oracle's own C++ (a missing atomic, a
// plain access shared between threads) is reported by ThreadSanitizer, and a wrong
// result by the exit status.
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
uint32_t or_chain(uint32_t x, uint32_t L);
void or_barrier_closed(uint32_t seed, uint32_t N, uint32_t R, uint32_t* chk);
void or_mutex_closed(uint32_t seed, uint32_t nwg, uint64_t total, uint32_t L, uint32_t W,
                     uint32_t* words);
void or_sem_closed(uint32_t seed, uint32_t nwg, uint64_t total, uint32_t* chk);
void or_bb_closed(uint32_t seed, uint32_t P, uint64_t items, uint64_t* out);
int or_barrier_threaded(int kind, uint32_t seed, uint32_t N, uint32_t R, uint32_t groups,
                        uint32_t* chk, double* seconds);
int or_mutex_threaded(int kind, uint32_t seed, uint32_t nwg, uint64_t total, uint32_t L,
                      uint32_t W, uint32_t imin, uint32_t imax, uint32_t* words,
                      double* seconds);
int or_sem_threaded(int kind, uint32_t K, uint32_t seed, uint32_t nwg, uint64_t total,
                    uint32_t imin, uint32_t imax, uint32_t* chk, uint32_t* maxocc,
                    uint32_t* state, double* seconds);
int or_serve_threaded(uint32_t seed, const uint32_t* L, const uint32_t* units, uint32_t n,
                      uint32_t K, uint32_t agents, uint32_t* out, uint32_t* maxuse,
                      uint64_t* counters, double* seconds);
int or_bb_threaded(uint32_t seed, uint32_t P, uint32_t C, uint64_t items, uint32_t capacity,
                   uint64_t* out, double* seconds);
}

static int failures = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

int main() {
  const uint32_t seed = 42;
  {  // barriers: central, counter tree, flag, per-XCD flag protocol, split central
    const uint32_t N = 6, R = 40;
    std::vector<uint32_t> want(N), got(N);
    or_barrier_closed(seed, N, R, want.data());
    for (int kind = 0; kind <= 4; ++kind) {
      expect(or_barrier_threaded(kind, seed, N, R, 2, got.data(), nullptr) == 0, "barrier rc");
      expect(got == want, "barrier checksums");
    }
  }
  {  // mutexes: every kind, two locks of three words; 16 agents put two in each of the
     // cohort lock's eight cohorts, so its local hand-overs run too, and 64 two in each
     // CU group of the CU-cohort lock (8 cohorts x 4 groups)
    const uint32_t L = 2, W = 3;
    const uint64_t total = 300;
    std::vector<uint32_t> want(L * W), got(L * W);
    for (int kind = 0; kind <= 10; ++kind) {
      const uint32_t nwg = kind == 10 ? 64 : 16;
      or_mutex_closed(seed, nwg, total, L, W, want.data());
      expect(or_mutex_threaded(kind, seed, nwg, total, L, W, 1, 4, got.data(), nullptr) == 0,
             "mutex rc");
      expect(got == want, "mutex words");
    }
  }
  {  // semaphores: every kind, K = 2 (the per-group chains, kind 10, need a unit per
     // group of eight: K = 9 over 16 agents)
    for (int kind = 0; kind <= 10; ++kind) {
      const uint32_t nwg = kind == 10 ? 16 : 6, K = kind == 10 ? 9 : 2;
      const uint64_t total = 300;
      std::vector<uint32_t> want(nwg), got(nwg);
      uint32_t maxocc = 0, state[4];
      or_sem_closed(seed, nwg, total, want.data());
      expect(or_sem_threaded(kind, K, seed, nwg, total, 1, 4, got.data(), &maxocc, state,
                             nullptr) == 0,
             "semaphore rc");
      expect(got == want && maxocc <= K && state[3] == total, "semaphore outputs");
    }
  }
  {  // serving queue: 64 requests, 4 agents, budget 3 units
    const uint32_t n = 64;
    std::vector<uint32_t> L(n), units(n), out(n);
    for (uint32_t r = 0; r < n; ++r) L[r] = (r * 37) % 50, units[r] = 1 + r % 3;
    uint32_t maxuse = 0;
    uint64_t counters[2];
    expect(or_serve_threaded(seed, L.data(), units.data(), n, 3, 4, out.data(), &maxuse,
                             counters, nullptr) == 0,
           "serve rc");
    bool ok = maxuse <= 3 && counters[0] == counters[1];
    for (uint32_t r = 0; r < n; ++r) ok = ok && out[r] == or_chain(seed ^ r, L[r]);
    expect(ok, "serve outputs");
  }
  {  // bounded buffer: 3 producers, 2 consumers, capacity 2
    uint64_t want[2], got[6];
    or_bb_closed(seed, 3, 500, want);
    expect(or_bb_threaded(seed, 3, 2, 500, 2, got, nullptr) == 0, "bounded buffer rc");
    expect(got[0] == want[0] && got[1] == want[1] && got[2] == 500 && got[5] == 0,
           "bounded buffer outputs");
  }
  if (failures == 0) std::printf("all threaded references agree with the closed forms\n");
  return failures ? 1 : 0;
}
