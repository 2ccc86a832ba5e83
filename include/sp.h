/*
 * sp.h -- inter-workgroup synchronization primitives for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libsp.so.  The primitives are those of Stuart & Owens, "Efficient
 * Synchronization Primitives for GPUs" (2011): barriers, mutexes and semaphores with
 * block semantics (Section 3: one leader per workgroup touches the primitive, the rest
 * of the workgroup waits at the workgroup barrier), and the memory-system
 * microbenchmarks of Section 3 that classify a GPU by the abstraction of Section 4.
 *
 * Conventions for every entry point:
 *   - Return SP_OK (0) on success or a negative SP_E_* code; nothing aborts the process.
 *   - Pointers documented "device" must point to device memory of the context's GPU
 *     (for example torch CUDA tensors); "host" pointers to host memory.  The caller owns
 *     every buffer it passes; the library owns only the state objects it creates.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream).  It is borrowed.
 *   - The *_run and sp_bench_* calls launch on `stream`, time the main kernel with HIP
 *     events recorded on that stream, wait for it, check the device watchdog word and
 *     fill `*st` (may be NULL).  Output buffers hold the results when the call returns.
 *   - Every device wait is bounded by sp_params.timeout_ms (wall clock); on expiry the
 *     kernel stops and the call returns SP_E_TIMEOUT.
 *   - A context and the objects created from it are used by one host thread at a time:
 *     all of a context's runs share its watchdog word and its last-error slot (the
 *     serving calls run their own observer thread inside the call).  Use one context per
 *     host thread for concurrent work.
 */
#ifndef SP_H
#define SP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------------------ */
#define SP_OK 0
#define SP_E_INVAL (-1)      /* bad argument (zero size, out-of-range kind, ...)       */
#define SP_E_HIP (-2)        /* a HIP runtime call failed; see sp_last_hip_error       */
#define SP_E_NORESIDENT (-3) /* a barrier needs more co-resident workgroups than fit   */
#define SP_E_TIMEOUT (-4)    /* the device watchdog expired                            */
#define SP_E_PARITY (-5)     /* a kernel's own consistency check failed                */
#define SP_E_RANGE (-6)      /* an allocation-free call's input exceeds its fixed        */
                             /* workspace (see sp_cond_run_bounded_buffer_noalloc)      */

/* ---- kinds -------------------------------------------------------------------------- */
/* Barriers (Section 5, Barrier; Section 2 for the centralized and tree barriers).      */
enum sp_barrier_kind {
  SP_BARRIER_CENTRAL = 0,       /* one monotone counter; waiters poll the counter      */
  SP_BARRIER_CENTRAL_SPLIT = 1, /* counter + separate release word set by last arriver */
  SP_BARRIER_TREE = 2,          /* two-level counter tree: fan_in groups, top counter  */
  SP_BARRIER_FLAG = 3,          /* decentralized flag barrier with a master workgroup  */
  SP_BARRIER_GRID_SYNC = 4,     /* comparator: HIP cooperative-groups grid.sync()      */
  SP_BARRIER_XCD = 5,           /* per-XCD: one L2 writeback per XCD and one           */
                                /* invalidation per CU per round                       */
  SP_BARRIER_DEFAULT = 15       /* the tuned default for this GPU                      */
};

/* Mutexes (Section 5, Mutex; Algorithms 1-3).                                          */
enum sp_mutex_kind {
  SP_MUTEX_SPIN_CAS = 0,     /* compare-and-swap 0 -> 1 until it succeeds              */
  SP_MUTEX_SPIN_EXCH = 1,    /* exchange with 1 until the old value is 0 (Algorithm 1; */
                             /* with sp_params.backoff set, Algorithm 2)               */
  SP_MUTEX_SPIN_BACKOFF = 2, /* compare-and-swap spin lock, backoff after each failure */
  SP_MUTEX_TICKET = 3,       /* fetch-and-add ticket mutex (Algorithm 3)               */
  SP_MUTEX_SLEEP = 4,        /* poll with loads + s_sleep, then one compare-and-swap   */
  SP_MUTEX_RING = 5,         /* Section 5's ring-buffer mutex: write one's id at the    */
                             /* ring's tail, poll until the head's entry is one's own;  */
                             /* unlock advances the head                                */
  SP_MUTEX_ARRAY = 6,        /* array queue lock: draw ticket t, poll only slot t mod Q */
                             /* (its own line) until it holds t; unlock grants the next */
  SP_MUTEX_ADAPTIVE = 7,     /* ticket mutex whose waiters sleep in proportion to their */
                             /* distance from the head, scaled by a hand-over time each */
                             /* workgroup learns online from its own waits              */
  SP_MUTEX_COHORT = 8,       /* XCD-cohort lock: a ticket lock per XCD in front of a    */
                             /* global ticket lock; the holder passes the global lock   */
                             /* to a waiter of its own XCD (at most cohort_passes       */
                             /* times in a row) without the L2 writeback, which only a  */
                             /* hand-over to another XCD needs.  State: 32 padded lines */
                             /* per lock (sp_mutex_run refuses more than 2^28 words)    */
  SP_MUTEX_MCS = 9,          /* MCS queue lock: a linked queue of per-workgroup nodes;  */
                             /* each waiter polls only its own node; unlock hands over  */
                             /* to the successor or frees the tail with a CAS.  State:  */
                             /* one padded node per lock and workgroup of the run       */
  SP_MUTEX_CU_COHORT = 10,   /* CU-cohort lock: SP_MUTEX_COHORT with a ticket lock per  */
                             /* CU in front of each XCD's; a holder passes the XCD lock */
                             /* to a waiter of its own CU (at most cohort_passes times  */
                             /* in a row) through a word in the CU's shared L1, with no */
                             /* cache maintenance.  State: 16 x 256 x 3 padded lines    */
                             /* per lock besides the XCD cohorts' (sp_mutex_run refuses */
                             /* more than 2^28 words)                                   */
  SP_MUTEX_DEFAULT = 15
};

/* Semaphores (Section 5, Semaphore; Algorithms 4-5).                                   */
enum sp_sem_kind {
  SP_SEM_SPIN = 0,         /* exchange-based spin semaphore (Algorithm 4)              */
  SP_SEM_SPIN_BACKOFF = 1, /* Algorithm 4 with backoff (sp_params.backoff NONE: exponential */
                           /* up to max(backoff_max, 8192) units); post_backoff below     */
  SP_SEM_TICKET = 2,       /* fetch-and-add semaphore, plain polling (Algorithm 5)      */
  SP_SEM_SLEEP = 3,        /* Algorithm 5, queued waiters s_sleep between polls         */
  SP_SEM_COUNTERS = 4,     /* two monotone counters: wait draws a ticket t (fetch-and-  */
                           /* add) and enters once posts + K > t; post adds one to the  */
                           /* posts; FIFO like Algorithm 5, one atomic per operation,   */
                           /* s_sleep between polls                                     */
  SP_SEM_ADAPTIVE = 5,     /* SP_SEM_COUNTERS' admission rule with proportional waiting  */
                           /* tuned online: a waiter d posts short of admission sleeps  */
                           /* about (d - 1) / 4 post intervals between polls, the       */
                           /* interval learned per workgroup from the rate at which the */
                           /* posts counter advanced while it waited, so the queue's    */
                           /* far end stops loading the counter's line                  */
  SP_SEM_COHORT = 6,       /* Algorithm 5's count with a queue per XCD: a post writes    */
                           /* back, decrements, and hands its unit to the oldest waiter  */
                           /* of its own XCD (at most cohort_passes times in a row), else */
                           /* to another XCD's waiter; each waiter polls its own slot.   */
                           /* K = 1: a post that sees a waiter counted skips the writeback */
                           /* for a waiter of its own XCD (same L2)                      */
  SP_SEM_ARRAY = 7,        /* SP_SEM_COUNTERS' admission rule with a grant slot per      */
                           /* ticket (64-bit counters): ticket t >= K polls slot t mod  */
                           /* 4096 (its own line) until it holds at least t + 1; the    */
                           /* post that draws p raises slot (p + K) mod 4096 to p + K + 1 */
                           /* with an atomic max, so no line is polled by the queue     */
  SP_SEM_CHAIN = 8,        /* K chains of tickets: ticket t >= K enters once the holder  */
                           /* of ticket t - K has posted, which stores t + 1 into slot t */
                           /* mod M (M = the largest multiple of K <= 4096, each waiter  */
                           /* polling its own line); the post needs no round trip.       */
                           /* K <= 4096; each post follows its own workgroup's wait      */
  SP_SEM_XCD_CHAIN = 9,    /* SP_SEM_CHAIN per XCD: the K units split over the XCDs'     */
                           /* queues (XCC id mod XCD count), each queue its own tickets, */
                           /* slots and chains; a post skips the L2 writeback, the next */
                           /* holder of its chain running on the same XCD.  XCD count <= */
                           /* K <= 4096 x XCD count; units do not move between XCDs     */
  SP_SEM_CU_LOCK = 10,     /* K = 1 only: the binary semaphore run as the CU-cohort lock */
                           /* (SP_MUTEX_CU_COHORT): a unit passed between workgroups of  */
                           /* one CU goes through the CU's L1 with no cache maintenance  */
  SP_SEM_DEFAULT = 15
};

/* Backoff policy (Section 5, Mutex: linear counter from I_min, wraps past I_max).     */
enum sp_backoff_kind {
  SP_BACKOFF_NONE = 0,
  SP_BACKOFF_PAPER = 1, /* wait I units, I += 1, I > I_max -> I = I_min                  */
  SP_BACKOFF_EXP = 2    /* wait I units, I = min(2 I, I_max)                             */
};
enum sp_backoff_unit {
  SP_UNIT_SLEEP = 0, /* one s_sleep 1 (64 shader clocks)                               */
  SP_UNIT_LOAD = 1   /* one uncontended agent-scope load (the paper's unit)             */
};

/* Microbenchmark operations and issue modes (Section 3).                              */
enum sp_op { SP_OP_ADD = 0, SP_OP_CAS = 1, SP_OP_EXCH = 2, SP_OP_LD = 3, SP_OP_ST = 4 };
enum sp_issue {
  SP_ISSUE_PER_LANE = 0,   /* every lane issues its own operations                     */
  SP_ISSUE_WAVE_LEADER = 1 /* lane 0 of each wavefront issues                           */
};

/* The twelve memory-system tests of Section 3 (Table 1): contention x access kind.    */
enum sp_paper12 {
  SP_P12_CONT_VOL_READ = 0,
  SP_P12_CONT_VOL_WRITE = 1,
  SP_P12_NONCONT_VOL_READ = 2,
  SP_P12_NONCONT_VOL_WRITE = 3,
  SP_P12_CONT_ATOM_READ = 4, /* atomic read = atomic add of 0                          */
  SP_P12_CONT_ATOM_WRITE = 5, /* atomic write = atomic exchange with 0                 */
  SP_P12_NONCONT_ATOM_READ = 6,
  SP_P12_NONCONT_ATOM_WRITE = 7,
  SP_P12_CONT_VOL_READ_AFTER_ATOM = 8, /* one atomic first, then the volatile loop     */
  SP_P12_CONT_VOL_WRITE_AFTER_ATOM = 9,
  SP_P12_NONCONT_VOL_READ_AFTER_ATOM = 10,
  SP_P12_NONCONT_VOL_WRITE_AFTER_ATOM = 11
};

/* ---- parameters and statistics ----------------------------------------------------- */
typedef struct sp_params {
  uint32_t backoff;      /* sp_backoff_kind                                              */
  uint32_t backoff_min;  /* I_min (units), >= 1                                          */
  uint32_t backoff_max;  /* I_max (units), >= backoff_min                                */
  uint32_t backoff_unit; /* sp_backoff_unit                                              */
  uint32_t poll_sleep;   /* s_sleep 1 count between two polls of a wait loop (0 = hot)  */
  uint32_t fan_in;       /* SP_BARRIER_TREE: number of groups (0 = number of XCDs)       */
  uint32_t pad_bytes;    /* spacing of state words, power of two in [4, 4096]            */
  uint32_t flags_packed; /* SP_BARRIER_FLAG: 1 = flags packed 4 B apart, 0 = pad_bytes  */
  uint32_t timeout_ms;   /* watchdog for every device wait (0 = 20000)                   */
  uint32_t verify;       /* mutex runs: check mutual exclusion inside every critical     */
                         /* section with an owner word (SP_E_PARITY on a violation)       */
  uint32_t cooperative;  /* barrier runs: 1 = hipLaunchCooperativeKernel; 0 = plain launch */
                         /* after the library's own co-residency check (a workgroup that   */
                         /* is not resident ends in SP_E_TIMEOUT through the watchdog)     */
  uint32_t coherent_cs;  /* mutexes and semaphores: 1 = the critical sections access the  */
                         /* protected words with agent-scope loads and stores, which every */
                         /* XCD sees without cache maintenance, so lock / wait skip the    */
                         /* acquire invalidate and unlock / post the release writeback.    */
                         /* Barriers: 1 = the data                                         */
                         /* exchanged across the barrier is accessed that way (the paper's */
                         /* volatile accesses), so the barrier does no cache maintenance   */
                         /* (and the per-XCD barrier needs no per-CU release hop).         */
                         /* 0 = plain accesses, fenced (the general contract)              */
  uint32_t xcd_copies;   /* SP_BARRIER_XCD: copies of the XCD stamps that the workgroups    */
                         /* poll for the release (default 64).  0 = one line per XCD stamp, */
                         /* which every poller reads.  C in [1, 256], a power of two: C     */
                         /* padded lines that each hold every XCD's stamp packed; each      */
                         /* XCD's master writes its stamp into every copy and the           */
                         /* workgroups of a CU poll copy (XCD + number of XCDs * rank of    */
                         /* the CU in its XCD) mod C, which spreads the polling over C      */
                         /* lines.  Timing only; results are the same.                      */
  uint32_t cohort_passes; /* SP_MUTEX_COHORT: holders of one XCD that may take the lock */
                           /* in a row before it goes back to the global queue, 1..255    */
                           /* (0 = 64); SP_SEM_COHORT: local hand-overs of one unit in a  */
                           /* row before it goes to another XCD                           */
  uint32_t flag_placement; /* SP_BARRIER_XCD: 0 = measured (default).  A signal between    */
                           /* two workgroups takes 30-40 % less time when its line lives   */
                           /* in memory close to their XCD, so sp_barrier_create times a   */
                           /* same-XCD hand-over on each 8 KiB chunk of a 512 KiB area for */
                           /* every XCD (~2 ms) and gives each XCD its fastest free chunk  */
                           /* for its arrival flags, the stamp copies it polls (when       */
                           /* xcd_copies is a multiple of the XCD count) and its CUs'      */
                           /* release lines, each when it fits in a chunk                  */
                           /* (sp_barrier_info reports the outcome).                       */
                           /* 1 = fixed layout (XCD-major blocks).  Timing only.           */
  uint32_t post_backoff;   /* SP_SEM_SPIN_BACKOFF (Algorithm 4): 0 = post retries at once  */
                           /* (Section 5's prose: post proceeds aggressively, only wait     */
                           /* backs off), 1 = post backs off after a failed exchange as     */
                           /* wait does (the Algorithm 4 listing)                           */
  uint32_t reserved[3];
} sp_params;

typedef struct sp_stats {
  double kernel_ms;        /* HIP-event time of the main kernel                          */
  uint32_t nwg;            /* workgroups launched                                        */
  uint32_t lanes;          /* threads per workgroup                                      */
  uint32_t resident_per_cu;/* occupancy limit reported for this kernel, workgroups / CU  */
  uint32_t device_error;   /* watchdog word after the run (0 = none)                     */
  uint64_t ops;            /* operations performed (rounds, acquisitions, pairs, ...)    */
  uint64_t reserved[4];
} sp_stats;

typedef struct sp_device_info {
  char name[64];
  char arch[64];           /* gcnArchName                                                */
  uint32_t cu_count;
  uint32_t xcd_count;      /* from the XCC id register of a probe launch (0 = unknown)   */
  uint32_t wall_clock_khz; /* frequency of the constant-rate wall clock                  */
  uint32_t clock_khz;      /* peak shader clock                                          */
  uint64_t hbm_bytes;
  uint32_t max_threads_per_cu;
  uint32_t reserved[7];
} sp_device_info;

typedef struct sp_ctx sp_ctx;
typedef struct sp_barrier sp_barrier;
typedef struct sp_mutex sp_mutex;
typedef struct sp_sem sp_sem;
typedef struct sp_graph sp_graph;

/* ---- context -------------------------------------------------------------------------
 * sp_init: binds to HIP device `device`, reads its properties and probes the XCC count.
 * Errors: SP_E_HIP (no such device).  *out is owned by the caller until sp_fini.       */
int sp_init(int device, sp_ctx** out);
int sp_fini(sp_ctx* ctx);
int sp_device_info_get(const sp_ctx* ctx, sp_device_info* out);
/* Fills *p with the library's defaults.                                                */
void sp_params_default(sp_params* p);
/* Installs the default kind and parameters that *_DEFAULT resolves to for a primitive
 * class (0 barrier, 1 mutex, 2 semaphore) and contention bucket (0 = low: fewer than
 * 64 workgroups per resource -- per lock, per semaphore unit; for a barrier fewer than
 * 40 workgroups -- 1 = high).  Used by the autotuner (future-work item of
 * Section 7: tuning backoff per GPU and contention level).  Until a call replaces them,
 * the defaults are a tuning pass's winners on an MI355X: barrier central (low) and
 * per-XCD with 64 stamp copies (high); mutex spin with the paper's backoff, I_max 8
 * (low) and the CU-cohort lock (high; a run with fewer than two workgroups per CU and
 * lock runs the XCD-cohort lock with the same parameters instead); semaphore the per-XCD
 * chains (both; outside their range of K the chain kind, then the array kind; K = 1 with
 * at least two workgroups per CU SP_SEM_CU_LOCK).                                       */
int sp_set_default(sp_ctx* ctx, uint32_t primitive, uint32_t bucket, uint32_t kind,
                   const sp_params* p);
/* Reads back what *_DEFAULT resolves to for a primitive class and bucket (as above):
 * *kind (host) and, unless p is NULL, *p (host) with the "auto" fields resolved.
 * Errors: SP_E_INVAL (bad context, class or bucket, kind NULL).                         */
int sp_get_default(const sp_ctx* ctx, uint32_t primitive, uint32_t bucket, uint32_t* kind,
                   sp_params* p);
const char* sp_strerror(int code);
int sp_last_hip_error(const sp_ctx* ctx);
/* Writes the XCC id of every workgroup of a plain launch of nwg x lanes into
 * out (device, nwg uint32).                                                             */
int sp_probe_xcc(sp_ctx* ctx, uint32_t nwg, uint32_t lanes, uint32_t* out, void* stream);

/* ---- co-residency ----------------------------------------------------------------------
 * A barrier (and every workload whose workgroups wait for each other) needs all of its
 * workgroups resident at once (Section 5: the barrier is the primitive that needs
 * persistent threads).  Every such run refuses with SP_E_NORESIDENT when
 * sp_resident_per_cu(occupancy of its kernel) * CUs < workgroups.
 * sp_resident_per_cu: workgroups of one kernel that fit on one CU at once -- the smaller
 * of the runtime's figure (runtime_per_cu) and the budget that the kernel's own resource
 * use leaves on gfx950: 8 wavefronts per SIMD and 4 SIMDs per CU, 512 VGPRs per lane per
 * SIMD allocated in granules of 8, 160 KiB of LDS per CU allocated in 512-byte granules.
 * A kernel whose registers the runtime under-counts therefore cannot pass the check and
 * then wait forever for a workgroup that never became resident.  Pure host arithmetic
 * (no GPU call); returns 0 for lanes == 0 or a NULL argument.                            */
typedef struct sp_occupancy {
  uint32_t runtime_per_cu; /* hipOccupancyMaxActiveBlocksPerMultiprocessor                 */
  uint32_t vgprs;          /* VGPRs per lane (hipFuncAttributes.numRegs)                     */
  uint32_t lds_bytes;      /* LDS per workgroup (hipFuncAttributes.sharedSizeBytes + dynamic) */
  uint32_t lanes;          /* threads per workgroup                                          */
  uint32_t reserved[4];
} sp_occupancy;
uint32_t sp_resident_per_cu(const sp_occupancy* occ);

/* ---- device memory for callers without their own allocator ------------------------
 * sp_buffer_alloc: `bytes` of device memory on the context's GPU, zero-filled; the
 * caller frees it with sp_buffer_free.  sp_buffer_read / sp_buffer_write copy between
 * a device buffer and host memory (synchronous).  Errors: SP_E_INVAL, SP_E_HIP.          */
int sp_buffer_alloc(sp_ctx* ctx, uint64_t bytes, void** out);
int sp_buffer_free(sp_ctx* ctx, void* p);
int sp_buffer_read(sp_ctx* ctx, void* host_dst, const void* dev_src, uint64_t bytes);
int sp_buffer_write(sp_ctx* ctx, void* dev_dst, const void* host_src, uint64_t bytes);

/* ---- barrier (Section 5, Barrier; Table 4 Barrier()) ------------------------------------
 * sp_barrier_create: state for a barrier among exactly nwg workgroups (all must be
 * co-resident, Section 5: the barrier is the primitive that needs persistent threads).
 * Device state (counters, flags) is allocated and zeroed here and freed by destroy.
 * Errors: SP_E_INVAL (nwg == 0, bad kind or params), SP_E_HIP.                          */
int sp_barrier_create(sp_ctx* ctx, uint32_t kind, uint32_t nwg, const sp_params* p,
                      sp_barrier** out);
int sp_barrier_destroy(sp_barrier* b);
/* Hash-exchange workload: `rounds` barriers; in round r workgroup w stores
 * splitmix32(seed ^ (w << 16) ^ r) into slot (r & 1, w) of a 2 x nwg array, waits at the
 * barrier, then XORs slot (r & 1, (w + r) mod nwg) into its checksum.  The slot is
 * written by the workgroup's last thread and read by thread 64 (another wavefront when
 * lanes > 64), so the barrier must order plain stores and loads of different
 * wavefronts.  out_checksums: device, nwg uint32.  lanes: multiple of 64, <= 1024.
 * Errors: SP_E_INVAL, SP_E_NORESIDENT (nwg exceeds lanes-dependent co-residency),
 * SP_E_TIMEOUT, SP_E_HIP.  The state is reset before every run.                          */
int sp_barrier_run_hash(sp_barrier* b, uint32_t lanes, uint32_t rounds, uint32_t seed,
                        uint32_t* out_checksums, sp_stats* st, void* stream);
/* sp_barrier_info_get: after a run (call it once the run has returned), how the last
 * run synchronized.  For SP_BARRIER_XCD: xcd_path = 1 if every workgroup's registration
 * fit (at most ceil(nwg / XCDs) rounded up to 32 workgroups and 64 CUs with workgroups
 * per XCD), so the per-XCD protocol was used; otherwise the run fell back to the counter
 * tree (same results) and cu_overflow counts the registrations that did not fit.
 * near_placed is known from creation on.  misplaced counts workgroups
 * that did not run on XCD (id mod XCDs), the dispatcher's usual placement: the barrier
 * reads each workgroup's XCD and does not depend on it.                                 */
typedef struct sp_barrier_info {
  uint32_t kind;
  uint32_t nwg;
  uint32_t xcd_path;
  uint32_t misplaced;
  uint32_t cu_overflow;
  uint32_t near_placed;  /* SP_BARRIER_XCD, what sits in measured chunks: bit 0 arrival */
                         /* flags, bit 1 stamp copies, bit 2 per-CU release lines; 0 =     */
                         /* fixed layout                                                   */
  uint32_t reserved[2];
} sp_barrier_info;
int sp_barrier_info_get(sp_barrier* b, sp_barrier_info* out);
/* Comparator: the same workload with the kernel boundary as the barrier (one launch per
 * round, Section 2's "end one kernel and begin another"); graph != 0 replays the
 * rounds from a captured HIP graph instead of launching them one by one.               */
int sp_barrier_run_hash_launches(sp_ctx* ctx, uint32_t nwg, uint32_t lanes, uint32_t rounds,
                                 uint32_t seed, uint32_t graph, uint32_t* slots /*device, 2*nwg*/,
                                 uint32_t* out_checksums, sp_stats* st, void* stream);

/* ---- mutex (Section 5, Mutex; Algorithms 1-3; Table 4 Lock()/Unlock()) -------------------
 * sp_mutex_create: nlocks independent mutexes, each guarding words_per_lock uint32
 * words that the run's critical sections update.  Each lock's state sits on its own
 * pad_bytes-aligned line; a ticket mutex keeps ticket and turn on separate lines.
 * Errors: SP_E_INVAL, SP_E_HIP.                                                        */
int sp_mutex_create(sp_ctx* ctx, uint32_t kind, uint32_t nlocks, uint32_t words_per_lock,
                    const sp_params* p, sp_mutex** out);
int sp_mutex_destroy(sp_mutex* m);
/* Contention workload: total_acq acquisitions split over nwg workgroups (total / nwg
 * each, the first total mod nwg do one more).  Workgroup w's j-th acquisition first
 * waits key(w, j, 2) mod (max_delay_cyc + 1) shader clocks outside any lock, then locks
 * mutex key(w, j, 1) mod nlocks, adds one to each of its words with plain loads and
 * stores spread over the workgroup's lanes, and unlocks.  key(w, j, s) =
 * sm32(sm32(sm32(seed ^ s) ^ w) ^ j).  out_words: device, nlocks x words_per_lock
 * uint32 (lock-major), the final word values.  out_finish: device, nwg uint64 wall-clock
 * ticks at which each workgroup finished, or NULL.  Errors: SP_E_INVAL, SP_E_TIMEOUT,
 * SP_E_HIP.                                                                             */
int sp_mutex_run(sp_mutex* m, uint32_t nwg, uint32_t lanes, uint64_t total_acq,
                 uint32_t max_delay_cyc, uint32_t seed, uint32_t* out_words,
                 uint64_t* out_finish, sp_stats* st, void* stream);

/* ---- semaphore (Section 5, Semaphore; Algorithms 4-5; Table 4 Wait()/Post()) ------------
 * sp_sem_create: a counting semaphore with initial value K >= 1.  Algorithm 4 keeps one
 * word S = K + 1; Algorithm 5 keeps count, ticket and turn on separate lines.
 * Errors: SP_E_INVAL (K == 0; SP_SEM_CHAIN with K > 4096; SP_SEM_XCD_CHAIN with K below
 * the XCD count or above 4096 per XCD), SP_E_HIP.  A SP_SEM_DEFAULT semaphore whose
 * bucket names one of these runs the next kind whose range K is in: SP_SEM_XCD_CHAIN,
 * then SP_SEM_CHAIN, then SP_SEM_ARRAY; at K = 1 SP_SEM_CHAIN gives way to
 * SP_SEM_CU_LOCK in a run with at least two workgroups per CU.  SP_SEM_CU_LOCK needs
 * K = 1 (else SP_E_INVAL).                                                             */
int sp_sem_create(sp_ctx* ctx, uint32_t kind, uint32_t K, const sp_params* p, sp_sem** out);
int sp_sem_destroy(sp_sem* s);
/* Workload: total_pairs wait/post pairs split over nwg workgroups as in sp_mutex_run.
 * Inside, the leader (if track) increments an occupancy counter, raises its running
 * maximum, counts the admission, XORs sm32(seed ^ (w << 16) ^ j) into the workgroup's
 * checksum, holds key(w, j, 3) mod (max_hold_cyc + 1) shader clocks and decrements the
 * occupancy.  out_chk: device, nwg uint32.  out_state: device, 8 uint32 =
 * {max occupancy, S (Alg. 4) or count (Alg. 5), ticket, turn, admissions, count,
 * occupancy, unserved} (SP_SEM_COUNTERS, SP_SEM_ADAPTIVE: count stays 0, ticket = tickets
 * drawn, turn = posts made; SP_SEM_ARRAY, SP_SEM_CHAIN, SP_SEM_XCD_CHAIN: the same, the
 * low 32 bits of their 64-bit counters (summed over the XCDs' queues); SP_SEM_COHORT: ticket and turn stay 0, unserved = local tickets drawn and not
 * served, over every XCD's queue, 0 at rest).
 * out_data: device, K uint32 (zeroed by the call), or NULL; K <= 4096.  Guarded data:
 * each admission adds one to a word with a plain load and store made by the workgroup's
 * last thread -- for K = 1 to the one word, ordered only by the semaphore's acquire and
 * release; for K > 1 to the word of a slot of a pool of K that the holder claims with a
 * compare-and-swap (first try at key(w, j, 4) mod K) and returns with a release before it
 * posts.  The words sum to total_pairs (K = 1: the word equals it); which slot each
 * admission took is not unique.
 * Errors: SP_E_INVAL, SP_E_TIMEOUT, SP_E_HIP.                                           */
int sp_sem_run(sp_sem* s, uint32_t nwg, uint32_t lanes, uint64_t total_pairs,
               uint32_t max_hold_cyc, uint32_t seed, uint32_t track, uint32_t* out_chk,
               uint32_t* out_state, uint32_t* out_data, sp_stats* st, void* stream);

/* ---- condition variables (Section 7's future work) ------------------------------------
 * Device API in include/sp/cond.hpp: cond_wait (register, unlock, wait, relock; Mesa
 * semantics), cond_signal_leader, cond_broadcast_leader.
 * sp_cond_run_bounded_buffer: the classic use.  Workgroups [0, producers) put their share
 * of `items` values (producer w's j-th value is sm32(seed ^ (w << 16) ^ j); shares split
 * as in sp_mutex_run) into a ring of `capacity` words; the other nwg - producers
 * workgroups take their share.  One mutex of kind mutex_kind (SP_MUTEX_SPIN_CAS, _TICKET,
 * _SLEEP, _ARRAY or _COHORT) guards the ring; producers wait on "not full" while it holds capacity
 * values, consumers on "not empty" while it is empty, and each signals the other after
 * its put or take.  All nwg workgroups must be co-resident.  out: device, 6 uint64 =
 * {xor of the values taken, their sum, values taken, values put, most values ever in the
 * ring (<= capacity), values left (0)}.  out_taken: device, items uint32, or NULL: every
 * value taken, consumer i's in order at the start of its share (consumer shares split as
 * the producers' are), so the values taken can be compared one by one, as a multiset, with
 * the values put.  p: poll_sleep, pad_bytes, timeout_ms are used.
 * Errors: SP_E_INVAL, SP_E_NORESIDENT, SP_E_TIMEOUT, SP_E_HIP.                          */
int sp_cond_run_bounded_buffer(sp_ctx* ctx, uint32_t mutex_kind, uint32_t nwg, uint32_t producers,
                               uint32_t lanes, uint32_t capacity, uint64_t items, uint32_t seed,
                               const sp_params* p, uint64_t* out, uint32_t* out_taken,
                               sp_stats* st, void* stream);
/* sp_cond_run_bounded_buffer_noalloc: for callers that cannot allocate device memory --
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same workload, arguments, outputs and errors as sp_cond_run_bounded_buffer, but the
 * mutex, condition-variable and ring state live in a fixed workspace of 1 MiB (262144
 * uint32 words) in device memory that the library holds on each GPU it runs on until the
 * process ends; the call allocates and frees nothing (and so, unlike
 * sp_cond_run_bounded_buffer, may be recorded into a graph).  The workspace takes the
 * mutex state (6 lines, plus Q lines for SP_MUTEX_ARRAY with Q = nwg rounded up to a power
 * of two >= 64, or 32 lines for SP_MUTEX_COHORT; a line is pad_bytes), 8 lines of 128
 * bytes, the ring (capacity words) and 8 words per workgroup; a request that needs more
 * returns SP_E_RANGE (with the default 128-byte padding any nwg <= 2048 fits with a
 * capacity of up to 179000 words).  The call clears the part it uses before its kernel
 * runs.  Every call on
 * one GPU uses the same workspace: calls that overlap on one GPU (on different streams,
 * or from different host threads) race and their results are undefined.               */
int sp_cond_run_bounded_buffer_noalloc(sp_ctx* ctx, uint32_t mutex_kind, uint32_t nwg,
                                       uint32_t producers, uint32_t lanes, uint32_t capacity,
                                       uint64_t items, uint32_t seed, const sp_params* p,
                                       uint64_t* out, uint32_t* out_taken, sp_stats* st,
                                       void* stream);

/* ---- memory-system microbenchmarks (Section 3; Tables 1-3) ------------------------------
 * sp_bench_atomic: issuer u (a lane, or a wavefront's lane 0) performs ops_per_issuer
 * operations; its i-th targets word perm[(u + i) mod T] of buf, words stride_bytes
 * apart.  Issuers are numbered globally: u = (workgroup * waves + wave) * issuers per
 * wave + issuing lane.  ADD adds 1; CAS increments by a load/compare-and-swap loop; EXCH
 * writes sm32(sm32(seed ^ u) ^ i); LD loads; ST stores sm32(seed ^ t) to word t.  All
 * are agent-scope relaxed atomics.  The call first fills buf: 0 for ADD, CAS and ST,
 * sm32(seed ^ t) for EXCH and LD (word t at byte offset t * stride_bytes).
 * perm: device, T uint32.  buf: device, T * stride_bytes bytes.  out_sum: device,
 * 1 uint64 = sum of every returned value (for EXCH: plus the final word values).
 * Errors: SP_E_INVAL (T == 0, stride not a multiple of 4, lanes not a multiple of 64).  */
int sp_bench_atomic(sp_ctx* ctx, uint32_t op, uint32_t nwg, uint32_t lanes, uint32_t T,
                    uint32_t stride_bytes, uint32_t mode, uint64_t ops_per_issuer,
                    uint32_t seed, const uint32_t* perm, uint32_t* buf, uint64_t* out_sum,
                    sp_stats* st, void* stream);
/* sp_bench_paper12: the twelve tests of Section 3.  Each workgroup's leader performs
 * n_ops accesses to one word: word 0 for contentious tests, word w at byte offset
 * w * stride_bytes (the paper uses 256 B) for noncontentious ones.  Volatile = agent-
 * scope relaxed load or store; atomic read = add of 0; atomic write = exchange with 0.
 * buf: device, nwg * stride_bytes bytes, zeroed by the call.  out_sum: device, 1 uint64
 * (sum of loaded values, which stays 0).                                               */
int sp_bench_paper12(sp_ctx* ctx, uint32_t test, uint32_t nwg, uint32_t lanes, uint32_t n_ops,
                     uint32_t stride_bytes, uint32_t* buf, uint64_t* out_sum, sp_stats* st,
                     void* stream);
/* sp_bench_stream: reads `bytes` (multiple of 16) of buf with 16-byte loads (four in
 * flight per lane) and sums the uint32 words into out_sum (device, 1 uint64).  nwg = 0:
 * 32 workgroups of 256 lanes per CU.                                                    */
int sp_bench_stream(sp_ctx* ctx, const void* buf, uint64_t bytes, uint32_t nwg, uint32_t reps,
                    uint64_t* out_sum, sp_stats* st, void* stream);
/* sp_bench_clock: one lane spins for `ms` milliseconds of the constant-rate wall clock
 * and counts shader clocks meanwhile (clock64 against wall_clock64).  out: device, 2
 * uint64 scratch; *mhz (host) = the shader clock rate observed.  ms in [1, 10000].      */
int sp_bench_clock(sp_ctx* ctx, uint32_t ms, uint64_t* out, double* mhz, void* stream);
/* sp_bench_fence: the cost of agent-scope fences (Section 4's question of what memory
 * operations cost, asked of gfx950's cache maintenance).  nwg co-resident workgroups of
 * `lanes` threads; each leader stores to `lines` (<= 1024) 128-byte lines of its own,
 * waits for all workgroups at a start counter, then issues `reps` (1..1000) fences of
 * kind 0 = release (write back the XCD's dirty L2 lines) or 1 = acquire (invalidate the
 * CU's L1 and the XCD's non-coherent L2 lines).  out: device, 4 * nwg uint64: per
 * workgroup {shader clocks for the reps, wall clock at start, wall clock at end, 0}.
 * Errors: SP_E_INVAL, SP_E_NORESIDENT, SP_E_TIMEOUT, SP_E_HIP.                           */
int sp_bench_fence(sp_ctx* ctx, uint32_t kind, uint32_t nwg, uint32_t lanes, uint32_t reps,
                   uint32_t lines, uint64_t* out, sp_stats* st, void* stream);
/* sp_bench_copy: copies `bytes` (multiple of 16) from src to dst (device, disjoint) with
 * 16-byte loads and stores, `reps` times; the streaming read+write reference kernel.   */
int sp_bench_copy(sp_ctx* ctx, void* dst, const void* src, uint64_t bytes, uint32_t reps,
                  sp_stats* st, void* stream);
/* sp_bench_litmus: memory-model litmus tests on `pairs` pairs of workgroups that run on
 * different XCDs, `iters` trials per pair, both sides meeting every trial.
 * test 0, message passing: plain data store, flag store; flag poll, plain data load;
 *   forbidden: the data older than the flag.  variant 0 release + acquire fences (the
 *   primitives' idiom), 1 no acquire, 2 no release, 3 neither.
 * test 1, store buffering: each side stores its word then loads the other's (agent-scope
 *   relaxed accesses); forbidden: both loads old.  variant 0 an agent-scope sequentially
 *   consistent fence between store and load, 1 none.
 * out: device, 1 uint64 = forbidden outcomes observed (0 expected for variant 0).
 * Errors: SP_E_INVAL (pairs not in [1, 1024], unknown test or variant), SP_E_TIMEOUT,
 * SP_E_HIP.                                                                             */
int sp_bench_litmus(sp_ctx* ctx, uint32_t test, uint32_t variant, uint32_t pairs,
                    uint32_t iters, uint64_t* out, sp_stats* st, void* stream);
/* sp_bench_pingpong: two workgroups hand a token back and forth `rounds` times through
 * two agent-scope words, measuring the one-way coherence latency that bounds every
 * signal between workgroups (Section 4's latency question; Section 5's flags).
 * mode: bit 0 (SP_PINGPONG_FENCED) = release store and acquire fence around each hand-over
 * (a signal that publishes plain data); clear = relaxed agent-scope store and polling
 * only (a signal that publishes nothing, or coherently accessed data).  Bit 1
 * (SP_PINGPONG_SAME_XCD) = the partner is workgroup `xcd_count` instead of workgroup 1,
 * which the dispatcher's round robin over the XCDs places on workgroup 0's XCD (out[2..3]
 * report where they ran).  Other bits: SP_E_INVAL.
 * words: device, 2048 bytes, zeroed by the call.  out: device, 4 uint32 = {word written by
 * the partner (ends at 2 * rounds), word written by workgroup 0 (ends at 2 * rounds - 1),
 * XCC id of workgroup 0, XCC id of the partner}.  st->kernel_ms / (2 * rounds) is the
 * one-way latency.  Errors: SP_E_INVAL (rounds == 0, bad mode), SP_E_TIMEOUT, SP_E_HIP.  */
#define SP_PINGPONG_FENCED 1u
#define SP_PINGPONG_SAME_XCD 2u
int sp_bench_pingpong(sp_ctx* ctx, uint32_t rounds, uint32_t mode, uint32_t* words,
                      uint32_t* out, sp_stats* st, void* stream);

/* ---- recorded batches (HIP graphs) ---------------------------------------------------
 * Section 7 leaves the tuning of these primitives per GPU and contention level to future
 * work; an autotuner times many short runs, and a fused sequence of persistent kernels is
 * cheaper to replay from a graph than to launch call by call.
 * sp_graph_begin: starts recording on `stream` (NULL: a stream owned by the context) and
 * returns the stream to record on in *capture_stream.  Until sp_graph_end, every
 * sp_barrier_run_hash, sp_mutex_run, sp_sem_run and sp_bench_* call made with that stream
 * records its state resets (fill kernels, never memset nodes) and kernels instead of
 * running them: it returns SP_OK at once, zeroes *st and leaves its outputs unwritten.
 * Cooperative launches (SP_BARRIER_GRID_SYNC, sp_params.cooperative) and the graph mode
 * of sp_barrier_run_hash_launches cannot be recorded (SP_E_INVAL), nor can calls that
 * allocate device memory: a ring or array mutex's run with more workgroups than any run
 * before it (run it once outside the recording), sp_bench_litmus, sp_bench_fence and
 * sp_cond_run_bounded_buffer, or that return a host result (sp_bench_clock).
 * sp_graph_end: stops recording and instantiates the graph (*out, owned by the caller).
 * sp_graph_launch: clears the watchdog word, replays the graph `replays` times back to
 * back on `stream`, times all replays with HIP events, waits, and reports SP_E_TIMEOUT if
 * any recorded kernel's watchdog expired.  st->kernel_ms covers every replay, st->ops =
 * replays.  Outputs of the recorded calls hold the last replay's results; the state
 * objects and buffers they name must outlive the graph.
 * Errors: SP_E_INVAL, SP_E_HIP (capture or instantiation failed), SP_E_TIMEOUT.          */
int sp_graph_begin(sp_ctx* ctx, void* stream, void** capture_stream);
int sp_graph_end(sp_ctx* ctx, void* capture_stream, sp_graph** out);
int sp_graph_launch(sp_graph* g, uint32_t replays, sp_stats* st, void* stream);
int sp_graph_destroy(sp_graph* g);

/* ---- persistent serving queue -------------------------------------------------------
 * The paper motivates inter-workgroup primitives with work queues that persistent
 * workgroups drain (Sections 1-2) and leaves the tuning of such designs to future work
 * (Section 7).  Workload: requests r = 0 .. n-1 arrive at host times t_arr_s[r] seconds
 * after the start (non-decreasing).  Request r computes the hash chain h_0 = seed ^ r,
 * h_{i+1} = splitmix32(h_i), out[r] = h_{L[r]}, and while it runs holds
 * ceil(nbytes[r] / unit_bytes) units of a workspace budget of budget_units units.
 *
 * sp_serve_run: one persistent kernel of nwg workgroups (all co-resident) drains a ring
 * of request descriptors in pinned host memory.  The host writes a descriptor when the
 * request arrives and publishes the ring's tail; a workgroup claims the next request with
 * one fetch-and-add, waits for its arrival, is admitted by a weighted fetch-and-add
 * semaphore over the budget (FIFO; include/sp/semaphore.hpp), computes the chain in its
 * leader lane, returns its units and stores a completion flag into pinned host memory.
 * sp_serve_run_launch_per_request: the comparator.  For each request (batch == 1) the
 * host launches one single-workgroup kernel at its arrival time, round robin over
 * `streams` streams, after admitting it against the same budget on the host; with
 * batch > 1 one launch covers every request that has arrived since the previous launch
 * (at most batch of them, one workgroup each).
 *
 * Both: latency[r] = host time at which the host saw request r's completion flag minus
 * its arrival time; the same host thread observes completions in both modes.  Inputs
 * L, nbytes, t_arr_s: host, n entries.  out: host, n uint32.  lat_us: host, n doubles,
 * or NULL.  The call allocates its ring, flags and device buffers, runs the whole stream
 * and returns when every request completed.  Errors: SP_E_INVAL (n == 0, a request
 * needing more units than the budget, t_arr_s decreasing, bad sizes),
 * SP_E_NORESIDENT (nwg not co-resident), SP_E_TIMEOUT (watchdog or host deadline),
 * SP_E_HIP.                                                                              */
typedef struct sp_serve_cfg {
  uint32_t nwg;          /* sp_serve_run: persistent workgroups                            */
  uint32_t lanes;        /* threads per workgroup, multiple of 64 (the leader lane works)  */
  uint32_t ring_slots;   /* descriptor ring, power of two in [64, 2^24] (0 = 65536)       */
  uint32_t budget_units; /* K: workspace units that may be held at once, in [1, 2^30)      */
  uint64_t unit_bytes;   /* bytes per budget unit (0 = 65536)                              */
  uint32_t seed;
  uint32_t poll_sleep;   /* s_sleep units between polls of the workgroup next in line     */
  uint32_t far_sleep;    /* cap on the s_sleep units of workgroups further back (0 = 64)   */
  uint32_t timeout_ms;   /* device watchdog and host deadline beyond the last arrival      */
                         /* (0 = 20000)                                                    */
  uint32_t streams;      /* launch comparator: streams used round robin, 1..4 (0 = 1)      */
  uint32_t batch;        /* launch comparator: requests per launch at most (0 = 1)         */
  uint32_t track;        /* 1: also track the maximum units in use (three more atomics)    */
  uint32_t graph_batch;  /* launch comparator: G in [1, 4096] = replay a HIP graph of G     */
                         /* one-workgroup kernel nodes (no dependencies between them)     */
                         /* once G requests have arrived; each node claims the next       */
                         /* request from a device counter.  A partial batch is launched   */
                         /* as one kernel when the budget or the ring stalls publishing,  */
                         /* and at the end.  0 = off; batch must then be 0 or 1           */
  uint32_t reserved[4];
} sp_serve_cfg;

typedef struct sp_serve_result {
  double wall_s;             /* first arrival to last observed completion                 */
  double p50_us, p99_us;     /* latency percentiles (nearest rank)                        */
  double mean_us, max_us;
  double req_per_s;          /* n / wall_s                                                */
  double publish_lag_max_us; /* worst delay of a publish or launch behind its arrival     */
  uint64_t completed;
  uint64_t launches;         /* kernel launches (1 for the persistent queue)              */
  uint32_t max_units_in_use; /* with track: the maximum seen (<= budget_units)            */
  uint32_t device_error;
  uint64_t units_issued;     /* final weighted-semaphore counters (persistent queue):     */
  uint64_t units_released;   /* both equal the sum of every request's units               */
  uint64_t reserved[2];
} sp_serve_result;

int sp_serve_run(sp_ctx* ctx, const sp_serve_cfg* cfg, uint32_t n, const uint32_t* L,
                 const uint64_t* nbytes, const double* t_arr_s, uint32_t* out, double* lat_us,
                 sp_serve_result* res);
int sp_serve_run_launch_per_request(sp_ctx* ctx, const sp_serve_cfg* cfg, uint32_t n,
                                    const uint32_t* L, const uint64_t* nbytes,
                                    const double* t_arr_s, uint32_t* out, double* lat_us,
                                    sp_serve_result* res);

#ifdef __cplusplus
}
#endif
#endif /* SP_H */
