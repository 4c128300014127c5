/*
 * Serial reference model of the per-cycle step of a bufferless deflection-routed
 * 2D-mesh chip multicore with a statically homed, set-associative LRU L2.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the HIP path is checked against.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the HIP library.
 *
 * Paper: Kumar & Sahu, "Bufferless NOC Simulation of Large Multicore System on GPU
 * Hardware" (arXiv 1508.03235).  The serial simulator there runs three phases per
 * cycle over every router (Sec. 7.1): memory access (phase one), oldest-first
 * deflection arbitration (phase two), link traversal / ejection / injection
 * (phase three).  This oracle keeps that three-loop structure.
 */
#ifndef NOCSIM_ORACLE_H
#define NOCSIM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Model parameters (one simulated chip). */
typedef struct {
  int32_t width, height;       /* mesh columns (x) and rows (y) */
  uint32_t seed_lo, seed_hi;   /* Philox key */
  int32_t l1_sets, l1_ways;    /* private L1: powers of two, ways <= 8 */
  int32_t l2_sets, l2_ways;    /* L2 slice per tile */
  int32_t l1_lat;              /* cycles from an L1 miss to its follow-up (>= 1) */
  int32_t mem_lat;             /* off-chip latency of an L2 miss (>= 1) */
  uint32_t op_thr;             /* memory op issued iff draw < op_thr */
  uint32_t shared_thr;         /* shared region iff draw < shared_thr (when private_lines > 0) */
  uint32_t bg_thr;             /* background flit generated iff draw < bg_thr */
  int32_t shared_lines;        /* lines [0, shared_lines) form the shared region */
  int32_t private_lines;       /* per-tile private region size (0 = no private region) */
  int32_t flags;               /* model variants, ORACLE_FLAG_* below (0 = the base model) */
  int32_t reply_flits;         /* flits of a reply packet, 1..16 (0 counts as 1) */
  int32_t router_delay;        /* cycles a flit takes per hop, 1..8 (0 counts as 1): a flit that
                                  arrives at a router waits router_delay - 1 cycles in its
                                  pipeline before it is arbitrated */
  int32_t mig_threshold;       /* LSPD migration (Sec. 3.3): the length N of each L2 way's history
                                  of its last accessors; a block moves to a remote tile that made
                                  more than half of them (0 = never, <= 16) */
} oracle_config;

/* Model variants: each bit replaces one reading of the base model by a more literal one.
   AGE_DEFLECT: a flit's priority is the number of times it has been deflected so far (more
     first; 0 at injection), ties by (injection cycle, source) (Sec. 4.2, Sec. 6.2.1, Sec. 7.1
     phase two).  The base model ranks by injection cycle alone.
   HIT_UNDER_MISS: a core with a miss outstanding keeps drawing ops; an L1 hit completes at
     once, a second miss waits until the first is filled and is then looked up again
     (Sec. 3.5).  The base model's core issues nothing while a miss is outstanding.
   INJECT_DELAY: a request or reply made in a cycle can enter the network from the next cycle
     on (the router's injection register, filled in phase three: Sec. 6.2.1, Sec. 7.1).  The
     base model injects it in the cycle it is made.
   LSPD: the logically shared, physically distributed L2 with a directory (Sec. 3.2, 3.4,
     6.2.2, Table 1): a block lives in the slice of the core that brought it from memory (local
     placement); an L1 miss looks in the core's own slice, then asks the directory (DA), which
     answers with the owner or a negative reply (DR); on a negative reply the block comes from
     memory into the local slice, otherwise the core asks the owner (RA) for it.  An owner that
     no longer holds the block answers with a trap and the core asks the directory again; a
     slice that evicts a block sends the directory an eviction notice.  Directory entries are
     kept in a location array indexed by line; the entry of a line belongs to the line's
     directory slice, line mod N, or with LSPD_CENTRAL to the one tile at the mesh centre.
     The base model homes each line statically at slice line mod N.  With mig_threshold > 0 a
     block migrates (Sec. 3.3): each L2 way keeps its last mig_threshold accessors; when a remote
     tile has made more than half of them the owner sends it the block (16 flits, Table 1) and
     keeps serving it from its own copy until the receiver's arrival notice comes back; then it
     drops the copy and keeps a forwarding pointer, answering a request that still reaches it
     with a redirection (1 flit).  The receiver claims the directory entry and its op
     completes with the directory's acknowledgement (a block under claim does not move on). */
enum {
  ORACLE_FLAG_AGE_DEFLECT = 1, ORACLE_FLAG_HIT_UNDER_MISS = 2, ORACLE_FLAG_INJECT_DELAY = 4,
  ORACLE_FLAG_LSPD = 8, ORACLE_FLAG_LSPD_CENTRAL = 16
};

enum {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,
  ORACLE_ENOMEM = -2,
  ORACLE_EINVARIANT = -4
};

/* Statistics block: 48 int64 counters.  Indices: */
enum {
  OS_CYCLES = 0,
  OS_INJ_REQ = 1, OS_INJ_REPLY = 2, OS_INJ_BG = 3,
  OS_EJ_REQ = 4, OS_EJ_REPLY = 5, OS_EJ_BG = 6,
  OS_LAT_REQ = 7, OS_LAT_REPLY = 8, OS_LAT_BG = 9,
  OS_LAT_MAX = 10,
  OS_TRAVERSALS = 11, OS_DEFLECTIONS = 12,
  OS_OPS_ISSUED = 13, OS_OPS_DONE = 14, OS_OP_LAT = 15,
  OS_L1_HIT = 16, OS_L1_MISS = 17, OS_L2_HIT = 18, OS_L2_MISS = 19,
  OS_REQ_MADE = 20, OS_REQ_RECV = 21, OS_REPLY_SENT = 22, OS_REPLY_RECV = 23,
  OS_INJ_BLOCKED = 24, OS_BG_GEN = 25, OS_OP_LAT_MAX = 26,
  OS_DIR_ACCESS = 27, OS_DIR_NACK = 28, OS_TRAP = 29, OS_DIR_EVICT = 30, /* LSPD directory */
  OS_HIST = 32, /* 16 bins: floor(log2(latency)), last bin open */
  OS_MIGRATE = 48, OS_REDIRECT = 49, /* LSPD migration: blocks moved, requests redirected */
  OS_COUNT = 64
};

typedef struct oracle_sim oracle_sim;

/* zipf_* are quantile tables of zipf_k + 1 entries (zipf_k = 65536), copied. */
int oracle_create(const oracle_config* cfg, const uint32_t* zipf_shared, const uint32_t* zipf_private,
                  int32_t zipf_k, oracle_sim** out);
/* Runs n cycles.  digests (may be NULL) receives one 64-bit state digest per cycle.
   check != 0 verifies the model invariants after every cycle (ORACLE_EINVARIANT on failure). */
int oracle_step(oracle_sim* s, int64_t n, uint64_t* digests, int32_t check);
int oracle_stats(const oracle_sim* s, int64_t* out /* OS_COUNT */);
int64_t oracle_cycle(const oracle_sim* s);
size_t oracle_dump_words(const oracle_sim* s);
int oracle_dump(const oracle_sim* s, int32_t* buf, size_t words);
int oracle_load(oracle_sim* s, const int32_t* buf, size_t words);
int oracle_force_op(oracle_sim* s, int32_t tile, int32_t line);
int oracle_force_bg(oracle_sim* s, int32_t tile, int32_t dst);
int oracle_set_rates(oracle_sim* s, uint32_t op_thr, uint32_t bg_thr);
/* 1 when no flit is in flight, every core is idle, and every queue is empty. */
int oracle_quiescent(const oracle_sim* s);
const char* oracle_invariant_msg(const oracle_sim* s);
void oracle_destroy(oracle_sim* s);

/* Stand-alone pieces, exported for unit tests. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Zipf ranks of n uniform draws through a quantile table (the sampler used in phase one). */
void oracle_zipf_ranks(const uint32_t* table, const uint32_t* u, int64_t n, int32_t* out);
/* Arbitration of one router: n flits given by (dst, inj, src) and, for the AGE_DEFLECT
   variant, their deflection counts (age = NULL: the base model's injection-time priority);
   writes for each flit the port it takes (0..3 = N,S,E,W, 4 = eject) and whether it was
   deflected. */
int oracle_arbitrate(int32_t width, int32_t height, int32_t tile, int32_t n, const int32_t* dst,
                     const int32_t* inj, const int32_t* src, const int32_t* age, int32_t* port,
                     int32_t* deflected);

#ifdef __cplusplus
}
#endif
#endif
