/*
 * Serial reference model (oracle) of the per-cycle step of a bufferless
 * deflection-routed 2D-mesh chip multicore with a statically homed L2.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the HIP library.  Plain C, one thread, written to be read against the
 * paper (Kumar & Sahu, arXiv 1508.03235):
 *
 *   - the cycle loop and its three phases over every router: Sec. 7.1 (serial
 *     version; phase one = memory access, phase two = arbitration, phase three
 *     = traversal, ejection, injection);
 *   - bufferless deflection routing, oldest first, X-then-Y productive
 *     preference kept after deflection, injection only into a free input:
 *     Sec. 4.2-4.3 and Sec. 6.2.1;
 *   - private L1 and a logically shared, physically distributed L2 with one
 *     copy of each line: Sec. 3.1; request policy (no miss under a miss):
 *     Sec. 3.5; statistics (requests made/received, replies sent/received,
 *     hits and misses): Sec. 6.2.2.
 *
 * Where the paper is silent or ambiguous the oracle follows the readings listed
 * in the design notes (static home = line mod N, injection-time age, one eject
 * per cycle, per-home reply queues as intrusive lists, Philox4x32-10 draws keyed
 * by (seed; cycle, tile, stream)).  Three more literal readings can be switched
 * on as variants (ORACLE_FLAG_*): priority by deflection count, hits served
 * under an outstanding miss, and injection through the router's injection
 * register one cycle after a flit is made; a router delay stretches every hop;
 * and the paper's own L2 model, the LSPD cache with a directory (Sec. 3.2,
 * 3.4, 6.2.2), replaces the static homes, optionally with block migration and
 * redirection (Sec. 3.3).  Every function below names the passage it follows.
 *
 * Parity pins: the Philox generator is pinned to published known-answer
 * vectors; routing to closed-form zero-load latencies and hand traces; the
 * arbitration to brute-force rule checks; the caches to a textbook LRU list and
 * to Mattson stack distances; conservation and drain to the equalities the
 * paper's statistics table shows (requests made = received, replies sent =
 * received).  The full-system counts themselves are not printed in the paper.
 */
#include "nocsim_oracle.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---- fixed encodings --------------------------------------------------------------- */
/* flit kinds; with the LSPD directory a request-class flit of kind K_DIR is a directory access
   or an eviction notice, and a K_REPLY flit with the control bit set is a directory reply or a
   trap (the control bit is bit 31 of the injection-cycle word, which cycles < 2^31 leave free) */
enum { K_REQ = 0, K_REPLY = 1, K_BG = 2, K_DIR = 3 };
enum { ST_IDLE = 0, ST_L1MISS = 1, ST_SEND = 2, ST_WAIT = 3, ST_FILL = 4, /* core states */
       ST_SEND_DA = 5, ST_SEND_RA = 6, ST_FILL_MEM = 7,                     /* LSPD only */
       ST_FILL_MIG = 8 };                                                   /* a migrated block */
#define CTL_BIT 0x80000000u
/* codes of the directory's and an owner's answers (queue node line word; sent as code + 4):
   the directory's acknowledgement of an ownership claim, a flit of a migrating block, a trap,
   a negative directory answer, or an owner tile >= 0 */
enum { CODE_ACK = -4, CODE_MIG = -3, CODE_TRAP = -2, CODE_NACK = -1 };
#define CODE_BASE 4
/* request types at a slice's service input (the high byte of C_L2Q): remote access, directory
   access, eviction notice, ownership claim, a migrated block's arrival at its new owner */
enum { Q_RA = 0, Q_DA = 1, Q_EV = 2, Q_CLAIM = 3, Q_ARRIVED = 4 };
/* migration (Sec. 3.3): a block moves as 16 flits (Table 1, L2 block migration); a queued reply
   carries this bit on its line word when it is a migration.  Each L2 way keeps the list of its
   last `mig` accessors, most recent first (-1 = none yet).  While a block this slice sends away
   is on its way, the slice's forwarding destination carries MIG_TRANSIT. */
/* a flit kind in the top two bits of the info word (shifted unsigned: kind 2 reaches bit 31) */
#define KIND_BITS(k) ((int32_t)((uint32_t)(k) << 30))
#define MIG_FLITS 16
#define MIG_MARK 0x40000000
#define MIG_TRANSIT 0x40000000
enum { PN = 0, PS = 1, PE = 2, PW = 3, PX = 4 };                        /* ports, 4 = eject */
/* per-tile core record (20 words); C_NEXT, C_READY, C_NLINE and C_NSENT are the tile's queue
   node as a requester, written by its home while it waits there */
enum {
  C_STATE = 0, C_WAKE = 1, C_LINE = 2, C_ISSUE = 3, C_L2Q = 4, C_L2Q_LINE = 5,
  C_HIT_H = 6, C_HIT_T = 7, C_MISS_H = 8, C_MISS_T = 9, C_BG = 10,
  C_NEXT = 11, C_READY = 12, C_NLINE = 13, C_FLINE = 14, C_FDST = 15,
  C_RCV = 16,   /* flits of the awaited reply received so far */
  C_NSENT = 17, /* flits of this tile's reply already injected by its home */
  C_DLINE = 18, /* hit under miss: line of the op waiting for the outstanding miss, -1 = none */
  C_DISSUE = 19,/* hit under miss: the waiting op's issue cycle */
  C_TARGET = 20,/* LSPD: the owner a remote-access request goes to */
  C_EV = 21,    /* LSPD: line whose eviction notice waits for injection, -1 = none */
  C_DSUM_LO = 22, C_DSUM_HI = 23, /* LSPD: checksum of the directory entries this tile keeps */
  C_CLAIM = 24, /* migration: line whose ownership claim waits for injection, -1 = none */
  C_FWD_LINE = 25, C_FWD_DST = 26, /* migration: the last block this slice gave away (or is giving
                                      away: MIG_TRANSIT), and to whom */
  C_NOTE = 27,  /* migration: the tile a block that migrated here came from, to be told of its
                   arrival; -1 = none */
  C_WORDS = 28
};
/* flit record: destination, injection cycle, source, kind<<30 | line, and the number of times
   the flit has been deflected (kept for the AGE_DEFLECT variant, 0 otherwise); the first four
   words are the flit as the canonical dump shows it */
enum { F_DST = 0, F_INJ = 1, F_SRC = 2, F_INFO = 3, F_AGE = 4, F_WORDS = 5 };
#define SLOT_WORDS (4 * F_WORDS) /* the four input slots of a tile */
#define AGE_LIMIT 65535          /* deflections a flit may take before the run is declared livelocked */
#define LINE_MASK 0x3FFFFFFF
#define DUMP_MAGIC 0x4E4F4353
#define DUMP_HEADER 16

struct oracle_sim {
  oracle_config cfg;
  int32_t W, H, N;
  int32_t reply_flits;   /* flits per reply packet */
  int32_t delay;         /* router delay D >= 1: cycles per hop */
  int32_t lspd;          /* 0 static homes; 1 directory interleaved by line; 2 central directory */
  int32_t dir_center;    /* the central directory's tile */
  int64_t lines;         /* size of the line space (location array entries) */
  int32_t* loc;          /* LSPD location array: [lines] owner tile or -1 */
  int32_t* l2h;          /* migration: [N][S2][W2][mig] the last accessors of each L2 way */
  int32_t mig;           /* migration: length of a block's access history (0 = no migration) */
  int32_t* seen;         /* [lines] scratch of the one-copy check */
  int32_t* scratch;      /* [2N], invariant checks */
  int64_t cycle;
  int32_t zk;
  uint32_t* zs;          /* shared-region quantile table, zk+1 entries */
  uint32_t* zp;          /* private-region quantile table */
  int32_t* link[2];      /* [N][4 ports][F_WORDS]: input slots, double buffered by cycle parity */
  int32_t* pipe;         /* [D-1][N][4 ports][F_WORDS]: flits that arrived at a router and wait for
                            arbitration; ring entry (a mod (D-1)) holds those arbitrated at cycle a */
  int32_t* core;         /* [N][C_WORDS] */
  int32_t* l1;           /* [N][S1][W1], most recently used first, -1 = invalid */
  int32_t* l2;           /* [N][S2][W2] */
  int64_t stats[OS_COUNT];
  /* scratch of one cycle */
  uint32_t* rnd;         /* [N][4] the tile's main draw of this cycle */
  int32_t* outp;         /* [N][4 ports][F_WORDS] flits routed out this cycle */
  int32_t* ej;           /* [N][F_WORDS] flit ejected this cycle (dst < 0: none) */
  int32_t* oldest_ok;    /* [N] 1 if the router's oldest flit was ejected or moved productively */
  int32_t check;
  int32_t bad;
  char msg[256];
};

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from that paper ------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* key schedule (Weyl) increments */
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const oracle_sim* s, int64_t cycle, int32_t tile, uint32_t stream, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)cycle, (uint32_t)tile, stream, 0u};
  uint32_t key[2] = {s->cfg.seed_lo, s->cfg.seed_hi};
  oracle_philox4x32_10(ctr, key, out);
}

static uint64_t mix64(uint64_t z) { /* SplitMix64 finalizer (Steele, Lea, Flood 2014) */
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Zipf rank from a quantile table: bucket = high 16 bits, linear position inside it from
   the low 16 bits. */
static int32_t zipf_rank(const uint32_t* q, uint32_t u) {
  uint32_t b = u >> 16, f = u & 0xFFFFu;
  uint32_t lo = q[b], hi = q[b + 1];
  return (int32_t)(lo + (uint32_t)(((uint64_t)f * (uint64_t)(hi - lo)) >> 16));
}

void oracle_zipf_ranks(const uint32_t* table, const uint32_t* u, int64_t n, int32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = zipf_rank(table, u[i]);
}

/* ---- geometry (Sec. 6.2.1: Input[0..3] = north, south, east, west) ---------------- */
static int port_valid(const oracle_sim* s, int32_t t, int p) {
  int32_t x = t % s->W, y = t / s->W;
  switch (p) {
    case PN: return y > 0;
    case PS: return y < s->H - 1;
    case PE: return x < s->W - 1;
    default: return x > 0;
  }
}
static int32_t neighbour(const oracle_sim* s, int32_t t, int p) {
  switch (p) {
    case PN: return t - s->W;
    case PS: return t + s->W;
    case PE: return t + 1;
    default: return t - 1;
  }
}
static int opposite(int p) { return p ^ 1; } /* N<->S, E<->W */

/* ---- caches: a set is a list of line tags, most recently used first --------------- */
/* Touch `line` in a set of `ways` tags: on a hit move it to the front; on a miss insert it at
   the front when `insert`, dropping the last entry (an invalid way if one exists, else the
   least recently used one).  Returns 1 on a hit.  Local victim selection: Sec. 3.4. */
static int cache_touch(int32_t* set, int ways, int32_t line, int insert) {
  for (int i = 0; i < ways; ++i) {
    if (set[i] == line) {
      for (int j = i; j > 0; --j) set[j] = set[j - 1];
      set[0] = line;
      return 1;
    }
  }
  if (insert) {
    for (int j = ways - 1; j > 0; --j) set[j] = set[j - 1];
    set[0] = line;
  }
  return 0;
}

static void check_set(oracle_sim* s, const int32_t* set, int ways, const char* what, int32_t tile) {
  for (int i = 0; i < ways; ++i) {
    if (set[i] < 0) {
      for (int j = i + 1; j < ways; ++j)
        if (set[j] >= 0 && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "%s tile %d: valid way after invalid", what, tile); }
      continue;
    }
    for (int j = i + 1; j < ways; ++j)
      if (set[j] == set[i] && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "%s tile %d: duplicate tag %d", what, tile, set[i]); }
  }
}

static int32_t* l1_set(oracle_sim* s, int32_t t, int32_t line) {
  int32_t set = line & (s->cfg.l1_sets - 1);
  return s->l1 + ((size_t)t * s->cfg.l1_sets + set) * s->cfg.l1_ways;
}
static int32_t* l2_set(oracle_sim* s, int32_t t, int32_t line) {
  /* a static home holds only its own lines: index by line / N; an LSPD slice holds any line */
  int32_t set = (s->lspd ? line : line / s->N) & (s->cfg.l2_sets - 1);
  return s->l2 + ((size_t)t * s->cfg.l2_sets + set) * s->cfg.l2_ways;
}

/* L2 lookup at home slice t: install on a miss (the block arrives from memory after
   mem_lat cycles; one copy per line, Sec. 3.1).  Returns 1 on a hit. */
static int l2_lookup(oracle_sim* s, int32_t t, int32_t line) {
  int32_t* set = l2_set(s, t, line);
  int hit = cache_touch(set, s->cfg.l2_ways, line, 1);
  if (hit) s->stats[OS_L2_HIT]++; else s->stats[OS_L2_MISS]++;
  if (s->check) {
    check_set(s, set, s->cfg.l2_ways, "L2", t);
    if (line % s->N != t && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "L2 slice %d got line %d", t, line); }
  }
  return hit;
}

/* ---- per-home reply queues: FIFOs threaded through the requesters' node words ------ */
static void list_append(oracle_sim* s, int32_t home, int head_w, int tail_w, int32_t rq, int32_t ready, int32_t line) {
  int32_t* h = s->core + (size_t)home * C_WORDS;
  int32_t* n = s->core + (size_t)rq * C_WORDS;
  n[C_NEXT] = -1;
  n[C_READY] = ready;
  n[C_NLINE] = line;
  n[C_NSENT] = 0;
  if (h[tail_w] >= 0) s->core[(size_t)h[tail_w] * C_WORDS + C_NEXT] = rq;
  else h[head_w] = rq;
  h[tail_w] = rq;
}
static int32_t list_pop(oracle_sim* s, int32_t home, int head_w, int tail_w) {
  int32_t* h = s->core + (size_t)home * C_WORDS;
  int32_t rq = h[head_w];
  h[head_w] = s->core[(size_t)rq * C_WORDS + C_NEXT];
  if (h[head_w] < 0) h[tail_w] = -1;
  return rq;
}

/* The line a drawn op addresses: the shared region, or the tile's private region (the
   synthetic stand-in for the per-core address traces of Sec. 6.2.3). */
static int32_t drawn_line(const oracle_sim* s, int32_t t, const uint32_t* r) {
  if (s->cfg.private_lines > 0 && r[1] >= s->cfg.shared_thr)
    return s->cfg.shared_lines + t * s->cfg.private_lines + zipf_rank(s->zp, r[2]);
  return zipf_rank(s->zs, r[2]);
}

/* Cycles between making a flit and its first chance to enter the network: 1 when the
   router's injection register sits in between (INJECT_DELAY), else 0. */
static int32_t inject_delay(const oracle_sim* s) { return (s->cfg.flags & ORACLE_FLAG_INJECT_DELAY) ? 1 : 0; }

/* ---- LSPD directory (Sec. 3.2, Sec. 6.2.2): the location array ------------------------ */
static int32_t dir_of(const oracle_sim* s, int32_t line) { return s->lspd == 2 ? s->dir_center : line % s->N; }
static uint64_t dir_term(int32_t line, int32_t owner) {
  return mix64(((uint64_t)(uint32_t)line << 32) | (uint32_t)owner);
}
/* Sets the directory entry of `line`, keeping the directory tile's checksum of its entries
   (the sum of dir_term over the entries that name an owner). */
static void dir_set(oracle_sim* s, int32_t line, int32_t owner) {
  int32_t* k = s->core + (size_t)dir_of(s, line) * C_WORDS;
  uint64_t sum = ((uint64_t)(uint32_t)k[C_DSUM_HI] << 32) | (uint32_t)k[C_DSUM_LO];
  if (s->loc[line] >= 0) sum -= dir_term(line, s->loc[line]);
  if (owner >= 0) sum += dir_term(line, owner);
  s->loc[line] = owner;
  k[C_DSUM_LO] = (int32_t)(uint32_t)sum;
  k[C_DSUM_HI] = (int32_t)(uint32_t)(sum >> 32);
}
/* A slice evicted `line` (its eviction notice, or at once when it keeps the entry itself): the
   entry names that slice until then (a slice that received a block by migration evicts nothing
   before the directory has acknowledged its claim). */
static void dir_evicted(oracle_sim* s, int32_t line, int32_t who) {
  if (s->check && s->loc[line] != who && !s->bad) {
    s->bad = 1;
    snprintf(s->msg, sizeof s->msg, "eviction notice of %d for line %d named %d", who, line, s->loc[line]);
  }
  dir_set(s, line, -1);
  s->stats[OS_DIR_EVICT]++;
}

/* L2 ways of an LSPD slice with their access histories (hist = NULL without migration; `mig`
   words per way, kept in the ways' order): find, move to the front, remove, insert at the front
   (returns the dropped last way; the new way's history starts empty). */
static int32_t* l2_hist(oracle_sim* s, int32_t t, int32_t line) {
  if (!s->mig) return NULL;
  return s->l2h + ((size_t)t * s->cfg.l2_sets + (line & (s->cfg.l2_sets - 1))) * s->cfg.l2_ways * s->mig;
}
static int l2_find(const int32_t* set, int ways, int32_t line) {
  for (int i = 0; i < ways; ++i)
    if (set[i] == line) return i;
  return -1;
}
static void hist_copy(int32_t* dst, const int32_t* src, int mig) {
  for (int m = 0; m < mig; ++m) dst[m] = src[m];
}
static void hist_clear(int32_t* h, int mig) {
  for (int m = 0; m < mig; ++m) h[m] = -1;
}
static void l2_front(int32_t* set, int32_t* hist, int mig, int i) {
  int32_t tag = set[i], h[16];
  if (hist) hist_copy(h, hist + i * mig, mig);
  for (int j = i; j > 0; --j) {
    set[j] = set[j - 1];
    if (hist) hist_copy(hist + j * mig, hist + (j - 1) * mig, mig);
  }
  set[0] = tag;
  if (hist) hist_copy(hist, h, mig);
}
static void l2_remove(int32_t* set, int32_t* hist, int mig, int ways, int i) {
  for (int j = i; j < ways - 1; ++j) {
    set[j] = set[j + 1];
    if (hist) hist_copy(hist + j * mig, hist + (j + 1) * mig, mig);
  }
  set[ways - 1] = -1;
  if (hist) hist_clear(hist + (ways - 1) * mig, mig);
}
static int32_t l2_insert(int32_t* set, int32_t* hist, int mig, int ways, int32_t line) {
  int32_t victim = set[ways - 1];
  for (int j = ways - 1; j > 0; --j) {
    set[j] = set[j - 1];
    if (hist) hist_copy(hist + j * mig, hist + (j - 1) * mig, mig);
  }
  set[0] = line;
  if (hist) hist_clear(hist, mig);
  return victim;
}
/* A block this slice sends away by migration is still on its way (its arrival not yet told). */
static int sending_block(const int32_t* k) { return k[C_FWD_DST] >= 0 && (k[C_FWD_DST] & MIG_TRANSIT); }
/* Sec. 3.3: records an access by `who` in a way's history of its last `mig` accessors and
   returns how many of them were `who`'s. */
static int hist_note(int32_t* h, int mig, int32_t who) {
  for (int m = mig - 1; m > 0; --m) h[m] = h[m - 1];
  h[0] = who;
  int n = 0;
  for (int m = 0; m < mig; ++m) n += h[m] == who;
  return n;
}

/* The directory's answer to tile `rq` asking for `line`: the owner, or a negative reply, in
   which case the entry now names rq, which brings the block from memory into its slice. */
static int32_t dir_lookup(oracle_sim* s, int32_t line, int32_t rq) {
  s->stats[OS_DIR_ACCESS]++;
  if (s->loc[line] >= 0) return s->loc[line];
  dir_set(s, line, rq);
  s->stats[OS_DIR_NACK]++;
  return CODE_NACK;
}

/* ---- phase one: memory access (Sec. 7.1, work in phase one; Sec. 3.5) -------------- */
static void phase_memory(oracle_sim* s, int32_t t) {
  const int64_t c = s->cycle;
  int32_t* k = s->core + (size_t)t * C_WORDS;
  const uint32_t* r = s->rnd + (size_t)t * 4;
  const int32_t delay = inject_delay(s);

  /* home L2 slice serves the request that was ejected here in the previous cycle; the reply
     can leave once the block is there (at once on a hit, after mem_lat on a miss) */
  if (k[C_L2Q] >= 0 && !s->lspd) {
    int32_t rq = k[C_L2Q], line = k[C_L2Q_LINE];
    if (l2_lookup(s, t, line)) list_append(s, t, C_HIT_H, C_HIT_T, rq, (int32_t)(c + delay), line);
    else list_append(s, t, C_MISS_H, C_MISS_T, rq, (int32_t)(c + s->cfg.mem_lat + delay), line);
    k[C_L2Q] = -1;
    k[C_L2Q_LINE] = -1;
  }
  /* LSPD: the message ejected here last cycle.  A remote access is served from this slice (the
     block goes back in reply_flits flits) or trapped if the slice no longer holds the line; a
     directory access is answered with the owner or a negative reply; an eviction notice clears
     the entry (which names the sender until then).  One-flit answers wait in the miss queue, which an
     LSPD slice does not otherwise use (Sec. 3.2, Sec. 6.2.2, Table 1). */
  if (k[C_L2Q] >= 0 && s->lspd) {
    int32_t type = k[C_L2Q] >> 24, who = k[C_L2Q] & 0xFFFFFF, line = k[C_L2Q_LINE];
    if (type == Q_RA) {
      int32_t* set = l2_set(s, t, line);
      int32_t* hist = l2_hist(s, t, line);
      int i = l2_find(set, s->cfg.l2_ways, line);
      if (i >= 0) {
        s->stats[OS_L2_HIT]++;
        int n = 0;
        if (hist) n = hist_note(hist + i * s->mig, s->mig, who);  /* Sec. 3.3: the block's last accessors */
        l2_front(set, hist, s->mig, i);
        /* Sec. 3.3: a remote tile has made most of the block's last `mig` accesses, so the block
           moves there.  Not while this slice still waits for the directory to acknowledge its
           own claim of the block, and not while another block of this slice is on its way. */
        const int claiming = k[C_STATE] == ST_WAIT && k[C_LINE] == line;
        const int sending = sending_block(k);
        if (s->mig && 2 * n > s->mig && !claiming && !sending) {
          /* the block goes whole; this slice keeps serving it until it has arrived */
          k[C_FWD_LINE] = line;
          k[C_FWD_DST] = who | MIG_TRANSIT;
          s->stats[OS_MIGRATE]++;
          list_append(s, t, C_HIT_H, C_HIT_T, who, (int32_t)(c + delay), line | MIG_MARK);
        } else {
          list_append(s, t, C_HIT_H, C_HIT_T, who, (int32_t)(c + delay), line);
        }
      } else if (s->mig && k[C_FWD_LINE] == line) {  /* Sec. 3.3: redirect to where it went */
        s->stats[OS_REDIRECT]++;
        list_append(s, t, C_MISS_H, C_MISS_T, who, (int32_t)(c + delay), k[C_FWD_DST] & ~MIG_TRANSIT);
      } else {
        s->stats[OS_TRAP]++;
        list_append(s, t, C_MISS_H, C_MISS_T, who, (int32_t)(c + delay), CODE_TRAP);
      }
    } else if (type == Q_DA) {
      list_append(s, t, C_MISS_H, C_MISS_T, who, (int32_t)(c + delay), dir_lookup(s, line, who));
    } else if (type == Q_EV) {
      dir_evicted(s, line, who);
    } else if (type == Q_ARRIVED) {  /* Sec. 3.3: the block reached its new owner: this slice's copy
                                         goes (if the slice has not evicted it meanwhile) */
      if (k[C_FWD_DST] == (who | MIG_TRANSIT)) {
        const int32_t fl = k[C_FWD_LINE];
        int32_t* set = l2_set(s, t, fl);
        int i = l2_find(set, s->cfg.l2_ways, fl);
        if (i >= 0) l2_remove(set, l2_hist(s, t, fl), s->mig, s->cfg.l2_ways, i);
        k[C_FWD_DST] = who;
      } else if (s->check && !s->bad) {
        s->bad = 1;
        snprintf(s->msg, sizeof s->msg, "arrival notice from %d at %d, which sends nothing there", who, t);
      }
    } else {  /* Sec. 3.3: the directory is updated to the block's new owner, which is told */
      dir_set(s, line, who);
      list_append(s, t, C_MISS_H, C_MISS_T, who, (int32_t)(c + delay), CODE_ACK);
    }
    k[C_L2Q] = -1;
    k[C_L2Q_LINE] = -1;
  }

  const int state = k[C_STATE];
  int l1_used = 0; /* the L1 serves at most one access per cycle */
  switch (state) {
    case ST_FILL:
      if (k[C_WAKE] == (int32_t)c) {            /* block arrives: L1 fill, op complete */
        l1_used = 1;
        int32_t* set = l1_set(s, t, k[C_LINE]);
        cache_touch(set, s->cfg.l1_ways, k[C_LINE], 1);
        if (s->check) check_set(s, set, s->cfg.l1_ways, "L1", t);
        int64_t lat = c - k[C_ISSUE];
        s->stats[OS_OPS_DONE]++;
        s->stats[OS_OP_LAT] += lat;
        if (lat > s->stats[OS_OP_LAT_MAX]) s->stats[OS_OP_LAT_MAX] = lat;
        k[C_STATE] = ST_IDLE;
      }
      break;
    case ST_FILL_MEM:
    case ST_FILL_MIG:
      if (k[C_WAKE] == (int32_t)c) {            /* LSPD: block from memory (or migrated here) into
                                                   the local slice and L1 */
        l1_used = 1;
        int32_t line = k[C_LINE];
        int32_t* set2 = l2_set(s, t, line);
        int32_t victim = l2_insert(set2, l2_hist(s, t, line), s->mig, s->cfg.l2_ways, line);
        if (s->check) check_set(s, set2, s->cfg.l2_ways, "L2", t);
        if (victim >= 0 && s->mig && victim == k[C_FWD_LINE] && sending_block(k)) {
          /* the block on its way elsewhere leaves this slice; its new owner's claim updates the
             directory, and requests still reaching here are redirected */
        } else if (victim >= 0) {               /* the evicted block leaves the directory */
          if (dir_of(s, victim) == t) dir_evicted(s, victim, t);
          else k[C_EV] = victim;
        }
        int claim = 0;
        if (state == ST_FILL_MIG) {             /* Sec. 3.3: the directory learns the new owner; */
          if (dir_of(s, line) == t) dir_set(s, line, t);  /* the op completes when it has */
          else claim = 1;
        }
        if (claim) {
          k[C_CLAIM] = line;
          k[C_STATE] = ST_WAIT;
          break;
        }
        int32_t* set = l1_set(s, t, line);
        cache_touch(set, s->cfg.l1_ways, line, 1);
        if (s->check) check_set(s, set, s->cfg.l1_ways, "L1", t);
        int64_t lat = c - k[C_ISSUE];
        s->stats[OS_OPS_DONE]++;
        s->stats[OS_OP_LAT] += lat;
        if (lat > s->stats[OS_OP_LAT_MAX]) s->stats[OS_OP_LAT_MAX] = lat;
        k[C_STATE] = ST_IDLE;
      }
      break;
    case ST_L1MISS:
      if (k[C_WAKE] == (int32_t)c && s->lspd) {
        /* LSPD: the core's own slice, then the directory (at once when this tile keeps the
           entry).  A pending eviction notice or claim goes out first, so that a core has at most
           one of each.  (An arrival notice goes out before the core's next directory or remote
           access, so a second migrated block cannot come in while it is pending.) */
        int32_t line = k[C_LINE];
        int32_t* set2 = l2_set(s, t, line);
        int32_t* hist = l2_hist(s, t, line);
        int i = l2_find(set2, s->cfg.l2_ways, line);
        if (k[C_EV] >= 0 || k[C_CLAIM] >= 0) {  /* notices first */
          k[C_WAKE] = (int32_t)(c + 1);
        } else if (i >= 0) {
          s->stats[OS_L2_HIT]++;
          if (hist) hist_note(hist + i * s->mig, s->mig, t);   /* the local core's access */
          l2_front(set2, hist, s->mig, i);
          k[C_STATE] = ST_FILL;
          k[C_WAKE] = (int32_t)(c + 1);
        } else if (s->mig && k[C_FWD_LINE] == line && sending_block(k)) {
          /* this slice sent the block away and has since evicted its copy: the core waits for
             the arrival notice before it asks for the block again (so that the notice cannot
             remove a copy that came back to this slice) */
          k[C_WAKE] = (int32_t)(c + 1);
        } else if (dir_of(s, line) == t) {
          int32_t o = dir_lookup(s, line, t);
          if (o == t && k[C_FWD_LINE] == line) {  /* this slice gave the block away and its new */
            o = k[C_FWD_DST] & ~MIG_TRANSIT;        /* owner's claim is still on the way */
            s->stats[OS_REDIRECT]++;
          }
          if (o == t) {                         /* stale (an older migration): look again */
            s->stats[OS_TRAP]++;
            k[C_WAKE] = (int32_t)(c + 1);
          } else {
            s->stats[OS_L2_MISS]++;
            if (o == CODE_NACK) {
              k[C_STATE] = ST_FILL_MEM;
              k[C_WAKE] = (int32_t)(c + s->cfg.mem_lat);
            } else {
              k[C_STATE] = ST_SEND_RA;
              k[C_TARGET] = o;
              k[C_WAKE] = (int32_t)(c + delay);
              s->stats[OS_REQ_MADE]++;
            }
          }
        } else {
          s->stats[OS_L2_MISS]++;
          k[C_STATE] = ST_SEND_DA;
          k[C_WAKE] = (int32_t)(c + delay);
        }
      } else if (k[C_WAKE] == (int32_t)c) {     /* L1 miss penalty over: go to the home slice */
        int32_t line = k[C_LINE];
        if (line % s->N == t) {
          int hit = l2_lookup(s, t, line);
          k[C_STATE] = ST_FILL;
          k[C_WAKE] = (int32_t)(hit ? c + 1 : c + s->cfg.mem_lat);
        } else {
          k[C_STATE] = ST_SEND;                 /* request flit waits for an injection slot */
          s->stats[OS_REQ_MADE]++;
        }
      }
      break;
    case ST_IDLE: {
      int issue = 0;
      int32_t line = 0, issued = (int32_t)c;
      if (k[C_DLINE] >= 0) {                    /* the op that waited for the last miss */
        line = k[C_DLINE];
        issued = k[C_DISSUE];
        k[C_DLINE] = -1;
        k[C_DISSUE] = 0;
        issue = 2;
      } else if (k[C_FLINE] >= 0) {
        line = k[C_FLINE];
        k[C_FLINE] = -1;
        issue = 1;
      } else if (r[0] < s->cfg.op_thr) {
        issue = 1;
        line = drawn_line(s, t, r);
      }
      if (issue) {
        if (issue == 1) s->stats[OS_OPS_ISSUED]++;
        l1_used = 1;
        k[C_LINE] = line;
        k[C_ISSUE] = issued;
        int32_t* set = l1_set(s, t, line);
        if (cache_touch(set, s->cfg.l1_ways, line, 0)) {
          int64_t lat = c - issued;
          s->stats[OS_L1_HIT]++;
          s->stats[OS_OPS_DONE]++;
          s->stats[OS_OP_LAT] += lat;
          if (lat > s->stats[OS_OP_LAT_MAX]) s->stats[OS_OP_LAT_MAX] = lat;
        } else {
          s->stats[OS_L1_MISS]++;
          k[C_STATE] = ST_L1MISS;
          k[C_WAKE] = (int32_t)(c + s->cfg.l1_lat);
        }
      }
      break;
    }
    default:
      break;
  }

  /* Hit under miss (Sec. 3.5): while its miss is outstanding the core keeps drawing; a hit
     completes at once, a miss waits (no miss under a miss) and stops further issue until the
     outstanding block is filled.  Its L1 outcome is counted when it is looked up again. */
  if ((s->cfg.flags & ORACLE_FLAG_HIT_UNDER_MISS) && state != ST_IDLE && !l1_used && k[C_DLINE] < 0 &&
      r[0] < s->cfg.op_thr) {
    int32_t line = drawn_line(s, t, r);
    s->stats[OS_OPS_ISSUED]++;
    if (cache_touch(l1_set(s, t, line), s->cfg.l1_ways, line, 0)) {
      s->stats[OS_L1_HIT]++;
      s->stats[OS_OPS_DONE]++;
    } else {
      k[C_DLINE] = line;
      k[C_DISSUE] = (int32_t)c;
    }
  }
}

/* The pipeline stage of tile t holding the flits it arbitrates in cycle a (router delay > 1). */
static int32_t* pipe_stage(const oracle_sim* s, int64_t a, int32_t t) {
  return s->pipe + ((size_t)(a % (s->delay - 1)) * s->N + t) * SLOT_WORDS;
}

/* ---- phase two: oldest-first deflection arbitration (Sec. 4.3, Sec. 6.2.1) ---------- */
/* Flit a goes before flit b: oldest first, by injection cycle, then source tile; with
   deflection counts (AGE_DEFLECT) the more deflected flit first, then as before. */
static int goes_before(int a, int b, const int32_t* inj, const int32_t* src, const int32_t* age) {
  if (age && age[a] != age[b]) return age[a] > age[b];
  if (inj[a] != inj[b]) return inj[a] < inj[b];
  return src[a] < src[b];
}

/* Flits are considered in priority order.  Each takes the eject link if it is destined here
   and the link is still free, else its first free productive port (X before Y), else the
   lowest-numbered free port (a deflection). */
static int arbitrate_router(int32_t W, int32_t H, int32_t t, int n, const int32_t* dst, const int32_t* inj,
                            const int32_t* src, const int32_t* age, int32_t* port, int32_t* defl) {
  int order[8];
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 1; i < n; ++i) {                 /* insertion sort by priority */
    int v = order[i], j = i - 1;
    while (j >= 0 && goes_before(v, order[j], inj, src, age)) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  int32_t x = t % W, y = t / W;
  int valid[4] = {y > 0, y < H - 1, x < W - 1, x > 0};
  int used[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < n; ++k) {
    int i = order[k];
    port[i] = -1;
    defl[i] = 0;
    if (dst[i] == t && !used[PX]) {
      port[i] = PX;
      used[PX] = 1;
      continue;
    }
    int32_t dx = dst[i] % W - x, dy = dst[i] / W - y;
    int pref[2], np = 0;
    if (dx > 0) pref[np++] = PE;
    else if (dx < 0) pref[np++] = PW;
    if (dy > 0) pref[np++] = PS;
    else if (dy < 0) pref[np++] = PN;
    for (int q = 0; q < np && port[i] < 0; ++q)
      if (!used[pref[q]]) port[i] = pref[q];
    if (port[i] < 0) {
      for (int p = 0; p < 4 && port[i] < 0; ++p)
        if (valid[p] && !used[p]) port[i] = p;
      defl[i] = 1;
    }
    if (port[i] < 0) return ORACLE_EINVAL;   /* more flits than ports */
    used[port[i]] = 1;
  }
  return ORACLE_OK;
}

int oracle_arbitrate(int32_t width, int32_t height, int32_t tile, int32_t n, const int32_t* dst, const int32_t* inj,
                     const int32_t* src, const int32_t* age, int32_t* port, int32_t* deflected) {
  if (width < 1 || height < 1 || tile < 0 || tile >= width * height || n < 0 || n > 5) return ORACLE_EINVAL;
  return arbitrate_router(width, height, tile, n, dst, inj, src, age, port, deflected);
}

/* Phase two of tile t: gather arrivals, add at most one injected flit when an input is
   free (Sec. 4.2: a node injects whenever it finds a free input port), arbitrate.
   A reply is a packet of reply_flits flits (Sec. 3.6, Table 1: a remote L2 access moves a
   block as several flits); the home injects them one per injection, and the queue head is
   popped with its last flit.  The queue is chosen anew each cycle, so flits of a miss reply
   and of a hit reply can interleave. */
static void phase_route(oracle_sim* s, int32_t t) {
  const int64_t c = s->cycle;
  int32_t* k = s->core + (size_t)t * C_WORDS;
  const int32_t* arrived = s->link[c & 1] + (size_t)t * SLOT_WORDS;
  /* with a router delay D > 1 the flits arbitrated now arrived D-1 cycles ago; this cycle's
     arrivals take their place in the pipeline */
  int32_t in[SLOT_WORDS];
  if (s->delay > 1) {
    int32_t* st = pipe_stage(s, c, t);
    memcpy(in, st, sizeof in);
    memcpy(st, arrived, sizeof in);
  } else {
    memcpy(in, arrived, sizeof in);
  }
  int32_t fl[5][F_WORDS];
  int n = 0, deg = 0;
  for (int p = 0; p < 4; ++p) {
    if (port_valid(s, t, p)) deg++;
    if (in[p * F_WORDS + F_DST] >= 0) {
      memcpy(fl[n], in + p * F_WORDS, sizeof fl[n]);
      n++;
    }
  }
  int arrivals = n;

  /* injection candidate: ready miss reply, ready hit reply, own request (made at least
     inject_delay cycles ago), test flit, background */
  /* (LSPD: the miss queue holds one-flit answers, and the core's own flit is a pending
     eviction notice, a directory access or a remote-access request) */
  int cls = -1;
  const int own = s->lspd ? (k[C_EV] >= 0 || k[C_NOTE] >= 0 || k[C_CLAIM] >= 0 || ((k[C_STATE] == ST_SEND_DA || k[C_STATE] == ST_SEND_RA) &&
                                              k[C_WAKE] <= (int32_t)c))
                          : (k[C_STATE] == ST_SEND && k[C_WAKE] + inject_delay(s) <= (int32_t)c);
  if (k[C_MISS_H] >= 0 && s->core[(size_t)k[C_MISS_H] * C_WORDS + C_READY] <= (int32_t)c) cls = 0;
  else if (k[C_HIT_H] >= 0 && s->core[(size_t)k[C_HIT_H] * C_WORDS + C_READY] <= (int32_t)c) cls = 1;
  else if (own) cls = 2;
  else if (k[C_FDST] >= 0) cls = 3;
  else if (k[C_BG] > 0) cls = 4;
  if (cls >= 0 && arrivals >= deg) {
    s->stats[OS_INJ_BLOCKED]++;
    cls = -1;
  }
  if (cls >= 0) {
    int32_t* f = fl[n++];
    f[F_INJ] = (int32_t)c;
    f[F_SRC] = t;
    f[F_AGE] = 0;
    if (cls == 0 && s->lspd) {                 /* directory reply or trap: one flit */
      int32_t rq = list_pop(s, t, C_MISS_H, C_MISS_T);
      f[F_DST] = rq;
      f[F_INJ] = (int32_t)((uint32_t)c | CTL_BIT);
      f[F_INFO] = KIND_BITS(K_REPLY) | (s->core[(size_t)rq * C_WORDS + C_NLINE] + CODE_BASE);
      s->stats[OS_INJ_REPLY]++;
    } else if (cls == 2 && s->lspd) {
      const int32_t line = k[C_LINE];
      if (k[C_EV] >= 0) {                       /* eviction notice to the block's directory */
        f[F_DST] = dir_of(s, k[C_EV]);
        f[F_INJ] = (int32_t)((uint32_t)c | CTL_BIT);
        f[F_INFO] = KIND_BITS(K_DIR) | k[C_EV];
        k[C_EV] = -1;
      } else if (k[C_NOTE] >= 0) {              /* Sec. 3.3: the migrated block has arrived; its */
        f[F_DST] = k[C_NOTE];                   /* source drops its copy */
        f[F_INJ] = (int32_t)((uint32_t)c | CTL_BIT);
        f[F_INFO] = KIND_BITS(K_REQ);
        k[C_NOTE] = -1;
      } else if (k[C_CLAIM] >= 0) {             /* a migrated block's new owner, to the directory */
        f[F_DST] = dir_of(s, k[C_CLAIM]);
        f[F_INJ] = (int32_t)((uint32_t)c | CTL_BIT);
        f[F_INFO] = KIND_BITS(K_BG) | k[C_CLAIM];
        k[C_CLAIM] = -1;
      } else if (k[C_STATE] == ST_SEND_DA) {    /* directory access */
        f[F_DST] = dir_of(s, line);
        f[F_INFO] = KIND_BITS(K_DIR) | line;
        k[C_STATE] = ST_WAIT;
      } else {                                  /* remote access at the owner */
        f[F_DST] = k[C_TARGET];
        f[F_INFO] = KIND_BITS(K_REQ) | line;
        k[C_TARGET] = -1;
        k[C_STATE] = ST_WAIT;
      }
      s->stats[OS_INJ_REQ]++;
    } else if (cls == 0 || cls == 1) {
      int32_t rq = k[cls == 0 ? C_MISS_H : C_HIT_H];
      int32_t* node = s->core + (size_t)rq * C_WORDS;
      /* a migrating block (Sec. 3.3, Table 1) goes as MIG_FLITS answer flits */
      const int mig_pk = s->lspd && (node[C_NLINE] & MIG_MARK);
      f[F_DST] = rq;
      if (mig_pk) {
        f[F_INJ] = (int32_t)((uint32_t)c | CTL_BIT);
        f[F_INFO] = KIND_BITS(K_REPLY) | (CODE_MIG + CODE_BASE);
      } else {
        f[F_INFO] = KIND_BITS(K_REPLY) | node[C_NLINE];
      }
      s->stats[OS_INJ_REPLY]++;
      if (++node[C_NSENT] == (mig_pk ? MIG_FLITS : s->reply_flits)) {  /* the packet's last flit */
        node[C_NSENT] = 0;
        if (cls == 0) list_pop(s, t, C_MISS_H, C_MISS_T);
        else list_pop(s, t, C_HIT_H, C_HIT_T);
        if (!mig_pk) s->stats[OS_REPLY_SENT]++;
      }
    } else if (cls == 2) {
      f[F_DST] = k[C_LINE] % s->N;
      f[F_INFO] = KIND_BITS(K_REQ) | k[C_LINE];
      k[C_STATE] = ST_WAIT;
      s->stats[OS_INJ_REQ]++;
    } else {
      if (cls == 3) {
        f[F_DST] = k[C_FDST];
        k[C_FDST] = -1;
      } else {
        uint32_t r2[4];
        draw(s, c, t, 1u, r2);
        int32_t d = (int32_t)(((uint64_t)r2[0] * (uint64_t)(s->N - 1)) >> 32);
        if (d >= t) d++;
        f[F_DST] = d;
        k[C_BG]--;
      }
      f[F_INFO] = KIND_BITS(K_BG);
      s->stats[OS_INJ_BG]++;
    }
  }

  const int aged = (s->cfg.flags & ORACLE_FLAG_AGE_DEFLECT) != 0;
  int32_t dst[5], inj[5], src[5], age[5], port[5], defl[5];
  for (int i = 0; i < n; ++i) {
    dst[i] = fl[i][F_DST]; inj[i] = (int32_t)((uint32_t)fl[i][F_INJ] & ~CTL_BIT); src[i] = fl[i][F_SRC];
    age[i] = fl[i][F_AGE];
  }
  int rc = arbitrate_router(s->W, s->H, t, n, dst, inj, src, aged ? age : NULL, port, defl);
  if (rc != ORACLE_OK && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "router %d: no port", t); }

  int32_t* out = s->outp + (size_t)t * SLOT_WORDS;
  int32_t* ej = s->ej + (size_t)t * F_WORDS;
  for (int i = 0; i < SLOT_WORDS; ++i) out[i] = -1;
  for (int i = 0; i < F_WORDS; ++i) ej[i] = -1;
  int first = -1; /* the router's highest-priority flit */
  for (int i = 0; i < n; ++i) {
    if (first < 0 || goes_before(i, first, inj, src, aged ? age : NULL)) first = i;
    if (port[i] == PX) {
      memcpy(ej, fl[i], sizeof fl[i]);
    } else if (port[i] >= 0) {
      if (defl[i] && aged) {                    /* Sec. 6.2.1: a deflected flit ages by one */
        if (fl[i][F_AGE] >= AGE_LIMIT && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "deflection count overflow at %d", t); }
        fl[i][F_AGE]++;
      }
      memcpy(out + port[i] * F_WORDS, fl[i], sizeof fl[i]);
      s->stats[OS_TRAVERSALS]++;
      if (defl[i]) s->stats[OS_DEFLECTIONS]++;
    }
  }
  s->oldest_ok[t] = first < 0 || !defl[first];
}

/* ---- phase three: traversal, ejection, generation (Sec. 7.1, work in phase three) --- */
static void phase_move(oracle_sim* s, int32_t t) {
  const int64_t c = s->cycle;
  int32_t* k = s->core + (size_t)t * C_WORDS;
  int32_t* nxt = s->link[(c + 1) & 1];
  const int32_t* out = s->outp + (size_t)t * SLOT_WORDS;
  for (int p = 0; p < 4; ++p) {
    if (!port_valid(s, t, p)) continue;
    int32_t nb = neighbour(s, t, p);
    memcpy(nxt + (size_t)nb * SLOT_WORDS + opposite(p) * F_WORDS, out + p * F_WORDS, F_WORDS * sizeof(int32_t));
  }
  const int32_t* ej = s->ej + (size_t)t * F_WORDS;
  if (ej[F_DST] >= 0) {
    int kind = (int)((uint32_t)ej[F_INFO] >> 30);
    const int ctl = ((uint32_t)ej[F_INJ] & CTL_BIT) != 0;
    const int cl = (kind == K_DIR || (kind == K_BG && ctl)) ? K_REQ : kind;  /* directory messages
                                                                               count as requests */
    int64_t lat = c - (int32_t)((uint32_t)ej[F_INJ] & ~CTL_BIT);
    s->stats[OS_EJ_REQ + cl]++;
    s->stats[OS_LAT_REQ + cl] += lat;
    if (lat > s->stats[OS_LAT_MAX]) s->stats[OS_LAT_MAX] = lat;
    int bin = 0;
    while (bin < 15 && (lat >> (bin + 1)) > 0) bin++;
    s->stats[OS_HIST + bin]++;
    if (s->check) {  /* every hop takes D cycles, and a route is Manhattan plus detours */
      int32_t sx = ej[F_SRC] % s->W, sy = ej[F_SRC] / s->W, x = t % s->W, y = t / s->W;
      int64_t man = labs((long)(sx - x)) + labs((long)(sy - y));
      if ((lat < s->delay * man || lat % s->delay != 0) && !s->bad) {
        s->bad = 1;
        snprintf(s->msg, sizeof s->msg, "flit latency %lld over %lld hops at %d", (long long)lat, (long long)man, t);
      }
    }
    if (kind == K_REQ && ctl) {                /* migration: the block this slice sent has arrived */
      k[C_L2Q] = ej[F_SRC] | (Q_ARRIVED << 24);
      k[C_L2Q_LINE] = k[C_FWD_LINE];          /* the block it sent (one at a time) */
    } else if (kind == K_REQ) {                /* request reaches its home slice (LSPD: the owner) */
      s->stats[OS_REQ_RECV]++;
      k[C_L2Q] = ej[F_SRC];
      k[C_L2Q_LINE] = ej[F_INFO] & LINE_MASK;
    } else if (kind == K_DIR) {                /* LSPD: directory access or eviction notice */
      k[C_L2Q] = ej[F_SRC] | ((ctl ? Q_EV : Q_DA) << 24);
      k[C_L2Q_LINE] = ej[F_INFO] & LINE_MASK;
    } else if (kind == K_BG && ctl) {          /* migration: the new owner's claim */
      k[C_L2Q] = ej[F_SRC] | (Q_CLAIM << 24);
      k[C_L2Q_LINE] = ej[F_INFO] & LINE_MASK;
    } else if (kind == K_REPLY && ctl) {       /* LSPD: directory reply or trap */
      if (k[C_STATE] != ST_WAIT && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "answer at idle tile %d", t); }
      int32_t code = (ej[F_INFO] & LINE_MASK) - CODE_BASE;
      if (code != CODE_MIG) k[C_WAKE] = (int32_t)(c + 1);
      if (code == CODE_MIG) {                  /* a flit of the block migrating here; with the */
        if (++k[C_RCV] == MIG_FLITS) {         /* last one it goes into the slice and L1, and */
          k[C_RCV] = 0;                        /* its source is told (Sec. 3.3) */
          k[C_STATE] = ST_FILL_MIG;
          k[C_WAKE] = (int32_t)(c + 1);
          if (s->check && k[C_NOTE] >= 0 && !s->bad) {
            s->bad = 1;
            snprintf(s->msg, sizeof s->msg, "tile %d receives a block with an arrival notice pending", t);
          }
          k[C_NOTE] = ej[F_SRC];
        }
      } else if (code == CODE_ACK) {           /* the directory names this slice: the migrated */
        k[C_STATE] = ST_FILL;                  /* block fills L1 and the op completes */
      } else if (code == CODE_NACK) {          /* not on chip: from memory into the local slice */
        k[C_STATE] = ST_FILL_MEM;
        k[C_WAKE] = (int32_t)(c + s->cfg.mem_lat);
      } else if (code == CODE_TRAP || code == t) {
        /* ask the directory again: its entry was stale (the owner had evicted the block, or
           this tile's own eviction notice has not reached the directory yet) */
        if (code == t) s->stats[OS_TRAP]++;
        k[C_STATE] = ST_SEND_DA;          /* (a redirection to this tile itself is stale too) */
      } else {
        k[C_STATE] = ST_SEND_RA;
        k[C_TARGET] = code;
        s->stats[OS_REQ_MADE]++;
      }
    } else if (kind == K_REPLY) {              /* a flit of the block reaches the requester */
      if (k[C_STATE] != ST_WAIT && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "reply at idle tile %d", t); }
      if (++k[C_RCV] == s->reply_flits) {      /* all flits in: the block is complete */
        k[C_RCV] = 0;
        s->stats[OS_REPLY_RECV]++;
        k[C_STATE] = ST_FILL;
        k[C_WAKE] = (int32_t)(c + 1);
      }
    }
  }
  if (s->N > 1 && s->rnd[(size_t)t * 4 + 3] < s->cfg.bg_thr) {
    k[C_BG]++;
    s->stats[OS_BG_GEN]++;
  }
}

/* ---- per-cycle state digest --------------------------------------------------------- */
/* Digest of the words tile t owns after cycle c: the four words of each of its input slots
   for the next cycle and its core record, then, in the AGE_DEFLECT variant, the deflection
   counts of those slots' flits packed in pairs (16 bits each, 0 for an empty slot).  The
   queue-node words (next, ready, line, flits sent) are written by the requester's home, not
   by the tile, so they are left out (zeroed); they are compared through the canonical dump
   instead. */
static uint64_t tile_digest(const oracle_sim* s, int64_t c, int32_t t) {
  int32_t w[16 + C_WORDS + 2 + 7 * 18];
  int32_t age[4];
  const int aged = (s->cfg.flags & ORACLE_FLAG_AGE_DEFLECT) != 0;
  const int32_t* slots = s->link[(c + 1) & 1] + (size_t)t * SLOT_WORDS;
  for (int p = 0; p < 4; ++p) {
    memcpy(w + 4 * p, slots + p * F_WORDS, 4 * sizeof(int32_t));
    age[p] = slots[p * F_WORDS + F_DST] >= 0 ? slots[p * F_WORDS + F_AGE] : 0;
  }
  memcpy(w + 16, s->core + (size_t)t * C_WORDS, C_WORDS * sizeof(int32_t));
  w[16 + C_NEXT] = w[16 + C_READY] = w[16 + C_NLINE] = w[16 + C_NSENT] = 0;
  int nw = 16 + C_WORDS;
  if (aged) {
    w[nw++] = (int32_t)((uint32_t)age[0] | ((uint32_t)age[1] << 16));
    w[nw++] = (int32_t)((uint32_t)age[2] | ((uint32_t)age[3] << 16));
  }
  /* the router's pipeline, stage by stage in the order the stages are arbitrated */
  for (int st = 1; st < s->delay; ++st) {
    const int32_t* f = pipe_stage(s, c + st, t);
    for (int p = 0; p < 4; ++p) {
      memcpy(w + nw, f + p * F_WORDS, 4 * sizeof(int32_t));
      nw += 4;
      age[p] = f[p * F_WORDS + F_DST] >= 0 ? f[p * F_WORDS + F_AGE] : 0;
    }
    if (aged) {
      w[nw++] = (int32_t)((uint32_t)age[0] | ((uint32_t)age[1] << 16));
      w[nw++] = (int32_t)((uint32_t)age[2] | ((uint32_t)age[3] << 16));
    }
  }
  uint64_t h = mix64(((uint64_t)(uint32_t)c << 32) | (uint32_t)t);
  for (int i = 0; i < nw / 2; ++i)
    h = mix64(h ^ (((uint64_t)(uint32_t)w[2 * i] << 32) | (uint32_t)w[2 * i + 1]));
  return h;
}

/* ---- invariants --------------------------------------------------------------------- */
static void check_cycle(oracle_sim* s) {
  const int64_t c = s->cycle;
  const int32_t* nxt = s->link[(c + 1) & 1];
  int64_t occupied = 0, req_fl = 0, ans_fl = 0;
  int32_t* rep_to = s->scratch;              /* reply flits in flight, per requester */
  int32_t* queued_at = s->scratch + s->N;    /* 1 while the requester sits in a home's queue */
  int32_t* mig_to = s->scratch + 2 * s->N;   /* flits of a migrating block in flight, per receiver */
  memset(s->scratch, 0, (size_t)s->N * 3 * sizeof(int32_t));
  for (int32_t t = 0; t < s->N; ++t) {
    for (int st = 0; st < s->delay; ++st) {    /* the link slots, then the pipeline stages */
      const int32_t* sl = st == 0 ? nxt + (size_t)t * SLOT_WORDS : pipe_stage(s, c + st, t);
      for (int p = 0; p < 4; ++p) {
        const int32_t* f = sl + p * F_WORDS;
        if (f[F_DST] < 0) continue;
        occupied++;
        int kind = (int)((uint32_t)f[F_INFO] >> 30);
        const int ctl = ((uint32_t)f[F_INJ] & CTL_BIT) != 0;
        const int mig_flit = kind == K_REPLY && ctl && (f[F_INFO] & LINE_MASK) == CODE_MIG + CODE_BASE;
        if ((kind == K_REQ && !ctl) || (kind == K_DIR && !ctl) || (kind == K_BG && ctl)) req_fl++;  /* remote or
                                                           directory access, ownership claim */
        if (kind == K_REPLY && ctl && !mig_flit) ans_fl++;       /* directory answer, trap, redirection */
        if (mig_flit) mig_to[f[F_DST]]++;
        if (kind == K_REPLY && !ctl) rep_to[f[F_DST]]++;
        if (!port_valid(s, t, p) && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "flit on a missing link at %d", t); }
      }
    }
    if (!s->oldest_ok[t] && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "first flit deflected at %d", t); }
  }
  int64_t inj = s->stats[OS_INJ_REQ] + s->stats[OS_INJ_REPLY] + s->stats[OS_INJ_BG];
  int64_t ejc = s->stats[OS_EJ_REQ] + s->stats[OS_EJ_REPLY] + s->stats[OS_EJ_BG];
  if (inj - ejc != occupied && !s->bad) {
    s->bad = 1;
    snprintf(s->msg, sizeof s->msg, "conservation: injected-ejected=%lld occupied=%lld", (long long)(inj - ejc), (long long)occupied);
  }
  /* every waiting requester is accounted for exactly once: request or reply in flight,
     request at its home slice's input, or queued at its home */
  int64_t waiting = 0, queued = 0, at_home = 0;
  for (int32_t t = 0; t < s->N; ++t) {
    const int32_t* k = s->core + (size_t)t * C_WORDS;
    if (k[C_STATE] == ST_WAIT) waiting++;
    if (k[C_L2Q] >= 0 && (k[C_L2Q] >> 24) != Q_EV && (k[C_L2Q] >> 24) != Q_ARRIVED) at_home++;
    if (k[C_CLAIM] >= 0) at_home++;   /* a claim waiting for injection */
    for (int which = 0; which < 2; ++which) {
      int32_t r = k[which ? C_MISS_H : C_HIT_H], last = -1;
      int64_t len = 0;
      while (r >= 0) {
        if (s->core[(size_t)r * C_WORDS + C_STATE] != ST_WAIT && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "queued tile %d not waiting", r); }
        queued_at[r] = 1;
        last = r;
        r = s->core[(size_t)r * C_WORDS + C_NEXT];
        if (++len > s->N) { if (!s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "cyclic reply list at %d", t); } break; }
      }
      if (last != k[which ? C_MISS_T : C_HIT_T] && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "bad list tail at %d", t); }
      queued += len;
    }
  }
  /* a waiting requester is in exactly one place: its request in flight, at its home's input,
     queued at the home (some of its reply's flits possibly sent), or its whole reply sent with
     flits still in flight; the flits in flight are those sent and not yet received */
  int64_t rep_pk = 0;
  for (int32_t r = 0; r < s->N; ++r) {
    const int32_t* k = s->core + (size_t)r * C_WORDS;
    const int32_t in_flight = rep_to[r] + mig_to[r];
    if (queued_at[r]) {
      if (in_flight != k[C_NSENT] - k[C_RCV] && !s->bad) { s->bad = 1; snprintf(s->msg, sizeof s->msg, "reply flits of queued tile %d", r); }
    } else if (in_flight > 0) {
      rep_pk++;
      const int32_t len = mig_to[r] ? MIG_FLITS : s->reply_flits;
      if ((k[C_STATE] != ST_WAIT || (rep_to[r] && mig_to[r]) || in_flight != len - k[C_RCV]) && !s->bad) {
        s->bad = 1;
        snprintf(s->msg, sizeof s->msg, "reply flits in flight to tile %d", r);
      }
    }
  }
  if (waiting != req_fl + ans_fl + rep_pk + queued + at_home && !s->bad) {
    s->bad = 1;
    snprintf(s->msg, sizeof s->msg, "requester accounting: waiting=%lld req=%lld answers=%lld reply=%lld queued=%lld at_home=%lld",
             (long long)waiting, (long long)req_fl, (long long)ans_fl, (long long)rep_pk, (long long)queued,
             (long long)at_home);
  }
  /* LSPD: one copy of a block on chip, and the directory names the slice that holds it (with
     migration: or the slice waits for the acknowledgement of its claim of it).  With migration
     a source keeps its copy until told of the block's arrival, and the block may move on before
     that, so besides that one copy only slices that have sent the block and wait for its
     arrival notice may hold it. */
  if (s->lspd) {
    const int32_t S2 = s->cfg.l2_sets, W2 = s->cfg.l2_ways;
    memset(s->seen, 0, (size_t)s->lines * sizeof(int32_t));
    for (int32_t t = 0; t < s->N && !s->bad; ++t) {
      const int32_t* k = s->core + (size_t)t * C_WORDS;
      for (int32_t i = 0; i < S2 * W2; ++i) {
        const int32_t line = s->l2[(size_t)t * S2 * W2 + i];
        if (line < 0) continue;
        const int claiming = s->mig && k[C_STATE] == ST_WAIT && k[C_LINE] == line;
        const int sending = s->mig && k[C_FWD_LINE] == line && sending_block(k);
        /* sources count in the high half, so that they are told apart from plain copies */
        s->seen[line] += sending ? 0x10000 : 1;
        if ((s->seen[line] & 0xFFFF) > 1 || (s->loc[line] != t && !claiming && !sending)) {
          s->bad = 1;
          snprintf(s->msg, sizeof s->msg, "slice %d holds line %d, directory names %d", t, line, s->loc[line]);
          break;
        }
      }
    }
  }
}

/* ---- the serial main loop (Sec. 7.1) --------------------------------------------------- */
int oracle_step(oracle_sim* s, int64_t n, uint64_t* digests, int32_t check) {
  if (!s || n < 0) return ORACLE_EINVAL;
  s->check = check;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t c = s->cycle;
    for (int32_t t = 0; t < s->N; ++t) draw(s, c, t, 0u, s->rnd + (size_t)t * 4);
    for (int32_t t = 0; t < s->N; ++t) phase_memory(s, t);
    for (int32_t t = 0; t < s->N; ++t) phase_route(s, t);
    for (int32_t t = 0; t < s->N; ++t) phase_move(s, t);
    if (digests) {
      uint64_t d = 0;
      for (int32_t t = 0; t < s->N; ++t) d += tile_digest(s, c, t);
      digests[i] = d;
    }
    if (check) check_cycle(s);
    s->stats[OS_CYCLES]++;
    s->cycle++;
    if (s->bad) return ORACLE_EINVARIANT;
  }
  return ORACLE_OK;
}

/* ---- creation, dump, hooks ------------------------------------------------------------ */
static int is_pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

int oracle_create(const oracle_config* cfg, const uint32_t* zs, const uint32_t* zp, int32_t zk, oracle_sim** out) {
  if (!cfg || !out || !zs) return ORACLE_EINVAL;
  *out = NULL;
  int64_t N = (int64_t)cfg->width * cfg->height;
  if (cfg->width < 1 || cfg->height < 1 || N > (1 << 20)) return ORACLE_EINVAL;
  if (!is_pow2(cfg->l1_sets) || !is_pow2(cfg->l1_ways) || cfg->l1_ways > 8) return ORACLE_EINVAL;
  if (!is_pow2(cfg->l2_sets) || !is_pow2(cfg->l2_ways) || cfg->l2_ways > 8) return ORACLE_EINVAL;
  if (cfg->l1_lat < 1 || cfg->mem_lat < 1 || cfg->shared_lines < 1 || cfg->private_lines < 0) return ORACLE_EINVAL;
  if ((int64_t)cfg->shared_lines + N * cfg->private_lines > (int64_t)LINE_MASK + 1) return ORACLE_EINVAL;
  if (zk != 65536 || (cfg->private_lines > 0 && !zp)) return ORACLE_EINVAL;
  /* a quantile table must not decrease and must stay inside its region */
  for (int i = 0; i < zk; ++i)
    if (zs[i] > zs[i + 1] || (cfg->private_lines > 0 && zp[i] > zp[i + 1])) return ORACLE_EINVAL;
  if (zs[zk] > (uint32_t)cfg->shared_lines || (cfg->private_lines > 0 && zp[zk] > (uint32_t)cfg->private_lines))
    return ORACLE_EINVAL;
  if (cfg->reply_flits < 0 || cfg->reply_flits > 16) return ORACLE_EINVAL;
  if (cfg->flags & ~(ORACLE_FLAG_AGE_DEFLECT | ORACLE_FLAG_HIT_UNDER_MISS | ORACLE_FLAG_INJECT_DELAY | ORACLE_FLAG_LSPD |
                     ORACLE_FLAG_LSPD_CENTRAL))
    return ORACLE_EINVAL;
  if (cfg->router_delay < 0 || cfg->router_delay > 8) return ORACLE_EINVAL;
  if ((cfg->flags & ORACLE_FLAG_LSPD_CENTRAL) && !(cfg->flags & ORACLE_FLAG_LSPD)) return ORACLE_EINVAL;
  if (cfg->mig_threshold < 0 || cfg->mig_threshold > 16 || (cfg->mig_threshold && !(cfg->flags & ORACLE_FLAG_LSPD)))
    return ORACLE_EINVAL;
  oracle_sim* s = (oracle_sim*)calloc(1, sizeof(oracle_sim));
  if (!s) return ORACLE_ENOMEM;
  s->cfg = *cfg;
  s->W = cfg->width;
  s->H = cfg->height;
  s->N = (int32_t)N;
  s->reply_flits = cfg->reply_flits > 0 ? cfg->reply_flits : 1;
  s->delay = cfg->router_delay > 0 ? cfg->router_delay : 1;
  s->lspd = (cfg->flags & ORACLE_FLAG_LSPD) ? ((cfg->flags & ORACLE_FLAG_LSPD_CENTRAL) ? 2 : 1) : 0;
  s->dir_center = (cfg->height / 2) * cfg->width + cfg->width / 2;
  s->lines = (int64_t)cfg->shared_lines + N * cfg->private_lines;
  s->mig = cfg->mig_threshold;
  s->zk = zk;
  s->zs = (uint32_t*)malloc((size_t)(zk + 1) * 4);
  s->zp = (uint32_t*)malloc((size_t)(zk + 1) * 4);
  s->link[0] = (int32_t*)malloc((size_t)N * SLOT_WORDS * 4);
  s->link[1] = (int32_t*)malloc((size_t)N * SLOT_WORDS * 4);
  s->core = (int32_t*)malloc((size_t)N * C_WORDS * 4);
  s->l1 = (int32_t*)malloc((size_t)N * cfg->l1_sets * cfg->l1_ways * 4);
  s->l2 = (int32_t*)malloc((size_t)N * cfg->l2_sets * cfg->l2_ways * 4);
  s->rnd = (uint32_t*)malloc((size_t)N * 4 * 4);
  s->outp = (int32_t*)malloc((size_t)N * SLOT_WORDS * 4);
  s->ej = (int32_t*)malloc((size_t)N * F_WORDS * 4);
  s->oldest_ok = (int32_t*)malloc((size_t)N * 4);
  s->scratch = (int32_t*)malloc((size_t)N * 3 * 4);
  s->pipe = (int32_t*)malloc((size_t)(s->delay - 1) * N * SLOT_WORDS * 4 + 4);
  s->loc = (int32_t*)malloc((size_t)(s->lspd ? s->lines : 0) * 4 + 4);
  s->seen = (int32_t*)malloc((size_t)(s->lspd ? s->lines : 0) * 4 + 4);
  s->l2h = (int32_t*)malloc((size_t)(s->mig ? N * cfg->l2_sets * cfg->l2_ways * s->mig : 0) * 4 + 4);
  if (!s->zs || !s->zp || !s->link[0] || !s->link[1] || !s->core || !s->l1 || !s->l2 || !s->rnd || !s->outp || !s->ej ||
      !s->oldest_ok || !s->scratch || !s->pipe || !s->loc || !s->seen || !s->l2h) {
    oracle_destroy(s);
    return ORACLE_ENOMEM;
  }
  memcpy(s->zs, zs, (size_t)(zk + 1) * 4);
  if (zp) memcpy(s->zp, zp, (size_t)(zk + 1) * 4);
  else memcpy(s->zp, zs, (size_t)(zk + 1) * 4);
  memset(s->link[0], 0xFF, (size_t)N * SLOT_WORDS * 4);
  memset(s->link[1], 0xFF, (size_t)N * SLOT_WORDS * 4);
  memset(s->pipe, 0xFF, (size_t)(s->delay - 1) * N * SLOT_WORDS * 4);
  if (s->lspd) memset(s->loc, 0xFF, (size_t)s->lines * 4);
  memset(s->core, 0xFF, (size_t)N * C_WORDS * 4);
  for (int64_t t = 0; t < N; ++t) {
    s->core[t * C_WORDS + C_STATE] = ST_IDLE;
    s->core[t * C_WORDS + C_BG] = 0;
    s->core[t * C_WORDS + C_RCV] = 0;
    s->core[t * C_WORDS + C_NSENT] = 0;
    s->core[t * C_WORDS + C_DISSUE] = 0;
    s->core[t * C_WORDS + C_DSUM_LO] = 0;
    s->core[t * C_WORDS + C_DSUM_HI] = 0;
  }
  memset(s->l1, 0xFF, (size_t)N * cfg->l1_sets * cfg->l1_ways * 4);
  memset(s->l2, 0xFF, (size_t)N * cfg->l2_sets * cfg->l2_ways * 4);
  if (s->mig) memset(s->l2h, 0xFF, (size_t)N * cfg->l2_sets * cfg->l2_ways * s->mig * 4);
  *out = s;
  return ORACLE_OK;
}

void oracle_destroy(oracle_sim* s) {
  if (!s) return;
  free(s->zs); free(s->zp); free(s->link[0]); free(s->link[1]); free(s->core); free(s->l1); free(s->l2);
  free(s->rnd); free(s->outp); free(s->ej); free(s->oldest_ok); free(s->scratch); free(s->pipe); free(s->loc);
  free(s->seen); free(s->l2h);
  free(s);
}

int oracle_stats(const oracle_sim* s, int64_t* out) {
  if (!s || !out) return ORACLE_EINVAL;
  memcpy(out, s->stats, sizeof s->stats);
  return ORACLE_OK;
}

int64_t oracle_cycle(const oracle_sim* s) { return s ? s->cycle : -1; }

size_t oracle_dump_words(const oracle_sim* s) {
  size_t N = (size_t)s->N;
  return DUMP_HEADER + N * 16 + N * C_WORDS + N * s->cfg.l1_sets * s->cfg.l1_ways + N * s->cfg.l2_sets * s->cfg.l2_ways +
         2 * OS_COUNT + N * 4 + (size_t)(s->delay - 1) * N * 20 + (size_t)(s->lspd ? s->lines : 0) +
         (size_t)(s->mig ? N * s->cfg.l2_sets * s->cfg.l2_ways * s->mig : 0);
}

/* Canonical state (format version 3): header {magic, 3, W, H, cycle (low, high), L1 sets,
   L1 ways, L2 sets, L2 ways, reply flits, core-record words, variant flags, 0...}, the four
   words of each input slot of the next cycle, core records, L1 and L2 tags (most recently used
   first), statistics as (low, high) word pairs, the deflection count of each input slot's
   flit (0 for an empty slot and outside the AGE_DEFLECT variant), and with a router delay
   D > 1 (header word 13) the routers' pipelines: stages 1..D-1, stage k holding the flits
   arbitrated k-1 cycles after the dump's cycle, four words per slot, then their deflection
   counts, with the LSPD directory (header word 14: 1 interleaved, 2 central) the location
   array, one word per line, and with migration (header word 15: the threshold) the access
   record of every L2 way. */
int oracle_dump(const oracle_sim* s, int32_t* buf, size_t words) {
  if (!s || !buf || words < oracle_dump_words(s)) return ORACLE_EINVAL;
  size_t N = (size_t)s->N, o = 0;
  int32_t hdr[DUMP_HEADER] = {DUMP_MAGIC, 4, s->W, s->H, (int32_t)(uint32_t)s->cycle, (int32_t)(s->cycle >> 32),
                              s->cfg.l1_sets, s->cfg.l1_ways, s->cfg.l2_sets, s->cfg.l2_ways, s->reply_flits,
                              C_WORDS, s->cfg.flags, s->delay, s->lspd, s->mig};
  memcpy(buf, hdr, sizeof hdr);
  o += DUMP_HEADER;
  const int32_t* slots = s->link[s->cycle & 1];
  for (size_t i = 0; i < N * 4; ++i) {
    memcpy(buf + o, slots + i * F_WORDS, 4 * sizeof(int32_t));
    o += 4;
  }
  memcpy(buf + o, s->core, N * C_WORDS * 4); o += N * C_WORDS;
  size_t n1 = N * s->cfg.l1_sets * s->cfg.l1_ways, n2 = N * s->cfg.l2_sets * s->cfg.l2_ways;
  memcpy(buf + o, s->l1, n1 * 4); o += n1;
  memcpy(buf + o, s->l2, n2 * 4); o += n2;
  for (int i = 0; i < OS_COUNT; ++i) {
    buf[o++] = (int32_t)(uint32_t)(uint64_t)s->stats[i];
    buf[o++] = (int32_t)((uint64_t)s->stats[i] >> 32);
  }
  for (size_t i = 0; i < N * 4; ++i) buf[o++] = slots[i * F_WORDS + F_DST] >= 0 ? slots[i * F_WORDS + F_AGE] : 0;
  for (int st = 1; st < s->delay; ++st) {
    const int32_t* f = pipe_stage(s, s->cycle + st - 1, 0);
    for (size_t i = 0; i < N * 4; ++i) {
      memcpy(buf + o, f + i * F_WORDS, 4 * sizeof(int32_t));
      o += 4;
    }
  }
  for (int st = 1; st < s->delay; ++st) {
    const int32_t* f = pipe_stage(s, s->cycle + st - 1, 0);
    for (size_t i = 0; i < N * 4; ++i) buf[o++] = f[i * F_WORDS + F_DST] >= 0 ? f[i * F_WORDS + F_AGE] : 0;
  }
  if (s->lspd) {
    memcpy(buf + o, s->loc, (size_t)s->lines * 4);
    o += (size_t)s->lines;
  }
  if (s->mig) memcpy(buf + o, s->l2h, N * s->cfg.l2_sets * s->cfg.l2_ways * s->mig * 4);
  return ORACLE_OK;
}

int oracle_load(oracle_sim* s, const int32_t* buf, size_t words) {
  if (!s || !buf || words < oracle_dump_words(s)) return ORACLE_EINVAL;
  if (buf[0] != DUMP_MAGIC || buf[1] != 4 || buf[2] != s->W || buf[3] != s->H || buf[6] != s->cfg.l1_sets ||
      buf[7] != s->cfg.l1_ways || buf[8] != s->cfg.l2_sets || buf[9] != s->cfg.l2_ways || buf[10] != s->reply_flits ||
      buf[11] != C_WORDS || buf[12] != s->cfg.flags || buf[13] != s->delay || buf[14] != s->lspd ||
      buf[15] != s->mig)
    return ORACLE_EINVAL;
  size_t N = (size_t)s->N, o = DUMP_HEADER;
  s->cycle = (int64_t)(((uint64_t)(uint32_t)buf[5] << 32) | (uint32_t)buf[4]);
  int32_t* slots = s->link[s->cycle & 1];
  for (size_t i = 0; i < N * 4; ++i) {
    memcpy(slots + i * F_WORDS, buf + o, 4 * sizeof(int32_t));
    o += 4;
  }
  memset(s->link[(s->cycle + 1) & 1], 0xFF, N * SLOT_WORDS * 4);
  memcpy(s->core, buf + o, N * C_WORDS * 4); o += N * C_WORDS;
  size_t n1 = N * s->cfg.l1_sets * s->cfg.l1_ways, n2 = N * s->cfg.l2_sets * s->cfg.l2_ways;
  memcpy(s->l1, buf + o, n1 * 4); o += n1;
  memcpy(s->l2, buf + o, n2 * 4); o += n2;
  for (int i = 0; i < OS_COUNT; ++i) {
    s->stats[i] = (int64_t)(((uint64_t)(uint32_t)buf[o + 1] << 32) | (uint32_t)buf[o]);
    o += 2;
  }
  for (size_t i = 0; i < N * 4; ++i) slots[i * F_WORDS + F_AGE] = slots[i * F_WORDS + F_DST] >= 0 ? buf[o + i] : -1;
  /* state that only a variant can hold */
  for (size_t i = 0; i < N * 4; ++i)
    if (buf[o + i] != 0 && !(s->cfg.flags & ORACLE_FLAG_AGE_DEFLECT)) return ORACLE_EINVAL;
  o += N * 4;
  for (int st = 1; st < s->delay; ++st) {
    int32_t* f = pipe_stage(s, s->cycle + st - 1, 0);
    const int32_t* ages = buf + o + (size_t)(s->delay - 1) * N * 16 + (size_t)(st - 1) * N * 4;
    for (size_t i = 0; i < N * 4; ++i) {
      memcpy(f + i * F_WORDS, buf + o + (size_t)(st - 1) * N * 16 + i * 4, 4 * sizeof(int32_t));
      if (ages[i] != 0 && !(s->cfg.flags & ORACLE_FLAG_AGE_DEFLECT)) return ORACLE_EINVAL;
      f[i * F_WORDS + F_AGE] = f[i * F_WORDS + F_DST] >= 0 ? ages[i] : -1;
    }
  }
  o += (size_t)(s->delay - 1) * N * 20;
  if (s->lspd) {
    for (int64_t i = 0; i < s->lines; ++i)
      if (buf[o + i] < -1 || buf[o + i] >= s->N) return ORACLE_EINVAL;
    memcpy(s->loc, buf + o, (size_t)s->lines * 4);
    o += (size_t)s->lines;
  }
  if (s->mig) memcpy(s->l2h, buf + o, N * s->cfg.l2_sets * s->cfg.l2_ways * s->mig * 4);
  for (size_t t = 0; t < N; ++t)
    if (s->core[t * C_WORDS + C_DLINE] >= 0 && !(s->cfg.flags & ORACLE_FLAG_HIT_UNDER_MISS)) return ORACLE_EINVAL;
  return ORACLE_OK;
}

int oracle_force_op(oracle_sim* s, int32_t tile, int32_t line) {
  if (!s || tile < 0 || tile >= s->N || line < 0 || line > LINE_MASK) return ORACLE_EINVAL;
  s->core[(size_t)tile * C_WORDS + C_FLINE] = line;
  return ORACLE_OK;
}

int oracle_force_bg(oracle_sim* s, int32_t tile, int32_t dst) {
  if (!s || tile < 0 || tile >= s->N || dst < 0 || dst >= s->N || dst == tile) return ORACLE_EINVAL;
  s->core[(size_t)tile * C_WORDS + C_FDST] = dst;
  return ORACLE_OK;
}

int oracle_set_rates(oracle_sim* s, uint32_t op_thr, uint32_t bg_thr) {
  if (!s) return ORACLE_EINVAL;
  s->cfg.op_thr = op_thr;
  s->cfg.bg_thr = bg_thr;
  return ORACLE_OK;
}

int oracle_quiescent(const oracle_sim* s) {
  const int32_t* cur = s->link[s->cycle & 1];
  for (size_t i = 0; i < (size_t)(s->delay - 1) * s->N * 4; ++i)
    if (s->pipe[i * F_WORDS + F_DST] >= 0) return 0;
  for (int32_t t = 0; t < s->N; ++t) {
    for (int p = 0; p < 4; ++p)
      if (cur[(size_t)t * SLOT_WORDS + p * F_WORDS] >= 0) return 0;
    const int32_t* k = s->core + (size_t)t * C_WORDS;
    if (k[C_STATE] != ST_IDLE || k[C_L2Q] >= 0 || k[C_HIT_H] >= 0 || k[C_MISS_H] >= 0 || k[C_BG] != 0 ||
        k[C_FLINE] >= 0 || k[C_FDST] >= 0 || k[C_RCV] != 0 || k[C_DLINE] >= 0 || k[C_EV] >= 0 || k[C_CLAIM] >= 0 ||
        k[C_NOTE] >= 0 || sending_block(k))
      return 0;
  }
  return 1;
}

const char* oracle_invariant_msg(const oracle_sim* s) { return s ? s->msg : ""; }
