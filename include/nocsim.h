/*
 * nocsim.h -- C ABI of the MI355X (gfx950) simulator of a bufferless deflection-routed
 * 2D-mesh chip multicore with a logically shared, physically distributed L2.
 *
 * Method: Kumar & Sahu, "Bufferless NOC Simulation of Large Multicore System on GPU
 * Hardware" (arXiv 1508.03235).  One call of the step advances every tile of every
 * simulated chip by whole cycles; each cycle runs the paper's three phases per router
 * (Sec. 7.1): the memory access (private L1, then the line's home L2 slice, Sec. 3.1-3.5),
 * oldest-first bufferless deflection arbitration with X-then-Y productive preference and
 * injection only into a free input (Sec. 4.2-4.3, Sec. 6.2.1), and link traversal,
 * ejection and injection.
 *
 * Conventions
 *  - Every function returns an int32 status: SIM_OK (0) or a negative SIM_E* code; nothing
 *    throws.  sim_strerror() names a code.
 *  - Device memory is owned by the caller: sim_state_bytes() sizes one buffer, which the
 *    caller allocates (e.g. torch.empty(bytes, dtype=torch.uint8, device="cuda")) and passes
 *    as `dev_mem` together with a hipStream_t (`stream`, NULL = default stream).  The
 *    library allocates no device memory; it keeps the pointer and never frees it.  The
 *    buffer must stay alive until sim_destroy()/simb_destroy().
 *  - Steps are asynchronous on the stream.  sim_stats, sim_dump, sim_load and the test hooks
 *    synchronise the stream.
 *  - A handle is bound to one stream and is not thread safe.  Two handles may share nothing.
 *  - Host pointers are plain host memory; `dev_*` pointers are device memory.
 *  - Tile numbering: tile = y * width + x, x = column, y = row; ports 0..3 = north (y-1),
 *    south (y+1), east (x+1), west (x-1).
 */
#ifndef NOCSIM_H
#define NOCSIM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SIM_OK = 0,
  SIM_EINVAL = -1,     /* bad argument or shape (see sim_state_bytes) */
  SIM_ENOMEM = -2,     /* device buffer too small */
  SIM_EHIP = -3,       /* a HIP runtime call failed; sim_last_hip_error() has the code */
  SIM_EINVARIANT = -4, /* a state index out of range was caught on the device */
  SIM_EBUSY = -5,      /* slot in use / no free slot */
  SIM_EHANG = -6,      /* a bounded cross-workgroup wait ran out; results are invalid */
  SIM_ELIVELOCK = -7   /* the watchdog (sim_set_watchdog) saw a flit older than its bound */
};

/* Model parameters of one simulated chip.  Bernoulli draws are u32 and succeed when
   draw < threshold (threshold = floor(p * 2^32)). */
typedef struct {
  int32_t width, height;      /* 1..2048 each, width*height < 2^20 */
  uint32_t seed_lo, seed_hi;  /* Philox4x32-10 key */
  int32_t l1_sets, l1_ways;   /* private L1 per tile: sets a power of two, ways in {1,2,4,8} */
  int32_t l2_sets, l2_ways;   /* L2 slice per tile, same constraints */
  int32_t l1_lat;             /* cycles from an L1 miss to its follow-up, >= 1 */
  int32_t mem_lat;            /* latency of an L2 miss (off-chip memory), >= 1 */
  uint32_t op_thr;            /* a memory op is issued by an idle core when draw < op_thr */
  uint32_t shared_thr;        /* the op goes to the shared region when draw < shared_thr */
  uint32_t bg_thr;            /* a background flit is generated when draw < bg_thr */
  int32_t shared_lines;       /* shared region = lines [0, shared_lines) */
  int32_t private_lines;      /* per-tile private region (0 = none); shared_lines +
                                 width*height*private_lines must be <= 2^30 */
  int32_t flags;              /* model variants, SIM_FLAG_* (0 = the base model) */
  int32_t reply_flits;        /* flits of a reply packet, 1..16 (0 counts as 1); requests and
                                 background flits are one flit */
  int32_t router_delay;       /* cycles per hop, 1..8 (0 counts as 1): a flit that arrives at a
                                 router waits router_delay - 1 cycles in the router's pipeline
                                 before it is arbitrated */
  int32_t mig_threshold;      /* with LSPD: block migration (Sec. 3.3), 0 = none, at most 16.  Each
                                 L2 way keeps its last mig_threshold accessors; when a remote tile
                                 has made more than half of them, the slice sends that tile the
                                 block (16 flits, Table 1) and keeps serving it from its own copy
                                 until the receiver's arrival notice (1 flit) comes back; then it
                                 drops the copy and answers later requests with a redirection
                                 (1 flit).  The receiver claims the directory entry (1 flit) and
                                 its op completes with the directory's acknowledgement (1 flit).
                                 A slice sends one block at a time. */
} sim_config;

/* Model variants (bits of sim_config.flags).  Each replaces one reading of the base model by a
   more literal reading of the paper.  Every variant, the directory and migration included, and
   a router delay above 1 run on both the one-tile-per-thread kernel and the general one.
   AGE_DEFLECT: a flit's priority is the number of times it has been deflected (more first,
     0 at injection; Sec. 4.2, Sec. 6.2.1, Sec. 7.1 phase two), ties by (injection cycle,
     source).  The base model ranks by (injection cycle, source) alone.  A flit deflected
     65,536 times stops the run with SIM_EINVARIANT.
   HIT_UNDER_MISS: a core with a miss outstanding keeps drawing ops; an L1 hit completes at
     once, a second miss is held and looked up again the cycle after the first is filled,
     its latency counted from its first issue (Sec. 3.5).
   INJECT_DELAY: requests and replies pass through the router's injection register and can
     enter the network only from the cycle after they are made (Sec. 6.2.1, Sec. 7.1 phase
     three).
   LSPD: the paper's logically shared, physically distributed L2 with a directory (Sec. 3.2,
     3.4, 6.2.2, Table 1) instead of static homes.  A block lives in the slice of the core that
     brought it from memory; an L1 miss looks in the core's own slice, then sends a directory
     access (1 flit) to the line's directory slice (line mod N, or with LSPD_CENTRAL the tile
     at (width/2, height/2)); the directory answers (1 flit) with the owner, or negatively and
     records the asker as owner, which then brings the block from memory into its slice (after
     mem_lat); an owner answers a remote access with reply_flits flits, or with a trap (1 flit)
     if it has evicted the block, and the core asks the directory again; a slice that evicts a
     block sends an eviction notice (1 flit) that clears the entry.  Directory entries live in
     a location array of one int32 per line (shared_lines + N * private_lines entries). */
enum {
  SIM_FLAG_AGE_DEFLECT = 1, SIM_FLAG_HIT_UNDER_MISS = 2, SIM_FLAG_INJECT_DELAY = 4, SIM_FLAG_LSPD = 8,
  SIM_FLAG_LSPD_CENTRAL = 16
};

/* Statistics: 64 int64 counters (index = position in `v`).  Latencies are in cycles from
   injection to ejection; op latency from issue to L1 fill. */
enum {
  SIM_ST_CYCLES = 0,
  SIM_ST_INJ_REQ = 1, SIM_ST_INJ_REPLY = 2, SIM_ST_INJ_BG = 3,
  SIM_ST_EJ_REQ = 4, SIM_ST_EJ_REPLY = 5, SIM_ST_EJ_BG = 6,
  SIM_ST_LAT_REQ = 7, SIM_ST_LAT_REPLY = 8, SIM_ST_LAT_BG = 9,
  SIM_ST_LAT_MAX = 10,
  SIM_ST_TRAVERSALS = 11,   /* flits sent over a link */
  SIM_ST_DEFLECTIONS = 12,  /* flits sent over a non-productive link */
  SIM_ST_OPS_ISSUED = 13, SIM_ST_OPS_DONE = 14, SIM_ST_OP_LAT = 15,
  SIM_ST_L1_HIT = 16, SIM_ST_L1_MISS = 17, SIM_ST_L2_HIT = 18, SIM_ST_L2_MISS = 19,
  SIM_ST_REQ_MADE = 20, SIM_ST_REQ_RECV = 21, SIM_ST_REPLY_SENT = 22, SIM_ST_REPLY_RECV = 23,
  SIM_ST_INJ_BLOCKED = 24,  /* tile-cycles with a flit to inject but no free input */
  SIM_ST_BG_GEN = 25, SIM_ST_OP_LAT_MAX = 26,
  SIM_ST_DIR_ACCESS = 27,   /* LSPD: directory look-ups (remote and local) */
  SIM_ST_DIR_NACK = 28,     /* LSPD: negative directory answers = blocks brought from memory */
  SIM_ST_TRAP = 29,         /* LSPD: stale directory answers (owner without the block) */
  SIM_ST_DIR_EVICT = 30,    /* LSPD: directory entries cleared by evictions */
  SIM_ST_HIST = 32,         /* 16 bins of floor(log2(latency)); the last bin is open */
  SIM_ST_MIGRATE = 48,      /* blocks migrated (Sec. 3.3) */
  SIM_ST_REDIRECT = 49,     /* requests redirected by a block's previous owner */
  SIM_ST_COUNT = 64
};
typedef struct { int64_t v[SIM_ST_COUNT]; } sim_stats_t;

typedef struct sim_chip sim_t;    /* one chip */
typedef struct sim_group simb_t;  /* many chips advanced by one launch */

/* Bytes of device state for one chip; 0 if the config is invalid.  Zipf tables are
   included. */
size_t sim_state_bytes(const sim_config* cfg);

/* The reciprocal constants the kernels divide by instead of a divide instruction (host-only,
   touches no device): out[0] = ceil(2^32 / width), so that tile / width = umulhi(tile, out[0])
   for tile < 2^20 (0 when width = 1); out[2], out[3] = ceil(2^(32+k) / tiles) and k =
   floor(log2 tiles) - 1, so that line / tiles = umulhi(line, out[2]) >> k for line < 2^30, which
   gives a line's home (line mod tiles) and its L2 set ((line / tiles) mod l2_sets) (0, 0 when
   tiles = 1); out[1] = 0.  EINVAL for width or tiles < 1. */
int sim_div_constants(int32_t width, int32_t tiles, uint32_t* out);

/* Creates one chip in `dev_mem` and initialises it (all links empty, cores idle, caches
   invalid, cycle 0).  zipf_shared / zipf_private: host arrays of zipf_k + 1 (= 65537)
   uint32 quantile boundaries (entry b = first rank whose CDF exceeds b/zipf_k; entry
   zipf_k = region size); zipf_private may be NULL when private_lines == 0.  Copied.  EINVAL
   when a table decreases or its last entry exceeds its region's size. */
int sim_create(const sim_config* cfg, const uint32_t* zipf_shared, const uint32_t* zipf_private,
               int32_t zipf_k, void* dev_mem, size_t bytes, void* stream, sim_t** out);

/* Advances the chip by n_cycles whole cycles (Sec. 7.1 main loop; each cycle = phase one
   memory access, phase two arbitration, phase three traversal/ejection/injection for all
   tiles).  dev_digests: NULL, or a device array of n_cycles uint64 that receives the state
   digest of each cycle (sum over tiles of a SplitMix64 chain over the tile's input slots and
   core words); asks for a slower checking launch.  Asynchronous. */
int sim_step(sim_t* h, int64_t n_cycles, uint64_t* dev_digests);

/* Waits for the chip's stream and reports SIM_EHANG if a cross-workgroup wait timed out. */
int sim_sync(sim_t* h);

/* Cycles run so far (counting steps already enqueued). */
int64_t sim_cycle(const sim_t* h);

/* Statistics of the chip (synchronises): the counts the paper's simulator reports (Sec. 6.2.2;
   requests made and received, replies sent and received, traps, as in Table 3) together with
   the latency, traffic and cache counters listed above. */
int sim_stats(sim_t* h, sim_stats_t* out);

/* Canonical state (synchronises): everything the cycle loop of Sec. 7.1 carries from one cycle
   to the next (the paper keeps no checkpoint; this one is for checkpoint / resume and for
   comparing simulators word by word).  16-word header {magic 0x4E4F4353, version 4, width,
   height, cycle lo, cycle hi, l1_sets, l1_ways, l2_sets, l2_ways, reply_flits (>= 1),
   core-record words (28), flags, router delay, LSPD mode (0 static homes, 1 interleaved
   directory, 2 central), migration threshold}, then per tile the 4 input slots of the next
   cycle ({dst (-1 = empty), inject cycle (bit 31: LSPD control flit), source, kind<<30 |
   line}), then per tile 28 core words {state, wake, line, issue, l2q, l2q_line, hit_head,
   hit_tail, miss_head, miss_tail, bg_pending, node_next, node_ready, node_line, force_line,
   force_dst, reply flits received, node flits sent, held line (-1 = none), held issue cycle,
   remote-access target, pending eviction line, directory checksum lo, hi, pending claim,
   forwarded line, its destination (| 0x40000000 while the block is on its way), the tile to
   tell of a migrated block's arrival}, then L1 and L2 tags per tile per
   set (most recently used first, -1 invalid), then the 64 statistics as (low, high) word
   pairs, then per tile the deflection counts of the 4 input slots' flits (0 when empty or
   without AGE_DEFLECT), then, when router_delay D > 1 (header word 13 = D), the routers'
   pipelines: stages k = 1..D-1 (stage k holds the flits arbitrated k-1 cycles after the
   dump's cycle), each as per tile 4 slots of 4 words, then the stages' deflection counts,
   then with LSPD the location array (owner tile per line, -1 = not on chip), then with
   migration the last migration-threshold accessors of every L2 way (most recent first, -1
   none), in the order of the L2 tags.
   sim_dump_words() gives the size in int32 words. */
size_t sim_dump_words(const sim_t* h);
int sim_dump(sim_t* h, int32_t* host_buf, size_t words);
/* Restores a canonical state produced by sim_dump (checkpoint / resume) and clears an error
   recorded by an earlier step (the state it belonged to is replaced).  EINVAL when the header
   does not match the chip (shape, caches, reply_flits, flags) or a word is out of range. */
int sim_load(sim_t* h, const int32_t* host_buf, size_t words);

/* Test hooks (synchronise): make `tile` issue a memory op on `line` at its next idle cycle;
   make `tile` inject a background flit to `dst` (priority just above random background). */
int sim_force_op(sim_t* h, int32_t tile, int32_t line);
int sim_force_bg(sim_t* h, int32_t tile, int32_t dst);
/* Changes the op-issue and background thresholds from the next step on (0, 0 = drain). */
int sim_set_rates(sim_t* h, uint32_t op_thr, uint32_t bg_thr);
/* Test hook for the time-out path (the behaviour of a stuck workgroup, forced from the host):
   patch `patch` (0 .. patches-1 of the current launch mapping; -1 = none) advances no further
   than cycle `cycle`, and a wait for a neighbouring patch's link slot gives up after `polls`
   polls (0 = the default, 2^25).  A wait that gives up records a hang in the chip's error word
   and ends its workgroup's launch; waiting neighbours see the error word and stop too, so every
   workgroup exits normally and sim_sync / sim_stats report SIM_EHANG.  The chip's state is then
   invalid until sim_load (which clears the error; call with patch -1 first). */
int sim_force_hang(sim_t* h, int32_t patch, int32_t cycle, int32_t polls);
/* Watchdog, a debug mode (the model has no such check; the paper's oldest-first priority is
   what makes a flit's age bounded, Sec. 4.2): with max_age > 0 every step of this chip checks,
   for every router in every cycle, that each of its flits left by exactly one port and that no
   flit waiting at it is older (current cycle - injection cycle) than max_age.  A violation
   stops the chip: SIM_ELIVELOCK for the age, SIM_EINVARIANT for a lost or duplicated flit
   (state invalid until sim_load).  The one-tile-per-thread kernel then runs its checking build
   (slower); results are otherwise unchanged.  Applies to sim_step, not to batches.  0 = off
   (the default). */
int sim_set_watchdog(sim_t* h, int32_t max_age);

/* Launch mapping: patch_w x patch_h tiles per workgroup (the chip is cut into patches; a tile
   on a patch edge waits for its neighbour's link slot to carry the cycle it needs, so patches
   synchronise with their neighbours only), `block` threads per workgroup (64..256, a multiple of 64),
   `chunk` cycles per launch.  0 keeps the current value.  EINVAL if the patch grid cannot
   be resident on the device at once.  sim_create's default: one workgroup for chips of at
   most 1,024 tiles; otherwise one row per workgroup of 64 or 128 threads (a row cut into
   equal strips of at most 128 tiles; whole rows up to 256 tiles below 64 columns) when the
   chip's own builds of the step kernel can hold all of them at once; otherwise square-ish
   patches, about one per compute unit; chunk 1,000. */
int sim_set_launch(sim_t* h, int32_t patch_w, int32_t patch_h, int32_t block, int32_t chunk);
int sim_get_launch(const sim_t* h, int32_t* patch_w, int32_t* patch_h, int32_t* block, int32_t* chunk);
/* Kernel choice: when every patch has at most `block` tiles the library runs a kernel that keeps
   one tile per thread in registers and interior links in LDS; generic_only = 1 forces the
   general kernel (several tiles per thread, all state in HBM).  Both give identical results. */
int sim_set_kernel(sim_t* h, int32_t generic_only);

int sim_destroy(sim_t* h);
const char* sim_strerror(int code);
int sim_last_hip_error(void);

/* ---- batches: many independent chips advanced by one persistent launch ----------------
   The batched step of many independent simulations (each chip is the paper's whole simulated
   system, Sec. 7.1; chips share nothing).  A batch groups chips created with sim_create (each
   in its own buffer) so that one launch advances all of them: workgroup w runs one patch of
   one chip, and chips never wait on each other.  The batch keeps a launch table and one error
   word per chip in a caller-owned device workspace of simb_state_bytes(max_chips,
   max_patches) bytes (256-byte aligned), sized for the most chips and patches it will ever
   hold.  The batch launches on its own stream; the caller orders any per-chip call with it.
   Chips keep their own launch mapping, except the workgroup size, which is the batch's
   `block`.  A chip cut into several patches needs all of its workgroups resident at once.
   Chips are identified by slot numbers 0 .. simb_slots()-1; a slot freed by simb_remove is
   reused by the next simb_add.  A chip belongs to at most one batch; the batch never frees a
   chip.  Not thread safe. */
size_t simb_state_bytes(int32_t max_chips, int64_t max_patches);  /* 0 if invalid */
/* Creates a batch of n >= 0 chips in slots 0..n-1.  block: threads per workgroup (64..256, a
   multiple of 64; 0 = the largest of the chips', which needs n > 0).  max_chips / max_patches:
   capacity of the workspace (0 = exactly the n chips given).  EINVAL when a chip of several
   patches cannot be resident under the batch's kernel, ENOMEM when `bytes` is too small. */
int simb_create(sim_t* const* chips, int32_t n, int32_t block, int32_t max_chips, int64_t max_patches,
                void* dev_mem, size_t bytes, void* stream, simb_t** out);
/* Continuous batching (a served job joins or leaves between steps).  simb_add puts `chip` in
   the lowest free slot (*slot); EBUSY when the workspace cannot hold it, EINVAL when it is
   already in the batch or cannot be resident.  simb_remove takes the chip in `slot` out (the
   chip itself stays valid and keeps its state). */
int simb_add(simb_t* b, sim_t* chip, int32_t* slot);
int simb_remove(simb_t* b, int32_t slot);
int32_t simb_slots(const simb_t* b);  /* number of slot numbers in use (free ones included) */
/* Statistics of the chip in `slot` (as sim_stats; synchronises). */
int simb_stats(simb_t* b, int32_t slot, sim_stats_t* out);
/* Advances the chip in slot i by cycles[i] >= 0 cycles (host array of simb_slots() entries;
   free slots' entries are ignored), one persistent launch per launch group per `chunk` cycles
   (the smallest chunk of the members); chips that need fewer cycles stop early.  Returns once
   the step has finished, with SIM_EHANG / SIM_EINVARIANT if a chip reported one. */
int simb_step(simb_t* b, const int64_t* cycles);
/* on = 1: simb_step replays one chunk of every launch group as a HIP graph (one kernel node
   per launch group, chained; groups of multi-patch chips are cooperative nodes), built on the
   first step and rebuilt after a membership or chunk change, instead of launching the chunks
   one by one.  Results are identical either way. */
int simb_set_graph(simb_t* b, int32_t on);
int simb_destroy(simb_t* b);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): the batched step of simb_create + simb_step in one
   call, with the launch table and the per-chip error words in a static device array of the
   library (about 516 KB per GPU, held until the process ends) instead of a caller workspace.
   Advances chips[i] by cycles[i] >= 0 cycles (n chips, distinct, created with sim_create on the
   current device); block as in simb_create.  Launches on `stream` and synchronises it; returns
   SIM_EHANG / SIM_EINVARIANT as simb_step does.  At most 1024 chips and 32768 patches in total
   per call: more is refused with SIM_ENOMEM before anything runs.  The call allocates nothing
   (no hipMalloc, hipFree or library allocation).  Every call on one GPU shares that GPU's array:
   calls that overlap on one GPU (other threads, other streams) race and are not allowed. */
int simb_step_noalloc(sim_t* const* chips, int32_t n, int32_t block, const int64_t* cycles, void* stream);

#ifdef __cplusplus
}
#endif
#endif
