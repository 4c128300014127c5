// MI355X (gfx950) simulator of a bufferless deflection-routed 2D-mesh chip multicore with a
// statically homed, set-associative LRU L2: the per-cycle step over every tile.
//
// Method: Kumar & Sahu, "Bufferless NOC Simulation of Large Multicore System on GPU Hardware"
// (arXiv 1508.03235).  Each cycle runs, for every tile, the paper's three phases (Sec. 7.1):
// the memory access (private L1, then the line's home L2 slice; Sec. 3.1-3.5), oldest-first
// bufferless deflection arbitration (Sec. 4.2-4.3, Sec. 6.2.1) and link traversal with
// ejection and injection.
//
// GPU design (not the paper's three kernels per cycle): one persistent launch runs many
// cycles.  A chip is cut into rectangular patches, one workgroup per patch.  The only state
// crossing a patch edge within a cycle is a link slot, so workgroups synchronise with their
// (up to four) neighbouring patches only, through the slots themselves: every slot word
// carries the cycle it is an input of (a stamp), and a tile on a patch edge polls its
// neighbour's slot until it holds the cycle it needs.  A per-patch flag records the cycles a
// patch has completed, written at the end of a launch (the next launch starts from it).  A
// chip that fits one workgroup needs no cross-workgroup synchronisation at all.  State is structure-of-arrays int32 in HBM:
// link slots double-buffered by cycle parity, core words, reply-queue nodes, L1/L2 tag sets
// stored most-recently-used first (a set is one or two 16-byte vectors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "nocsim.h"

namespace {

// ---- encodings ---------------------------------------------------------------------------
// With the LSPD directory, KIND_DIR flits are directory accesses or (control bit) eviction
// notices, and KIND_REPLY flits with the control bit are directory answers or traps; the control
// bit is bit 31 of the inject-cycle word (cycles stay below 2^31).
constexpr int KIND_REQ = 0, KIND_REPLY = 1, KIND_BG = 2, KIND_DIR = 3;
constexpr int CORE_IDLE = 0, CORE_L1MISS = 1, CORE_SEND = 2, CORE_WAIT = 3, CORE_FILL = 4;
constexpr int CORE_SEND_DA = 5, CORE_SEND_RA = 6, CORE_FILL_MEM = 7, CORE_FILL_MIG = 8;  // LSPD
constexpr uint32_t CTL_BIT = 0x80000000u;
// answers (queue node line word, sent as code + CODE_BASE): claim acknowledged, a flit of a
// migrating block, trap, negative directory answer, or an owner tile >= 0
constexpr int CODE_ACK = -4, CODE_MIG = -3, CODE_TRAP = -2, CODE_NACK = -1, CODE_BASE = 4;
// message types at a slice's service input (l2q >> 24): remote access, directory access, eviction
// notice, ownership claim, a migrated block's arrival at its new owner
constexpr int Q_RA = 0, Q_DA = 1, Q_EV = 2, Q_CLAIM = 3, Q_ARRIVED = 4;
// A chip's error word: 0 none, 1 a bounded wait ran out, 2 a state index out of range, 3 an
// interior slot from the wrong cycle, 4 a deflection count past its 16 bits, and with the
// watchdog on, ERR_WATCHDOG a flit older than its bound and ERR_ROUTER a router whose flits
// did not each leave by exactly one port.
constexpr int ERR_WATCHDOG = 5, ERR_ROUTER = 6;
// migration (Sec. 3.3): a block moves as 16 flits (Table 1); a queued reply that is a migration
// carries MIG_MARK on its line word; each L2 way keeps its last `mig` accessors (most recent
// first, -1 none), in the ways' order; while a block a slice sends away is on its way, the
// slice's forwarding destination carries MIG_TRANSIT
constexpr int MIG_FLITS = 16;
constexpr int MIG_MARK = 0x40000000;
constexpr int MIG_TRANSIT = 0x40000000;
constexpr int MIG_MAX = 16;  // longest access history
constexpr int32_t LINE_MASK = 0x3FFFFFFF;
// words of a tile's record in the canonical dump: state, wake, line, issue, l2q, l2q_line,
// hit head/tail, miss head/tail, bg_pending, node next/ready/line, force_line, force_dst,
// reply flits received, node flits sent, held line, held issue cycle, remote-access target,
// pending eviction line, directory checksum (low, high), pending claim, forwarded line, its
// destination, a spare word
constexpr int CORE_RECORD = 28;
constexpr int DUMP_VERSION = 4;
// model variants (sim_config.flags)
constexpr int32_t VARIANT_FLAGS = SIM_FLAG_AGE_DEFLECT | SIM_FLAG_HIT_UNDER_MISS | SIM_FLAG_INJECT_DELAY | SIM_FLAG_LSPD |
                                  SIM_FLAG_LSPD_CENTRAL;
constexpr int AGE_MAX = 0xFFFF;  // deflections a flit may take; one more stops the run (livelock)
constexpr int ZIPF_K = 65536;
constexpr int MAX_PATCHES = 4096;
constexpr int FLAG_STRIDE = 32;  // ints between patch flags (128 B)
constexpr int NSTAT = SIM_ST_COUNT;
constexpr int SPIN_LIMIT = 1 << 25;  // polls before a neighbour wait is declared hung

// Device descriptor of one chip; lives at the start of the chip's buffer.
struct ChipDev {
  int32_t W, H, N, n_patches;
  uint32_t key0, key1, op_thr, shared_thr;
  uint32_t bg_thr, w_magic;  // w_magic = ceil(2^32 / W) (W > 1): tile / W = umulhi(tile, w_magic)
  uint32_t n_magic, n_shift; // line / N = umulhi(line, n_magic) >> n_shift for line < 2^30, N >= 2
  int32_t w1_shift, w2_shift; // log2 of the way counts
  int32_t s1, w1, s2, w2;
  int32_t l1_lat, mem_lat, shared_lines, private_lines;
  int32_t reply_flits;       // flits per reply packet (Sec. 3.6, Table 1); 1 = single-flit replies
  int32_t variants;          // SIM_FLAG_* model variants
  int32_t inj_delay;         // 1 when a flit can enter the network only the cycle after it is made
  int32_t rdelay;            // router delay D >= 1: cycles per hop
  int32_t lspd;              // 0 static homes; 1 LSPD, directory interleaved by line; 2 central directory
  int32_t dir_center;        // the central directory's tile
  int32_t lines;             // line space: shared_lines + N * private_lines
  int32_t mig;               // migration threshold (0 = none)
  int32_t pw, ph, pgx, pgy;  // patch shape and patch grid
  int32_t stop, max_patches; // cycle the chip stops at (single-chip launches); flag capacity
  int32_t spin_limit;        // polls before a cross-workgroup wait gives up (reports a hang)
  int32_t watch_age;         // watchdog (debug): 0 off; else the oldest age a flit may reach
  int32_t halt_patch, halt_cycle;  // test hook: this patch advances no further than halt_cycle
  int4* link;                // [2 parity][4 port][N]
  int4* pipe;                // [D-1][4 port][N]: raw slot words of flits waiting in the routers'
                             // pipelines; entry (a mod (D-1)) holds those arbitrated in cycle a
  int4* core;                // [6][N]; group 3: force_dst, reply flits received, held line, held issue;
                             // group 4 (LSPD): remote-access target, pending eviction, directory checksum lo, hi;
                             // group 5 (migration): pending claim, forwarded line, its destination, spare
  int32_t* l2h;              // migration: [N][s2][w2][mig] the last accessors of each L2 way
  int32_t* loc;              // LSPD location array [lines]: owner tile or -1; entry L belongs to L's directory tile
  int4* node;                // [N]: next, ready, line, reply flits already injected by the home
  int32_t* l1;               // [N][s1][w1]
  int32_t* l2;               // [N][s2][w2]
  const uint32_t* zs;
  const uint32_t* zp;
  int32_t* flags;                 // [n_patches * FLAG_STRIDE]: cycles completed by each patch
  unsigned long long* stats;      // [NSTAT]
  int32_t* err;                   // nonzero after a failed wait
};

// One workgroup's work item: a patch of a chip, and the cycle the chip stops at.
struct LaunchEntry {
  ChipDev* chip;
  int32_t patch;
  int32_t stop;
};

// All chip state is in device global memory; pointers are cast to the global address space so
// accesses compile to global (not flat) instructions with a scalar base.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int4 gload4(const int4* p) {
  const v4i v = *(const __attribute__((address_space(1))) v4i*)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore4(int4* p, const int4& a) {
  v4i v;
  v.x = a.x; v.y = a.y; v.z = a.z; v.w = a.w;
  *(__attribute__((address_space(1))) v4i*)p = v;
}
__device__ __forceinline__ int2 gload2(const int2* p) {
  const v2i v = *(const __attribute__((address_space(1))) v2i*)p;
  return make_int2(v.x, v.y);
}
__device__ __forceinline__ void gstore2(int2* p, const int2& a) {
  v2i v;
  v.x = a.x; v.y = a.y;
  *(__attribute__((address_space(1))) v2i*)p = v;
}

// ---- coherent access for state that crosses workgroups -------------------------------------
// Link slots on a patch edge and reply-queue nodes of a multi-patch chip are read and written
// by different workgroups, possibly on different XCDs; they use device-scope relaxed atomics,
// and stores are ordered before the cycle flag with s_waitcnt.
__device__ __forceinline__ int ld_coh(const int* p) {
  return __hip_atomic_load(gp(const_cast<int*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(int* p, int v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A wait that gave up: records a hang unless another workgroup already recorded an error (a
// workgroup that stops on an invariant failure leaves its neighbours waiting; its code is kept).
__device__ __forceinline__ void note_hang(int* err) {
  int none = 0;
  __hip_atomic_compare_exchange_strong(gp(err), &none, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int4 ld_slot(const int4* p, bool coh) {
  if (!coh) return gload4(p);
  unsigned long long* q = reinterpret_cast<unsigned long long*>(const_cast<int4*>(p));
  unsigned long long a = __hip_atomic_load(gp(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long b = __hip_atomic_load(gp(q + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_int4((int)(uint32_t)a, (int)(uint32_t)(a >> 32), (int)(uint32_t)b, (int)(uint32_t)(b >> 32));
}
__device__ __forceinline__ void st_slot(int4* p, int4 v, bool coh) {
  if (!coh) { gstore4(p, v); return; }
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(gp(q), (unsigned long long)(uint32_t)v.x | ((unsigned long long)(uint32_t)v.y << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(gp(q + 1), (unsigned long long)(uint32_t)v.z | ((unsigned long long)(uint32_t)v.w << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool COH> __device__ __forceinline__ void st_i(int* p, int v) { if (COH) st_coh(p, v); else *gp(p) = v; }

// ---- link-slot encoding -------------------------------------------------------------------------
// A slot holds a flit {dst, inject cycle, src, kind<<30 | line} for the cycle it is an input of.
// Tile indices take bits 0-19 of the dst and src words; bits 28-31 of both carry that cycle
// (mod 16), so each 64-bit half of a slot says by itself which cycle it belongs to.  A tile on a
// patch edge polls its neighbour's slot until both halves carry the cycle it needs: the data and
// the "ready" signal arrive together, with no separate flag and no store drain.  A slot is
// rewritten every second cycle, so the stamp it can hold besides the awaited cycle c is c-2.
// Bits 20-27 of the dst word and of the src word hold the low and high byte of the flit's
// deflection count (priority by deflection count; 0 otherwise).  An empty slot has 0xFFFFF in
// the tile bits of its dst word; its other words are not read (slot_encode writes src 0xFFFFF,
// count 0 and -1s, slot_encode_row leaves them as they come).
constexpr uint32_t TILE_BITS_MASK = 0xFFFFFu;
constexpr int AGE_SHIFT = 20;
constexpr int STAMP_SHIFT = 28;
constexpr uint32_t STAMP_MASK = 0xFu;

__device__ __forceinline__ int4 slot_encode(const int4& f, uint32_t stamp) {
  const uint32_t s = (stamp & STAMP_MASK) << STAMP_SHIFT;
  const bool empty = f.x < 0;  // selects, not a branch: every word of f is read either way
  return make_int4((int)((empty ? TILE_BITS_MASK : (uint32_t)f.x) | s), empty ? -1 : f.y,
                   (int)((empty ? TILE_BITS_MASK : (uint32_t)f.z) | s), empty ? -1 : f.w);
}
// The same for a flit row whose empty form has dst = -1 exactly (the other words of an empty
// row may be anything): two instructions, the stamp put over bits 28-31 of dst and src.
constexpr uint32_t STAMP_OFF = ~(STAMP_MASK << STAMP_SHIFT);
__device__ __forceinline__ int4 slot_encode_row(const int4& f, uint32_t stamp) {
  const uint32_t s = (stamp & STAMP_MASK) << STAMP_SHIFT;
  return make_int4((int)(((uint32_t)f.x & STAMP_OFF) | s), f.y, (int)(((uint32_t)f.z & STAMP_OFF) | s), f.w);
}
__device__ __forceinline__ int4 slot_encode_aged(const int4& f, uint32_t stamp, uint32_t age) {
  int4 w = slot_encode(f, stamp);
  if (f.x >= 0) {
    w.x |= (int)((age & 0xFFu) << AGE_SHIFT);
    w.z |= (int)((age >> 8) << AGE_SHIFT);
  }
  return w;
}
__device__ __forceinline__ uint32_t slot_age(const int4& w) {  // 0 for an empty slot (also all ones)
  if (((uint32_t)w.x & TILE_BITS_MASK) == TILE_BITS_MASK) return 0u;
  return (((uint32_t)w.x >> AGE_SHIFT) & 0xFFu) | ((((uint32_t)w.z >> AGE_SHIFT) & 0xFFu) << 8);
}
__device__ __forceinline__ int4 slot_decode(const int4& w) {
  const uint32_t d = (uint32_t)w.x & TILE_BITS_MASK;
  if (d == TILE_BITS_MASK) return make_int4(-1, -1, -1, -1);
  return make_int4((int)d, w.y, (int)((uint32_t)w.z & TILE_BITS_MASK), w.w);
}
// The same, keeping the deflection count in bits 20-27 of the dst and src words (the
// one-tile-per-thread kernel's flit rows under priority by deflection count).
__device__ __forceinline__ int4 slot_decode_aged(const int4& w) {
  if (((uint32_t)w.x & TILE_BITS_MASK) == TILE_BITS_MASK) return make_int4(-1, -1, -1, -1);
  return make_int4((int)((uint32_t)w.x & STAMP_OFF), w.y, (int)((uint32_t)w.z & STAMP_OFF), w.w);
}
// deflection count of such a row (0 when empty)
__device__ __forceinline__ uint32_t row_age(const int4& f) {
  if (f.x < 0) return 0u;
  return (((uint32_t)f.x >> AGE_SHIFT) & 0xFFu) | ((((uint32_t)f.z >> AGE_SHIFT) & 0xFFu) << 8);
}
// the row without its count
__device__ __forceinline__ int4 row_clean(const int4& f) {
  if (f.x < 0) return f;
  return make_int4((int)((uint32_t)f.x & TILE_BITS_MASK), f.y, (int)((uint32_t)f.z & TILE_BITS_MASK), f.w);
}
__device__ __forceinline__ int4 sel4(bool p, const int4& a, const int4& b) {  // p ? a : b, per word
  return make_int4(p ? a.x : b.x, p ? a.y : b.y, p ? a.z : b.z, p ? a.w : b.w);
}
// The same through a mask the optimizer cannot see through: selects between two records would
// otherwise be folded into one load from a selected address, which takes both out of registers.
__device__ __forceinline__ int4 pick4(bool p, const int4& a, const int4& b) {
  int m = -(int)p;
  asm volatile("" : "+v"(m));
  return make_int4((a.x & m) | (b.x & ~m), (a.y & m) | (b.y & ~m), (a.z & m) | (b.z & ~m), (a.w & m) | (b.w & ~m));
}
__device__ __forceinline__ bool slot_has_stamp(const int4& w, uint32_t stamp) {
  return ((uint32_t)w.x >> STAMP_SHIFT) == (stamp & STAMP_MASK) && ((uint32_t)w.z >> STAMP_SHIFT) == (stamp & STAMP_MASK);
}

// ---- counter-based randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -----------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    // one 32x32->64 product per multiplier (a single instruction for both halves)
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0, p1 = (unsigned long long)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    // three-input exclusive or in one instruction (gfx950 bitop3, truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96), n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Exact line / N and line mod N for lines < 2^30 without a divide: n_magic = ceil(2^(32+k) / N),
// k = floor(log2 N) - 1 (so n_magic < 2^32 and the rounding error stays below 1/N).
__device__ __forceinline__ uint32_t div_n(const ChipDev& C, uint32_t v) {
  return C.N > 1 ? __umulhi(v, C.n_magic) >> C.n_shift : v;
}
__device__ __forceinline__ uint32_t mod_n(const ChipDev& C, uint32_t v) { return v - div_n(C, v) * (uint32_t)C.N; }

// Zipf rank through a quantile table: bucket from the high half of u, linear position inside
// the bucket from the low half.
__device__ __forceinline__ int zipf_rank(const uint32_t* __restrict__ q, uint32_t u) {
  const uint32_t b = u >> 16, f = u & 0xFFFFu;
  const uint32_t lo = *gp(q + b), hi = *gp(q + b + 1);
  return (int)(lo + (uint32_t)(((unsigned long long)f * (hi - lo)) >> 16));
}

// ---- set-associative LRU sets: tags most recently used first -------------------------------
// Register copies of a set: load `ways` tags (positions >= ways read as -2, which no line
// matches), update in registers, store `ways` tags back.  `ways` is the same in every lane (one
// chip per workgroup); reading it from the first lane keeps the branches on it scalar even
// when the compiler has parked the value in a vector register.
__device__ __forceinline__ void set_load(const int* p, int ways, int (&v)[8]) {
  ways = __builtin_amdgcn_readfirstlane(ways);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = -2;
  if (ways == 8) {
    const int4 a = gload4(reinterpret_cast<const int4*>(p)), b = gload4(reinterpret_cast<const int4*>(p) + 1);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else if (ways == 4) {
    const int4 a = gload4(reinterpret_cast<const int4*>(p));
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else if (ways == 2) {
    const int2 a = gload2(reinterpret_cast<const int2*>(p));
    v[0] = a.x; v[1] = a.y;
  } else {
    v[0] = *gp(p);
  }
}
__device__ __forceinline__ void set_store(int* p, int ways, const int (&v)[8]) {
  ways = __builtin_amdgcn_readfirstlane(ways);
  if (ways == 8) {
    gstore4(reinterpret_cast<int4*>(p), make_int4(v[0], v[1], v[2], v[3]));
    gstore4(reinterpret_cast<int4*>(p) + 1, make_int4(v[4], v[5], v[6], v[7]));
  } else if (ways == 4) {
    gstore4(reinterpret_cast<int4*>(p), make_int4(v[0], v[1], v[2], v[3]));
  } else if (ways == 2) {
    gstore2(reinterpret_cast<int2*>(p), make_int2(v[0], v[1]));
  } else {
    *gp(p) = v[0];
  }
}
// Touch `line`: a hit moves it to the front; a miss inserts it at the front when `insert`,
// dropping the last way.  `changed` tells whether the set must be written back.
__device__ __forceinline__ bool set_touch(int (&v)[8], int ways, int line, bool insert, bool& changed) {
  ways = __builtin_amdgcn_readfirstlane(ways);
  int pos = 8;  // positions >= ways hold -2 and empty ways -1: neither matches a line (>= 0)
#pragma unroll
  for (int i = 7; i >= 0; --i)
    if (v[i] == line) pos = i;
  const bool hit = pos < 8;
  changed = false;
  if (pos == 0 || (!hit && !insert)) return hit;
  const int lim = hit ? pos : ways - 1;
#pragma unroll
  for (int i = 7; i >= 1; --i)
    if (i <= lim) v[i] = v[i - 1];
  v[0] = line;
  changed = true;
  return hit;
}

// LSPD slice ways with their access records (h, moved along when `rec`); positions are handled
// with unrolled selects so that the arrays stay in registers.
__device__ __forceinline__ int way_of(const int (&v)[8], int line) {
  int pos = -1;
#pragma unroll
  for (int i = 7; i >= 0; --i)
    if (v[i] == line) pos = i;
  return pos;
}
// (way i, 0 <= i < 8, as an OR of masked words: a chain of selects between the ways would be
// folded into one load at a computed offset, which takes the array out of registers)
__device__ __forceinline__ int way_pick(const int (&v)[8], int i) {
  int x = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) x |= v[k] & -(int)(i == k);
  return x;
}
__device__ __forceinline__ void way_front(int (&v)[8], int i) {
  const int tag = way_pick(v, i);
#pragma unroll
  for (int k = 7; k >= 1; --k)
    if (k <= i) v[k] = v[k - 1];
  v[0] = tag;
}
__device__ __forceinline__ void way_remove(int (&v)[8], int ways, int i) {
  ways = __builtin_amdgcn_readfirstlane(ways);
#pragma unroll
  for (int k = 0; k < 7; ++k)
    if (k >= i && k < ways - 1) v[k] = v[k + 1];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k == ways - 1) v[k] = -1;
}
// inserts `line` at the front; returns the way it pushed out (or -1)
__device__ __forceinline__ int way_insert(int (&v)[8], int ways, int line) {
  ways = __builtin_amdgcn_readfirstlane(ways);
  const int victim = way_pick(v, ways - 1);
#pragma unroll
  for (int k = 7; k >= 1; --k)
    if (k <= ways - 1) v[k] = v[k - 1];
  v[0] = line;
  return victim;
}

// Access histories of an LSPD slice's ways (migration, Sec. 3.3), in HBM beside the tags and in
// their order: `mig` words per way, most recent accessor first.  Only the slice's own tile
// reads or writes them, so they are plain loads and stores, applied at once.
__device__ __forceinline__ void hist_copy(int* dst, const int* src, int mig) {
  for (int m = 0; m < mig; ++m) *gp(dst + m) = *gp(src + m);
}
__device__ __forceinline__ void hist_clear(int* h, int mig) {
  for (int m = 0; m < mig; ++m) *gp(h + m) = -1;
}
// way i's history moves to the front (the ways before it move back one)
__device__ __forceinline__ void hist_front(int* h, int mig, int i) {
  int keep[MIG_MAX];
  for (int m = 0; m < mig; ++m) keep[m] = *gp(h + i * mig + m);
  for (int j = i; j > 0; --j) hist_copy(h + j * mig, h + (j - 1) * mig, mig);
  for (int m = 0; m < mig; ++m) *gp(h + m) = keep[m];
}
// way i's history goes (the ways after it move up one; the last is cleared)
__device__ __forceinline__ void hist_remove(int* h, int mig, int ways, int i) {
  for (int j = i; j < ways - 1; ++j) hist_copy(h + j * mig, h + (j + 1) * mig, mig);
  hist_clear(h + (ways - 1) * mig, mig);
}
// every way moves back one (the last is dropped); the front starts empty
__device__ __forceinline__ void hist_insert(int* h, int mig, int ways) {
  for (int j = ways - 1; j > 0; --j) hist_copy(h + j * mig, h + (j - 1) * mig, mig);
  hist_clear(h, mig);
}
// way i was accessed by `who`: recorded first; returns how many of the way's last `mig`
// accesses are who's
__device__ __forceinline__ int hist_note(int* h, int mig, int i, int who) {
  int* w = h + i * mig;
  int n = 1;
  for (int m = mig - 1; m > 0; --m) {
    const int v = *gp(w + m - 1);
    *gp(w + m) = v;
    n += v == who;
  }
  *gp(w) = who;
  return n;
}

// Queue nodes {next, ready, line, 0}: device-scope atomics when several workgroups share a chip.
template <bool COH> __device__ __forceinline__ int4 ld_node(const int4* p) { return ld_slot(p, COH); }
template <bool COH> __device__ __forceinline__ void st_node(int4* p, int4 v) { st_slot(p, v, COH); }

// Per-workgroup counters in LDS (rare events) and per-thread counters in registers (every
// cycle: link traversals, deflections, injections, ejections, latency sums).
struct LdsStats {
  unsigned long long v[NSTAT];
};
struct Acc {
  int trav, defl;
  int inj_req, inj_reply, inj_bg, ej_req, ej_reply, ej_bg;
  unsigned long long lat_req, lat_reply, lat_bg;
  // events counted in registers by the one-tile-per-thread kernel
  int l2_hit, l2_miss, ops_done, ops_issued, l1_hit, l1_miss, req_made, inj_blocked, reply_sent, req_recv,
      reply_recv, bg_gen, lat_max, op_lat_max;
  unsigned long long op_lat;
};
__device__ __forceinline__ void lds_add(LdsStats& L, int i, unsigned long long d) { atomicAdd(&L.v[i], d); }

// ---- one tile, one cycle ---------------------------------------------------------------------
// Phase one (Sec. 7.1, memory access), phase two (arbitration) and phase three (traversal,
// ejection, injection) of tile t in cycle c.  Reads the input slots of parity c, writes the
// neighbours' slots of parity c+1; every other word it writes is owned by t, except the
// queue nodes of requesters queued at t (t is their home while they wait).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {  // SplitMix64 finalizer
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ unsigned long long mix_pair(unsigned long long h, int a, int b) {
  return mix64(h ^ (((unsigned long long)(uint32_t)a << 32) | (uint32_t)b));
}

// VAR: 0 = the base model only; 1 = model variants and router delay; 2 = also the LSPD
// directory (the paths a level does not need are compiled out)
template <bool MULTI, int VAR>
__device__ __forceinline__ bool tile_step(const ChipDev& C, int t, int x, int y, int c, const bool cross[4], bool step,
                                          bool digest, unsigned long long& dsum, Acc& acc, LdsStats& L) {
  const int N = C.N;
  const int cur = c & 1, nxt = cur ^ 1;
  const bool v0 = y > 0, v1 = y < C.H - 1, v2 = x < C.W - 1, v3 = x > 0;
  const int4 EMPTY = make_int4(-1, -1, -1, -1);

  // inputs of cycle c: interior slots were written by this workgroup before its last barrier;
  // edge slots are polled until both halves carry cycle c
  const int4* in0 = &C.link[(cur * 4 + 0) * N + t];
  const int4* in1 = &C.link[(cur * 4 + 1) * N + t];
  const int4* in2 = &C.link[(cur * 4 + 2) * N + t];
  const int4* in3 = &C.link[(cur * 4 + 3) * N + t];
  const bool e0 = MULTI && cross[0] && v0, e1 = MULTI && cross[1] && v1, e2 = MULTI && cross[2] && v2,
             e3 = MULTI && cross[3] && v3;
  int4 w0 = v0 ? ld_slot(in0, e0) : EMPTY;
  int4 w1 = v1 ? ld_slot(in1, e1) : EMPTY;
  int4 w2 = v2 ? ld_slot(in2, e2) : EMPTY;
  int4 w3 = v3 ? ld_slot(in3, e3) : EMPTY;
  if (MULTI) {
    int spins = 0;
    for (;;) {
      const bool p0 = e0 && !slot_has_stamp(w0, (uint32_t)c), p1 = e1 && !slot_has_stamp(w1, (uint32_t)c);
      const bool p2 = e2 && !slot_has_stamp(w2, (uint32_t)c), p3 = e3 && !slot_has_stamp(w3, (uint32_t)c);
      if (!(p0 | p1 | p2 | p3)) break;
      if ((++spins & 63) == 0 && (spins > C.spin_limit || ld_coh(C.err))) {
        note_hang(C.err);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
      if (p0) w0 = ld_slot(in0, true);
      if (p1) w1 = ld_slot(in1, true);
      if (p2) w2 = ld_slot(in2, true);
      if (p3) w3 = ld_slot(in3, true);
    }
  }
  if ((v0 && !e0 && !slot_has_stamp(w0, (uint32_t)c)) || (v1 && !e1 && !slot_has_stamp(w1, (uint32_t)c)) ||
      (v2 && !e2 && !slot_has_stamp(w2, (uint32_t)c)) || (v3 && !e3 && !slot_has_stamp(w3, (uint32_t)c))) {
    st_coh(C.err, 3);  // an interior slot from the wrong cycle: a synchronisation bug
    return false;
  }
  // Router delay D > 1: this cycle's arrivals wait D-1 cycles in the router's pipeline; the
  // flits arbitrated now are the ones that arrived D-1 cycles ago (stored below, in phase three)
  const int4 a0w = w0, a1w = w1, a2w = w2, a3w = w3;
  int4* pipe_now = nullptr;
  if (VAR && C.rdelay > 1) {
    pipe_now = &C.pipe[(size_t)((uint32_t)c % (uint32_t)(C.rdelay - 1)) * 4 * N + t];
    w0 = v0 ? gload4(pipe_now) : EMPTY;
    w1 = v1 ? gload4(pipe_now + N) : EMPTY;
    w2 = v2 ? gload4(pipe_now + 2 * N) : EMPTY;
    w3 = v3 ? gload4(pipe_now + 3 * N) : EMPTY;
  }
  int4 f0 = v0 ? slot_decode(w0) : EMPTY;
  int4 f1 = v1 ? slot_decode(w1) : EMPTY;
  int4 f2 = v2 ? slot_decode(w2) : EMPTY;
  int4 f3 = v3 ? slot_decode(w3) : EMPTY;
  int4 k0 = gload4(&C.core[t]);          // state, wake, line, issue
  int4 k1 = gload4(&C.core[N + t]);      // l2q, l2q_line, hit_head, hit_tail
  int4 k2 = gload4(&C.core[2 * N + t]);  // miss_head, miss_tail, bg_pending, force_line
  const int4 k3 = gload4(&C.core[3 * N + t]);  // force_dst, reply flits received, held op
  int fdst = k3.x, rcv = k3.y, hline = k3.z, hissue = k3.w;
  const bool aged = VAR && (C.variants & SIM_FLAG_AGE_DEFLECT);
  const int rdelay = VAR ? C.rdelay : 1, inj_delay = VAR ? C.inj_delay : 0;
  const bool lspd = VAR == 2 && C.lspd != 0;
  // LSPD core words: remote-access target, pending eviction, directory checksum (constant
  // -1, -1, 0, 0 without the directory)
  int4 k4 = lspd ? gload4(&C.core[4 * N + t]) : make_int4(-1, -1, 0, 0);
  // migration words: pending claim, forwarded line, its destination, spare (all -1 without)
  int4 k5 = lspd ? gload4(&C.core[5 * N + t]) : make_int4(-1, -1, -1, -1);
  const bool mig = lspd && C.mig > 0;
  const uint32_t a0 = aged && v0 ? slot_age(w0) : 0u, a1 = aged && v1 ? slot_age(w1) : 0u;
  const uint32_t a2 = aged && v2 ? slot_age(w2) : 0u, a3 = aged && v3 ? slot_age(w3) : 0u;

  if (digest) {  // state owned by t after cycle c-1: its inputs of cycle c, its core words, its pipeline
    unsigned long long h = mix64(((unsigned long long)(uint32_t)(c - 1) << 32) | (uint32_t)t);
    auto mix_slots = [&](const int4& x0, const int4& x1, const int4& x2, const int4& x3) {
      const int4 g0 = v0 ? slot_decode(x0) : EMPTY, g1 = v1 ? slot_decode(x1) : EMPTY;
      const int4 g2 = v2 ? slot_decode(x2) : EMPTY, g3 = v3 ? slot_decode(x3) : EMPTY;
      h = mix_pair(h, g0.x, g0.y); h = mix_pair(h, g0.z, g0.w);
      h = mix_pair(h, g1.x, g1.y); h = mix_pair(h, g1.z, g1.w);
      h = mix_pair(h, g2.x, g2.y); h = mix_pair(h, g2.z, g2.w);
      h = mix_pair(h, g3.x, g3.y); h = mix_pair(h, g3.z, g3.w);
    };
    auto mix_ages = [&](const int4& x0, const int4& x1, const int4& x2, const int4& x3) {
      const uint32_t b0 = v0 ? slot_age(x0) : 0u, b1 = v1 ? slot_age(x1) : 0u;
      const uint32_t b2 = v2 ? slot_age(x2) : 0u, b3 = v3 ? slot_age(x3) : 0u;
      h = mix_pair(h, (int)(b0 | (b1 << 16)), (int)(b2 | (b3 << 16)));
    };
    mix_slots(a0w, a1w, a2w, a3w);
    h = mix_pair(h, k0.x, k0.y); h = mix_pair(h, k0.z, k0.w);
    h = mix_pair(h, k1.x, k1.y); h = mix_pair(h, k1.z, k1.w);
    h = mix_pair(h, k2.x, k2.y);
    h = mix_pair(h, k2.z, 0);   // bg_pending; the queue-node words are written by the home
    h = mix_pair(h, 0, 0);
    h = mix_pair(h, k2.w, fdst);
    h = mix_pair(h, rcv, 0);    // reply flits received; the node's sent count is the home's
    h = mix_pair(h, hline, hissue);
    h = mix_pair(h, k4.x, k4.y);
    h = mix_pair(h, k4.z, k4.w);
    h = mix_pair(h, k5.x, k5.y);
    h = mix_pair(h, k5.z, k5.w);
    if (aged) mix_ages(a0w, a1w, a2w, a3w);
    for (int st = 1; st < rdelay; ++st) {  // stage st: the flits arbitrated in cycle c-1+st
      const int4* pp = &C.pipe[(size_t)(((uint32_t)c + (uint32_t)(st - 1)) % (uint32_t)max(rdelay - 1, 1)) * 4 * N + t];
      const int4 x0 = v0 ? gload4(pp) : EMPTY, x1 = v1 ? gload4(pp + N) : EMPTY;
      const int4 x2 = v2 ? gload4(pp + 2 * N) : EMPTY, x3 = v3 ? gload4(pp + 3 * N) : EMPTY;
      mix_slots(x0, x1, x2, x3);
      if (aged) mix_ages(x0, x1, x2, x3);
    }
    dsum += h;
  }
  if (!step) return true;
  bool d0 = false, d1 = false, d2 = false, d3 = false;
  const uint4 r = philox((uint32_t)c, (uint32_t)t, 0u, 0u, C.key0, C.key1);

  // ---- every load of the cycle is issued before any store -----------------------------------
  // Indices read from state are checked before they address memory: a corrupt index sets the
  // chip's error word (reported as SIM_EINVARIANT) instead of faulting.
#define GUARD(i)                                                   \
  if ((unsigned)(i) >= (unsigned)N) {                              \
    st_coh(C.err, 2);                                              \
    return false;                                                  \
  }
#define GUARD_LINE(l)                                              \
  if ((unsigned)(l) >= (unsigned)C.lines) {                        \
    st_coh(C.err, 2);                                              \
    return false;                                                  \
  }
  const bool svc = k1.x >= 0;  // a request was ejected here last cycle: home-slice lookup
  const int svc_type = lspd ? (k1.x >> 24) : Q_RA, svc_who = lspd ? (k1.x & 0xFFFFFF) : k1.x;
  if (svc) { GUARD(svc_who) }
  if (lspd && svc) { GUARD_LINE(k1.y) }
  if (lspd && k4.x >= 0) { GUARD(k4.x) }
  if (lspd && k4.y >= 0) { GUARD_LINE(k4.y) }
  if (lspd && k5.x >= 0) { GUARD_LINE(k5.x) }
  if (lspd && k5.z >= 0) { GUARD(k5.z & ~MIG_TRANSIT) }
  if (lspd && k5.w >= 0) { GUARD(k5.w) }
  if (k1.z >= 0) { GUARD(k1.z) }
  if (k1.w >= 0) { GUARD(k1.w) }
  if (k2.x >= 0) { GUARD(k2.x) }
  if (k2.y >= 0) { GUARD(k2.y) }
  const bool wake = k0.y == c;
  // LSPD: a block from memory, or one that migrated here, goes into the slice
  const bool fill_mem = lspd && (k0.x == CORE_FILL_MEM || k0.x == CORE_FILL_MIG) && wake;
  const bool fill_mig = fill_mem && k0.x == CORE_FILL_MIG;
  const bool fill = (k0.x == CORE_FILL && wake) || fill_mem;
  const bool missed = k0.x == CORE_L1MISS && wake;
  const bool local = !lspd && missed && mod_n(C, (uint32_t)k0.z) == (uint32_t)t;
  // LSPD: the core's own slice (after an L1 miss, unless an eviction notice is still pending,
  // and when a block from memory is installed) and the directory entries this cycle touches
  auto dir_of = [&](int line) -> int { return C.lspd == 2 ? C.dir_center : (int)mod_n(C, (uint32_t)line); };
  const bool slice_look = lspd && missed && k4.y < 0 && k5.x < 0;
  if (slice_look || fill_mem) { GUARD_LINE(k0.z) }
  const bool dir_core = (slice_look || fill_mig) && dir_of(k0.z) == t;
  const int loc_svc = lspd && svc && (svc_type == Q_DA || svc_type == Q_CLAIM) ? *gp(&C.loc[k1.y]) : -1;
  const int loc_core = dir_core ? *gp(&C.loc[k0.z]) : -1;
  const bool retry = VAR && k0.x == CORE_IDLE && hline >= 0;  // the op held back by the last miss
  const bool forced = k0.x == CORE_IDLE && !retry && k2.w >= 0;
  const bool drawn_idle = k0.x == CORE_IDLE && !retry && !forced && r.x < C.op_thr;
  // hit under miss (Sec. 3.5): a core with a miss outstanding still draws, unless the L1 is busy
  // with the fill or an op is already held
  const bool drawn_hum = VAR && (C.variants & SIM_FLAG_HIT_UNDER_MISS) && k0.x != CORE_IDLE && !fill && hline < 0 &&
                         r.x < C.op_thr;
  const bool drawn = drawn_idle || drawn_hum;
  // L2 set: a static home holds only its own lines (index line / N); an LSPD slice any line
  const uint32_t ixR = lspd ? (uint32_t)k1.y : div_n(C, (uint32_t)k1.y), ixL = lspd ? (uint32_t)k0.z : div_n(C, (uint32_t)k0.z);
  int* setR = C.l2 + ((size_t)t * C.s2 + (ixR & (uint32_t)(C.s2 - 1))) * C.w2;
  int* setL = C.l2 + ((size_t)t * C.s2 + (ixL & (uint32_t)(C.s2 - 1))) * C.w2;
  int vR[8], vL[8], u[8];
  if (svc && (svc_type == Q_RA || svc_type == Q_ARRIVED)) set_load(setR, C.w2, vR);
  if (local || slice_look || fill_mem) set_load(setL, C.w2, vL);
  // migration: the access histories of those two sets (the ways' order, C.mig words per way)
  const int mg = mig ? C.mig : 0;
  int* histR = mig ? C.l2h + (size_t)(setR - C.l2) * mg : nullptr;
  int* histL = mig ? C.l2h + (size_t)(setL - C.l2) * mg : nullptr;
  int4 nh = EMPTY, nm = EMPTY;  // nodes at the hit-queue and miss-queue heads: next, ready, line
  if (k1.z >= 0) nh = ld_node<MULTI>(&C.node[k1.z]);
  if (k2.x >= 0) nm = ld_node<MULTI>(&C.node[k2.x]);
  int line_op = k0.z;  // the line of the op that touches L1 this cycle (fill or issue)
  if (retry) line_op = hline;
  else if (forced) line_op = k2.w;
  else if (drawn)
    line_op = (C.private_lines > 0 && r.y >= C.shared_thr) ? C.shared_lines + t * C.private_lines + zipf_rank(C.zp, r.z)
                                                           : zipf_rank(C.zs, r.z);
  int* set1 = C.l1 + ((size_t)t * C.s1 + (line_op & (C.s1 - 1))) * C.w1;
  if (fill || retry || forced || drawn) set_load(set1, C.w1, u);

  // ---- phase one: home L2 service, then the core (Sec. 7.1, phase one; Sec. 3.5) ----------
  bool dirtyR = false, dirtyL = false, dirty1 = false, d4 = false, d5 = false;
  int node_tail = -1, node_rq = -1, node_ready = 0, node_line = 0, node_w = 0;
  // appends requester rq to this tile's hit queue (replies with the block) or miss queue (a
  // static home's memory misses; an LSPD slice's one-flit answers); its node is written below
  auto enqueue = [&](bool hitq, int rq, int ready, int word) {
    node_rq = rq;
    node_ready = ready;
    node_line = word;
    const int4 fresh = make_int4(-1, ready, word, 0);
    if (hitq) {
      if (k1.w >= 0) {
        node_tail = k1.w;
        if (k1.w == k1.z) nh.x = rq;
      } else {
        k1.z = rq;
        nh = fresh;
      }
      k1.w = rq;
    } else {
      if (k2.y >= 0) {
        node_tail = k2.y;
        if (k2.y == k2.x) nm.x = rq;
      } else {
        k2.x = rq;
        nm = fresh;
      }
      k2.y = rq;
    }
  };
  // LSPD directory entries of this tile: each write also moves the tile's checksum
  unsigned long long dsum_dir = (unsigned long long)(uint32_t)k4.z | ((unsigned long long)(uint32_t)k4.w << 32);
  int fwd_line = -1, fwd_val = 0;  // the entry written by the service, read again by the core
  auto dir_write = [&](int line, int old_owner, int owner) {
    if (old_owner >= 0) dsum_dir -= mix64(((unsigned long long)(uint32_t)line << 32) | (uint32_t)old_owner);
    if (owner >= 0) dsum_dir += mix64(((unsigned long long)(uint32_t)line << 32) | (uint32_t)owner);
    *gp(&C.loc[line]) = owner;
    fwd_line = line;
    fwd_val = owner;
    d4 = true;
  };
  if (svc && !lspd) {
    const int rq = k1.x, line = k1.y;
    const bool hit = set_touch(vR, C.w2, line, true, dirtyR);
    lds_add(L, hit ? SIM_ST_L2_HIT : SIM_ST_L2_MISS, 1);
    enqueue(hit, rq, (hit ? c : c + C.mem_lat) + inj_delay, line);
    k1.x = -1;
    k1.y = -1;
    d1 = true;
    d2 = true;
  } else if (svc) {  // LSPD (Sec. 3.2, Sec. 6.2.2): remote access, directory access, eviction notice
    const int who = svc_who, line = k1.y;
    if (svc_type == Q_RA) {
      const int i = way_of(vR, line);
      if (i >= 0) {
        lds_add(L, SIM_ST_L2_HIT, 1);
        int n = 0;
        if (mig) {  // Sec. 3.3: the block's list of its last accessors
          n = hist_note(histR, mg, i, who);
          hist_front(histR, mg, i);
        }
        way_front(vR, i);
        dirtyR = true;
        // a remote tile made most of the block's last accesses: the block moves there, unless it
        // has just moved here and this slice still waits for the directory to acknowledge its
        // claim, or another block of this slice is still on its way
        const bool claiming = k0.x == CORE_WAIT && k0.z == line;
        const bool sending = k5.z >= 0 && (k5.z & MIG_TRANSIT);
        if (mig && 2 * n > mg && !claiming && !sending) {
          k5.y = line;  // the block goes whole; this slice serves it until told of its arrival
          k5.z = who | MIG_TRANSIT;
          d5 = true;
          lds_add(L, SIM_ST_MIGRATE, 1);
          enqueue(true, who, c + inj_delay, line | MIG_MARK);
        } else {
          enqueue(true, who, c + inj_delay, line);
        }
      } else if (mig && k5.y == line) {  // Sec. 3.3: redirected to where the block went
        lds_add(L, SIM_ST_REDIRECT, 1);
        enqueue(false, who, c + inj_delay, k5.z & ~MIG_TRANSIT);
      } else {
        lds_add(L, SIM_ST_TRAP, 1);
        enqueue(false, who, c + inj_delay, CODE_TRAP);
      }
    } else if (svc_type == Q_ARRIVED) {  // Sec. 3.3: the block sent away has arrived: this copy goes
      if (k5.z == (who | MIG_TRANSIT)) {
        const int i = way_of(vR, line);
        if (i >= 0) {
          way_remove(vR, C.w2, i);
          if (mig) hist_remove(histR, mg, C.w2, i);
          dirtyR = true;
        }
        k5.z = who;
        d5 = true;
      }
    } else if (svc_type == Q_CLAIM) {  // the directory names the block's new owner and tells it
      dir_write(line, loc_svc, who);
      enqueue(false, who, c + inj_delay, CODE_ACK);
    } else if (svc_type == Q_DA) {
      lds_add(L, SIM_ST_DIR_ACCESS, 1);
      int code = loc_svc;
      if (loc_svc < 0) {  // not on chip: the asker will bring it from memory
        dir_write(line, -1, who);
        lds_add(L, SIM_ST_DIR_NACK, 1);
        code = CODE_NACK;
      }
      enqueue(false, who, c + inj_delay, code);
    } else {  // the entry names the evicting slice until its notice arrives
      dir_write(line, who, -1);
      lds_add(L, SIM_ST_DIR_EVICT, 1);
    }
    k1.x = -1;
    k1.y = -1;
    d1 = true;
    d2 = true;
  }
  // the core's slice access below sees the service's changes when both touch one set
  if (lspd && svc && (svc_type == Q_RA || svc_type == Q_ARRIVED) && (slice_look || fill_mem) && setL == setR) {
#pragma unroll
    for (int i = 0; i < 8; ++i) vL[i] = vR[i];
    dirtyL = dirtyL || dirtyR;
    dirtyR = false;
  }
  if (fill) {  // the block arrived: fill L1, the op completes
    bool claim = false;
    if (fill_mem) {  // LSPD: into the local slice too; an evicted block leaves the directory
      const int victim = way_insert(vL, C.w2, k0.z);
      if (mig) hist_insert(histL, mg, C.w2);  // its history starts empty
      dirtyL = true;
      if (victim >= 0 && mig && victim == k5.y && k5.z >= 0 && (k5.z & MIG_TRANSIT)) {
        // the block on its way elsewhere leaves this slice: its new owner's claim updates the
        // directory, and requests still reaching here are redirected
      } else if (victim >= 0) {
        GUARD_LINE(victim)
        if (dir_of(victim) == t) {
          dir_write(victim, t, -1);
          lds_add(L, SIM_ST_DIR_EVICT, 1);
        } else {
          k4.y = victim;
          d4 = true;
        }
      }
      if (fill_mig) {  // Sec. 3.3: the directory learns the new owner; the op completes when it has
        if (dir_of(k0.z) == t) {
          dir_write(k0.z, fwd_line == k0.z ? fwd_val : loc_core, t);
        } else {
          claim = true;
          k5.x = k0.z;
          d5 = true;
          k0.x = CORE_WAIT;
          d0 = true;
        }
      }
    }
    if (!claim) {
      set_touch(u, C.w1, line_op, true, dirty1);
      const unsigned long long lat = (unsigned long long)(c - k0.w);
      lds_add(L, SIM_ST_OPS_DONE, 1);
      lds_add(L, SIM_ST_OP_LAT, lat);
      atomicMax(&L.v[SIM_ST_OP_LAT_MAX], lat);
      k0.x = CORE_IDLE;
      d0 = true;
    }
  } else if (missed && lspd) {  // LSPD: own slice, then the directory (Sec. 3.2)
    const int i = way_of(vL, k0.z);
    if (!slice_look) {
      k0.y = c + 1;  // a pending eviction notice or claim goes out first
    } else if (i >= 0) {
      lds_add(L, SIM_ST_L2_HIT, 1);
      if (mig) {  // the local core's access
        hist_note(histL, mg, i, t);
        hist_front(histL, mg, i);
      }
      way_front(vL, i);
      dirtyL = true;
      k0.x = CORE_FILL;
      k0.y = c + 1;
    } else if (mig && k5.y == k0.z && k5.z >= 0 && (k5.z & MIG_TRANSIT)) {
      // this slice sent the block away and has since evicted its copy: the core waits for the
      // arrival notice before it asks for the block again (so that the notice cannot remove a
      // copy that came back to this slice)
      k0.y = c + 1;
    } else if (dir_core) {  // this tile keeps the entry: look it up at once
      lds_add(L, SIM_ST_DIR_ACCESS, 1);
      int o = fwd_line == k0.z ? fwd_val : loc_core;
      if (o == t && k5.y == k0.z) {  // this slice gave the block away; the new owner's claim
        o = k5.z & ~MIG_TRANSIT;     // is still on the way
        lds_add(L, SIM_ST_REDIRECT, 1);
      }
      if (o == t) {  // stale (an older migration): look again next cycle
        lds_add(L, SIM_ST_TRAP, 1);
        k0.y = c + 1;
      } else {
        lds_add(L, SIM_ST_L2_MISS, 1);
        if (o < 0) {
          dir_write(k0.z, -1, t);
          lds_add(L, SIM_ST_DIR_NACK, 1);
          k0.x = CORE_FILL_MEM;
          k0.y = c + C.mem_lat;
        } else {
          k0.x = CORE_SEND_RA;
          k4.x = o;
          d4 = true;
          k0.y = c + inj_delay;
          lds_add(L, SIM_ST_REQ_MADE, 1);
        }
      }
    } else {
      lds_add(L, SIM_ST_L2_MISS, 1);
      k0.x = CORE_SEND_DA;
      k0.y = c + inj_delay;
    }
    d0 = true;
  } else if (missed) {  // L1 miss penalty over: local home slice, or a request flit
    if (local) {
      if (svc && setL == setR) {
#pragma unroll
        for (int i = 0; i < 8; ++i) vL[i] = vR[i];
      }
      const bool hit = set_touch(vL, C.w2, k0.z, true, dirtyL);
      lds_add(L, hit ? SIM_ST_L2_HIT : SIM_ST_L2_MISS, 1);
      k0.x = CORE_FILL;
      k0.y = hit ? c + 1 : c + C.mem_lat;
    } else {
      k0.x = CORE_SEND;
      lds_add(L, SIM_ST_REQ_MADE, 1);
    }
    d0 = true;
  } else if (retry || forced || drawn_idle) {
    const int issued = retry ? hissue : c;  // a held op counts from its first issue
    if (retry) {
      hline = -1;
      hissue = 0;
      d3 = true;
    } else {
      lds_add(L, SIM_ST_OPS_ISSUED, 1);
    }
    if (forced) {
      k2.w = -1;
      d2 = true;
    }
    k0.z = line_op;
    k0.w = issued;
    d0 = true;
    if (set_touch(u, C.w1, line_op, false, dirty1)) {
      const unsigned long long lat = (unsigned long long)(c - issued);
      lds_add(L, SIM_ST_L1_HIT, 1);
      lds_add(L, SIM_ST_OPS_DONE, 1);
      if (retry) {
        lds_add(L, SIM_ST_OP_LAT, lat);
        atomicMax(&L.v[SIM_ST_OP_LAT_MAX], lat);
      }
    } else {
      lds_add(L, SIM_ST_L1_MISS, 1);
      k0.x = CORE_L1MISS;
      k0.y = c + C.l1_lat;
    }
  }
  if (drawn_hum) {  // a hit completes under the miss; a miss is held until the fill
    lds_add(L, SIM_ST_OPS_ISSUED, 1);
    if (set_touch(u, C.w1, line_op, false, dirty1)) {
      lds_add(L, SIM_ST_L1_HIT, 1);
      lds_add(L, SIM_ST_OPS_DONE, 1);
    } else {
      hline = line_op;
      hissue = c;
      d3 = true;
    }
  }

  // ---- phase two: injection into a free input, then oldest-first arbitration ----------------
  const int arrivals = (f0.x >= 0) + (f1.x >= 0) + (f2.x >= 0) + (f3.x >= 0);
  const int deg = (int)v0 + (int)v1 + (int)v2 + (int)v3;
  // (LSPD: the miss queue holds one-flit answers, and the core's own flit is a pending
  // eviction notice, a directory access or a remote-access request)
  const bool own = lspd ? (k4.y >= 0 || k5.w >= 0 || k5.x >= 0 || ((k0.x == CORE_SEND_DA || k0.x == CORE_SEND_RA) && k0.y <= c))
                        : (k0.x == CORE_SEND && k0.y + inj_delay <= c);
  int cls = -1;
  if (k2.x >= 0 && nm.y <= c) cls = 0;
  else if (k1.z >= 0 && nh.y <= c) cls = 1;
  else if (own) cls = 2;
  else if (fdst >= 0) cls = 3;
  else if (k2.z > 0) cls = 4;
  if (cls >= 0 && arrivals >= deg) {
    lds_add(L, SIM_ST_INJ_BLOCKED, 1);
    cls = -1;
  }
  int4 fi = EMPTY;
  if (cls >= 0) {
    fi.y = c;
    fi.z = t;
    if (cls == 0 && lspd) {  // directory answer or trap: one flit, control bit set
      fi.x = k2.x;
      fi.y = (int)((uint32_t)c | CTL_BIT);
      fi.w = (KIND_REPLY << 30) | (nm.z + CODE_BASE);
      k2.x = nm.x;
      if (nm.x < 0) k2.y = -1;
      acc.inj_reply++;
      d2 = true;
    } else if (cls == 2 && lspd) {
      if (k4.y >= 0) {  // eviction notice to the block's directory tile
        fi.x = dir_of(k4.y);
        fi.y = (int)((uint32_t)c | CTL_BIT);
        fi.w = (KIND_DIR << 30) | k4.y;
        k4.y = -1;
        d4 = true;
      } else if (k5.w >= 0) {  // Sec. 3.3: the migrated block has arrived; its source drops its copy
        fi.x = k5.w;
        fi.y = (int)((uint32_t)c | CTL_BIT);
        fi.w = KIND_REQ << 30;
        k5.w = -1;
        d5 = true;
      } else if (k5.x >= 0) {  // a migrated block's new owner, to its directory tile
        fi.x = dir_of(k5.x);
        fi.y = (int)((uint32_t)c | CTL_BIT);
        fi.w = (KIND_BG << 30) | k5.x;
        k5.x = -1;
        d5 = true;
      } else if (k0.x == CORE_SEND_DA) {  // directory access
        fi.x = dir_of(k0.z);
        fi.w = (KIND_DIR << 30) | k0.z;
        k0.x = CORE_WAIT;
        d0 = true;
      } else {  // remote access at the owner
        fi.x = k4.x;
        fi.w = (KIND_REQ << 30) | k0.z;
        k4.x = -1;
        d4 = true;
        k0.x = CORE_WAIT;
        d0 = true;
      }
      acc.inj_req++;
    } else if (cls <= 1) {  // a flit of the head's reply; the head is popped with the packet's last flit
      const int4 hd = pick4(cls == 0, nm, nh);
      const int rq = cls == 0 ? k2.x : k1.z;
      const int sent = hd.w + 1;
      // a migrating block (Sec. 3.3, Table 1) goes as MIG_FLITS answer flits
      const bool mig_pk = lspd && (hd.z & MIG_MARK);
      const int len = mig_pk ? MIG_FLITS : C.reply_flits;
      const bool last = sent >= len;
      if (last) {
        if (cls == 0) {
          k2.x = hd.x;
          if (hd.x < 0) k2.y = -1;
        } else {
          k1.z = hd.x;
          if (hd.x < 0) k1.w = -1;
        }
        if (!mig_pk) lds_add(L, SIM_ST_REPLY_SENT, 1);
      }
      // the sent count goes to the head's node; a node appended this cycle is written whole
      // below, so its count rides with that store
      if (len > 1) {
        if (rq == node_rq) node_w = last ? 0 : sent;
        else st_i<MULTI>(reinterpret_cast<int*>(&C.node[rq]) + 3, last ? 0 : sent);
      }
      fi.x = rq;
      fi.w = mig_pk ? (KIND_REPLY << 30) | (CODE_MIG + CODE_BASE) : (KIND_REPLY << 30) | hd.z;
      if (mig_pk) fi.y = (int)((uint32_t)c | CTL_BIT);
      acc.inj_reply++;
      d1 = true;
      d2 = true;
    } else if (cls == 2) {
      fi.x = (int)mod_n(C, (uint32_t)k0.z);
      fi.w = (KIND_REQ << 30) | k0.z;
      k0.x = CORE_WAIT;
      d0 = true;
      acc.inj_req++;
    } else {
      if (cls == 3) {
        fi.x = fdst;
        fdst = -1;
        d3 = true;
      } else {
        const uint4 r2 = philox((uint32_t)c, (uint32_t)t, 1u, 0u, C.key0, C.key1);
        int d = (int)__umulhi(r2.x, (uint32_t)(N - 1));
        fi.x = d + (d >= t);
        k2.z -= 1;
        d2 = true;
      }
      fi.w = (int)(KIND_BG << 30);
      acc.inj_bg++;
    }
  }

  // Oldest first (key: inject cycle, then source tile; empty slots sort last); with priority by
  // deflection count the count comes first, most deflected first (key 0xFFFF - count).  Only
  // (key, dst, index) tuples are sorted; the port of flit i is packed at bits 3i..3i+2 of
  // `ports` (7 = none) and each flit is stored straight into its neighbour's slot.
  // (without the count, qa is 0 for every slot: the empty ones still sort last on qh)
  uint32_t qa0 = !aged ? 0u : f0.x < 0 ? ~0u : AGE_MAX - a0, qa1 = !aged ? 0u : f1.x < 0 ? ~0u : AGE_MAX - a1;
  uint32_t qa2 = !aged ? 0u : f2.x < 0 ? ~0u : AGE_MAX - a2, qa3 = !aged ? 0u : f3.x < 0 ? ~0u : AGE_MAX - a3;
  uint32_t qa4 = !aged ? 0u : fi.x < 0 ? ~0u : (uint32_t)AGE_MAX;
  const uint32_t ym = lspd ? ~CTL_BIT : ~0u;  // the inject cycle without the LSPD control bit
  uint32_t qh0 = f0.x < 0 ? ~0u : (uint32_t)f0.y & ym, ql0 = f0.x < 0 ? ~0u : (uint32_t)f0.z;
  uint32_t qh1 = f1.x < 0 ? ~0u : (uint32_t)f1.y & ym, ql1 = f1.x < 0 ? ~0u : (uint32_t)f1.z;
  uint32_t qh2 = f2.x < 0 ? ~0u : (uint32_t)f2.y & ym, ql2 = f2.x < 0 ? ~0u : (uint32_t)f2.z;
  uint32_t qh3 = f3.x < 0 ? ~0u : (uint32_t)f3.y & ym, ql3 = f3.x < 0 ? ~0u : (uint32_t)f3.z;
  uint32_t qh4 = fi.x < 0 ? ~0u : (uint32_t)fi.y & ym, ql4 = fi.x < 0 ? ~0u : (uint32_t)fi.z;
  int sd0 = f0.x, sd1 = f1.x, sd2 = f2.x, sd3 = f3.x, sd4 = fi.x;
  int si0 = 0, si1 = 1, si2 = 2, si3 = 3, si4 = 4;
#define CSWAP(a, b)                                                                              \
  if (qa##b < qa##a || (qa##b == qa##a && (qh##b < qh##a || (qh##b == qh##a && ql##b < ql##a)))) { \
    uint32_t ta = qa##a; qa##a = qa##b; qa##b = ta;                                              \
    uint32_t th = qh##a; qh##a = qh##b; qh##b = th;                                              \
    uint32_t tl = ql##a; ql##a = ql##b; ql##b = tl;                                              \
    int td = sd##a; sd##a = sd##b; sd##b = td;                                                   \
    int ti = si##a; si##a = si##b; si##b = ti;                                                   \
  }
  CSWAP(0, 1) CSWAP(3, 4) CSWAP(2, 4) CSWAP(2, 3) CSWAP(1, 4) CSWAP(0, 3) CSWAP(0, 2) CSWAP(1, 3) CSWAP(1, 2)
#undef CSWAP

  const unsigned valid = (v0 ? 1u : 0u) | (v1 ? 2u : 0u) | (v2 ? 4u : 0u) | (v3 ? 8u : 0u);
  unsigned used = 0, dm = 0;  // dm: bit i set when flit i is deflected
  uint32_t ports = 0x7FFFu;
  auto assign = [&](int dst, int idx) {
    if (dst < 0) return;
    unsigned port;
    if (dst == t && !(used & 16u)) {
      port = 4;
    } else {
      const int drow = C.W > 1 ? (int)__umulhi((uint32_t)dst, C.w_magic) : dst;
      const int dx = (dst - drow * C.W) - x, dy = drow - y;
      const int px = dx > 0 ? 2 : (dx < 0 ? 3 : -1);
      const int py = dy > 0 ? 1 : (dy < 0 ? 0 : -1);
      if (px >= 0 && !(used & (1u << px))) port = (unsigned)px;
      else if (py >= 0 && !(used & (1u << py))) port = (unsigned)py;
      else {
        port = (unsigned)__builtin_ctz(valid & ~used & 15u);
        acc.defl++;
        dm |= 1u << idx;
      }
      acc.trav++;
    }
    used |= 1u << port;
    ports = (ports & ~(7u << (3 * idx))) | (port << (3 * idx));
  };
  assign(sd0, si0);
  assign(sd1, si1);
  assign(sd2, si2);
  assign(sd3, si3);
  assign(sd4, si4);
  if (C.watch_age > 0) {  // watchdog (debug mode): every live flit leaves by exactly one port,
    const int nlive = (f0.x >= 0) + (f1.x >= 0) + (f2.x >= 0) + (f3.x >= 0) + (fi.x >= 0);
    uint32_t oldest = 0;  // and none is older than the bound (the oldest flit always advances)
    if (f0.x >= 0) oldest = max(oldest, (uint32_t)c - ((uint32_t)f0.y & ym));
    if (f1.x >= 0) oldest = max(oldest, (uint32_t)c - ((uint32_t)f1.y & ym));
    if (f2.x >= 0) oldest = max(oldest, (uint32_t)c - ((uint32_t)f2.y & ym));
    if (f3.x >= 0) oldest = max(oldest, (uint32_t)c - ((uint32_t)f3.y & ym));
    if (__builtin_popcount(used) != nlive) {
      st_coh(C.err, ERR_ROUTER);
      return false;
    }
    if (oldest > (uint32_t)C.watch_age) {
      st_coh(C.err, ERR_WATCHDOG);
      return false;
    }
  }

  // ---- phase three: stores (caches, queue nodes, slots, core words) -------------------------
  if (pipe_now) {  // this cycle's arrivals enter the pipeline
    if (v0) gstore4(pipe_now, a0w);
    if (v1) gstore4(pipe_now + N, a1w);
    if (v2) gstore4(pipe_now + 2 * N, a2w);
    if (v3) gstore4(pipe_now + 3 * N, a3w);
  }
  if (dirtyR) set_store(setR, C.w2, vR);
  if (dirtyL) set_store(setL, C.w2, vL);
  if (dirty1) set_store(set1, C.w1, u);
  if (node_rq >= 0) {
    st_node<MULTI>(&C.node[node_rq], make_int4(-1, node_ready, node_line, node_w));
    if (node_tail >= 0) st_i<MULTI>(reinterpret_cast<int*>(&C.node[node_tail]), node_rq);
  }
  int4 oe = EMPTY;
  const uint32_t ns = (uint32_t)(c + 1);
  // a flit's deflection count after this cycle (Sec. 6.2.1: one more when deflected here)
  auto age_out = [&](uint32_t a, int i) -> uint32_t {
    if (!aged) return 0u;
    const uint32_t n = a + ((dm >> i) & 1u);
    if (n > (uint32_t)AGE_MAX) {
      st_coh(C.err, 4);  // a flit deflected 65,536 times: reported as an invariant failure
      return (uint32_t)AGE_MAX;
    }
    return n;
  };
  auto send = [&](const int4& f, unsigned port, uint32_t age) {
    if (port == 4) { oe = f; return; }
    if (port > 3) return;
    const int nbr = port == 0 ? t - C.W : port == 1 ? t + C.W : port == 2 ? t + 1 : t - 1;
    const int slot = (int)(port ^ 1u);
    const bool cx = MULTI && (port == 0 ? cross[0] : port == 1 ? cross[1] : port == 2 ? cross[2] : cross[3]);
    st_slot(&C.link[(nxt * 4 + slot) * N + nbr], slot_encode_aged(f, ns, age), cx);
  };
  send(f0, ports & 7u, age_out(a0, 0));
  send(f1, (ports >> 3) & 7u, age_out(a1, 1));
  send(f2, (ports >> 6) & 7u, age_out(a2, 2));
  send(f3, (ports >> 9) & 7u, age_out(a3, 3));
  send(fi, (ports >> 12) & 7u, age_out(0u, 4));
  const unsigned idle = valid & ~used;  // links that carry nothing next cycle
  const int4 E = slot_encode(EMPTY, ns);
  if (idle & 1u) st_slot(&C.link[(nxt * 4 + 1) * N + t - C.W], E, MULTI && cross[0]);
  if (idle & 2u) st_slot(&C.link[(nxt * 4 + 0) * N + t + C.W], E, MULTI && cross[1]);
  if (idle & 4u) st_slot(&C.link[(nxt * 4 + 3) * N + t + 1], E, MULTI && cross[2]);
  if (idle & 8u) st_slot(&C.link[(nxt * 4 + 2) * N + t - 1], E, MULTI && cross[3]);

  if (oe.x >= 0) {
    const int kind = (int)((uint32_t)oe.w >> 30);
    const bool ctl = lspd && ((uint32_t)oe.y & CTL_BIT);
    const int lat = c - (int)((uint32_t)oe.y & ym);
    const unsigned long long ulat = (unsigned long long)lat;
    // directory messages and ownership claims count as requests
    const bool as_req = kind == KIND_REQ || kind == KIND_DIR || (kind == KIND_BG && ctl);
    const bool as_bg = kind == KIND_BG && !ctl;
    acc.ej_req += as_req;
    acc.ej_reply += kind == KIND_REPLY;
    acc.ej_bg += as_bg;
    acc.lat_req += as_req ? ulat : 0ull;
    acc.lat_reply += kind == KIND_REPLY ? ulat : 0ull;
    acc.lat_bg += as_bg ? ulat : 0ull;
    atomicMax(&L.v[SIM_ST_LAT_MAX], (unsigned long long)lat);
    lds_add(L, SIM_ST_HIST + min(15, 31 - __builtin_clz((unsigned)max(lat, 1))), 1);
    if (kind == KIND_REQ && ctl) {  // migration: the block this slice sent has arrived
      k1.x = oe.z | (Q_ARRIVED << 24);
      k1.y = k5.y;  // the block it sent (one at a time)
      d1 = true;
    } else if (kind == KIND_REQ) {
      lds_add(L, SIM_ST_REQ_RECV, 1);
      k1.x = oe.z;
      k1.y = oe.w & LINE_MASK;
      d1 = true;
    } else if (kind == KIND_DIR) {  // LSPD: directory access or (control bit) eviction notice
      k1.x = oe.z | ((ctl ? Q_EV : Q_DA) << 24);
      k1.y = oe.w & LINE_MASK;
      d1 = true;
    } else if (kind == KIND_BG && ctl) {  // migration: the new owner's claim
      k1.x = oe.z | (Q_CLAIM << 24);
      k1.y = oe.w & LINE_MASK;
      d1 = true;
    } else if (kind == KIND_REPLY && ctl) {  // LSPD: the directory's answer, a trap, a redirection
      const int code = (oe.w & LINE_MASK) - CODE_BASE;
      if (code == CODE_MIG) {  // a flit of the block migrating here; the last one fills it in
        rcv += 1;
        d3 = true;
        if (rcv >= MIG_FLITS) {  // the whole block is in; its source is told (Sec. 3.3)
          rcv = 0;
          k5.w = oe.z;
          d5 = true;
          k0.x = CORE_FILL_MIG;
          k0.y = c + 1;
        }
      } else if (code == CODE_ACK) {  // the directory names this slice: L1 fill, op complete
        k0.x = CORE_FILL;
        k0.y = c + 1;
      } else if (code == CODE_NACK) {  // not on chip: from memory into the local slice
        k0.x = CORE_FILL_MEM;
        k0.y = c + C.mem_lat;
      } else if (code == CODE_TRAP || code == t) {  // stale entry: ask the directory again
        if (code == t) lds_add(L, SIM_ST_TRAP, 1);
        k0.x = CORE_SEND_DA;
        k0.y = c + 1;
      } else {
        k0.x = CORE_SEND_RA;
        k0.y = c + 1;
        k4.x = code;
        d4 = true;
        lds_add(L, SIM_ST_REQ_MADE, 1);
      }
      d0 = true;
    } else if (kind == KIND_REPLY) {  // a flit of the block; the last one completes it
      rcv += 1;
      d3 = true;
      if (rcv >= C.reply_flits) {
        rcv = 0;
        lds_add(L, SIM_ST_REPLY_RECV, 1);
        k0.x = CORE_FILL;
        k0.y = c + 1;
        d0 = true;
      }
    }
  }
  if (N > 1 && r.w < C.bg_thr) {
    k2.z += 1;
    d2 = true;
    lds_add(L, SIM_ST_BG_GEN, 1);
  }
  if (d0) gstore4(&C.core[t], k0);
  if (d1) gstore4(&C.core[N + t], k1);
  if (d2) gstore4(&C.core[2 * N + t], k2);
  if (d3) gstore4(&C.core[3 * N + t], make_int4(fdst, rcv, hline, hissue));
  if (d4) {
    k4.z = (int)(uint32_t)dsum_dir;
    k4.w = (int)(uint32_t)(dsum_dir >> 32);
    gstore4(&C.core[4 * N + t], k4);
  }
  if (d5) gstore4(&C.core[5 * N + t], k5);
#undef GUARD
#undef GUARD_LINE
  return true;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds a workgroup's counters to the chip's statistics (once per launch).
__device__ __forceinline__ void flush_counters(const Acc& acc, LdsStats& L, const ChipDev& C, int patch, int c0, int c_done) {
  {
    int v[8] = {acc.trav, acc.defl, acc.inj_req, acc.inj_reply, acc.inj_bg, acc.ej_req, acc.ej_reply, acc.ej_bg};
    const int idx[8] = {SIM_ST_TRAVERSALS, SIM_ST_DEFLECTIONS, SIM_ST_INJ_REQ, SIM_ST_INJ_REPLY, SIM_ST_INJ_BG,
                        SIM_ST_EJ_REQ, SIM_ST_EJ_REPLY, SIM_ST_EJ_BG};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int s = wave_sum_i(v[i]);
      if ((threadIdx.x & 63) == 0 && s) atomicAdd(&L.v[idx[i]], (unsigned long long)s);
    }
    const unsigned long long lat[4] = {acc.lat_req, acc.lat_reply, acc.lat_bg, acc.op_lat};
    const int lidx[4] = {SIM_ST_LAT_REQ, SIM_ST_LAT_REPLY, SIM_ST_LAT_BG, SIM_ST_OP_LAT};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned long long s = wave_sum(lat[k]);
      if ((threadIdx.x & 63) == 0 && s) atomicAdd(&L.v[lidx[k]], s);
    }
    int w[12] = {acc.l2_hit, acc.l2_miss, acc.ops_done, acc.ops_issued, acc.l1_hit, acc.l1_miss, acc.req_made,
                 acc.inj_blocked, acc.reply_sent, acc.req_recv, acc.reply_recv, acc.bg_gen};
    const int widx[12] = {SIM_ST_L2_HIT, SIM_ST_L2_MISS, SIM_ST_OPS_DONE, SIM_ST_OPS_ISSUED, SIM_ST_L1_HIT,
                          SIM_ST_L1_MISS, SIM_ST_REQ_MADE, SIM_ST_INJ_BLOCKED, SIM_ST_REPLY_SENT, SIM_ST_REQ_RECV,
                          SIM_ST_REPLY_RECV, SIM_ST_BG_GEN};
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const int s = wave_sum_i(w[i]);
      if ((threadIdx.x & 63) == 0 && s) atomicAdd(&L.v[widx[i]], (unsigned long long)s);
    }
    if (acc.lat_max) atomicMax(&L.v[SIM_ST_LAT_MAX], (unsigned long long)acc.lat_max);
    if (acc.op_lat_max) atomicMax(&L.v[SIM_ST_OP_LAT_MAX], (unsigned long long)acc.op_lat_max);
  }
  __syncthreads();
  if (patch == 0 && threadIdx.x == 0 && c_done > c0) L.v[SIM_ST_CYCLES] += (unsigned long long)(c_done - c0);
  __syncthreads();
  for (int i = threadIdx.x; i < NSTAT; i += blockDim.x) {
    if (!L.v[i]) continue;
    if (i == SIM_ST_LAT_MAX || i == SIM_ST_OP_LAT_MAX) atomicMax(&C.stats[i], L.v[i]);
    else atomicAdd(&C.stats[i], L.v[i]);
  }
}

// ---- the persistent step kernel ----------------------------------------------------------------
// Workgroup w runs patch table[w].patch of chip table[w].chip from the cycle its flag records
// up to min(flag + chunk, stop): one barrier per cycle inside the patch; patch edges are
// synchronised through the stamped slots.  digests (optional, single chip): digests[c -
// digest_base] += this patch's share of the digest of cycle c.
template <bool MULTI, int VAR>
__global__ void __launch_bounds__(256) step_kernel(const LaunchEntry* __restrict__ table, int chunk,
                                                   unsigned long long* digests, int digest_base) {
  __shared__ LdsStats L;
  __shared__ int s_fail;
  const LaunchEntry e = table[blockIdx.x];
  const ChipDev C = *e.chip;
  const int patch = e.patch;
  const int pxi = patch % C.pgx, pyi = patch / C.pgx;
  const int x0 = pxi * C.pw, y0 = pyi * C.ph;
  const int cols = min(C.pw, C.W - x0), rows = min(C.ph, C.H - y0);
  const int ntiles = cols * rows;
  for (int i = threadIdx.x; i < NSTAT; i += blockDim.x) L.v[i] = 0;
  if (threadIdx.x == 0) s_fail = 0;
  Acc acc = {};
  const int c0 = ld_coh(&C.flags[patch * FLAG_STRIDE]);
  const int c_end = max(c0, min(min(c0 + chunk, e.stop >= 0 ? e.stop : C.stop), patch == C.halt_patch ? C.halt_cycle : INT_MAX));
  int c_done = c0;
  __syncthreads();

  for (int c = c0; c <= c_end; ++c) {
    const bool step = c < c_end;
    const bool dig = digests != nullptr && c > c0;
    if (!step && !dig) break;
    unsigned long long h = 0;
    bool ok = true;
    for (int j = threadIdx.x; j < ntiles; j += blockDim.x) {
      const int lx = j % cols, ly = j / cols, x = x0 + lx, y = y0 + ly;
      const bool cross[4] = {ly == 0 && y > 0, ly == rows - 1 && y < C.H - 1, lx == cols - 1 && x < C.W - 1,
                             lx == 0 && x > 0};
      ok = ok && tile_step<MULTI, VAR>(C, y * C.W + x, x, y, c, cross, step, dig, h, acc, L);
    }
    if (dig) {
      h = wave_sum(h);
      if ((threadIdx.x & 63) == 0) atomicAdd(&digests[c - 1 - digest_base], h);
    }
    if (!ok) s_fail = 1;
    // Every store of cycle c completes before the barrier: interior slots are read by other
    // waves of this workgroup in cycle c+1, and a queue node written in cycle c must be
    // performed before its next writer (another home, reached only through at least three
    // more cycles of flit traffic) can touch it.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (s_fail) break;
    if (step) c_done = c + 1;
  }
  if (threadIdx.x == 0) st_coh(&C.flags[patch * FLAG_STRIDE], c_done);

  flush_counters(acc, L, C, patch, c0, c_done);
}

// ---- the one-tile-per-thread step kernel --------------------------------------------------------
// Used when a patch has no more tiles than its workgroup has threads (the mapping of large chips
// and of small chips in a batch).  Same model and same results as step_kernel; organised for a
// short cycle:
//  - a thread owns one tile for the whole launch; the tile's core words stay in registers;
//  - link slots between two tiles of the patch live in LDS; only patch-edge slots go through
//    global memory (stamped, polled), and the per-cycle barrier waits on LDS only;
//  - in cycle c-1 the thread issues cycle c's loads that do not depend on link inputs (L2 sets
//    of a home lookup and of a local miss, the op's L1 set, queue-head nodes); the random words
//    of a cycle and their Zipf table words are drawn one cycle before that, so the op's line
//    is known when its L1 set is loaded;
//  - a cycle issues its first read of the patch-edge slots, then runs phase one (which reads no
//    link input) while those reads are in flight, then polls; the patch-edge outputs go out
//    right after arbitration, before the rest of the cycle's stores;
//  - every thread drains its global stores (s_waitcnt vmcnt(0)) once per cycle, after issuing
//    that cycle's loads: a queue node stored in cycle c is therefore performed before the home
//    finishes cycle c+1, while its next writer is at least three cycles of flit traffic away.
constexpr int FAST_MAX = 256;

// Productive ports of a flit with destination d at the tile (x, y), as five bits in the order the
// assignment tries them: bit 0 the eject port (d is the tile itself), bit 1 east and bit 2 west
// (the X port), bit 3 north and bit 4 south (the Y port).  The destination's row is d / W by
// the reciprocal (wm = ceil(2^32 / W)); with W = 1, wm = 0 and wsel = ~0 make the row d itself.
// The offsets' signs plus one (0, 1, 2), clamped in one instruction each, index a table of
// nine 5-bit entries; the caller passes x - 1 and y - 1 (xm1, ym1) so that the +1 is free.
__device__ __forceinline__ uint32_t clamp02(int v) {  // max(0, min(v, 2)) in one instruction
  int r;
  asm("v_med3_i32 %0, %1, 0, 2" : "=v"(r) : "v"(v));
  return (uint32_t)r;
}
constexpr unsigned long long PROD_TABLE =  // entry 3 (sign x + 1) + (sign y + 1), 5 bits each
    (12ull << 0) | (4ull << 5) | (20ull << 10) |   // west: with north, alone, with south
    (8ull << 15) | (1ull << 20) | (16ull << 25) |  // north, eject, south
    (10ull << 30) | (2ull << 35) | (18ull << 40);  // east: with north, alone, with south
__device__ __forceinline__ uint32_t prod_mask(int d, int xm1, int ym1, int negW, uint32_t wm, uint32_t wsel) {
  const int drow = (int)(__umulhi((uint32_t)d, wm) | ((uint32_t)d & wsel));
  const uint32_t ux = clamp02(d - xm1 + __mul24(drow, negW)), uy = clamp02(drow - ym1);
  return (uint32_t)(PROD_TABLE >> (__umul24(ux, 15u) + __umul24(uy, 5u))) & 31u;
}

// One step of the oldest-first assignment, for the flit with sort key q (prod_mask at bits 3-7,
// input index i as i ^ 7 at bits 0-2; all ones when empty): the eject port if it is destined
// here and the port is free, else its X-productive port, else its Y-productive port, if free,
// else the lowest free valid port (a deflection; a destined flit that lost the eject port is
// deflected too).  `taken` holds the ports in two orders at once: bits 0-4 as prod_mask orders
// them, bits 5-8 north, south, east, west (the deflection order; ports off the mesh start out
// taken), so the lowest free bit of (mask | 5-8) is the flit's port.  The flit's input index is
// recorded in the port's 3-bit field of `inv` (port 4 = eject), which starts as all 7s (none).
// ndefl counts deflections; with DEFL_MASK the deflected flits' input indices are marked in dm.
constexpr uint32_t CODE_PORT = 4u | (2u << 3) | (3u << 6) | (0u << 9) | (1u << 12) |  // port of
                               (0u << 15) | (1u << 18) | (2u << 21) | (3u << 24) | (7u << 27);  // each bit
constexpr unsigned long long CODE_TWIN =  // the port's bit in the other order, 4 bits per code
    (0ull << 0) | (7ull << 4) | (8ull << 8) | (5ull << 12) | (6ull << 16) | (3ull << 20) | (4ull << 24) |
    (1ull << 28) | (2ull << 32) | (9ull << 36);
template <bool DEFL_MASK>
__device__ __forceinline__ void arb_assign_mask(unsigned long long q, uint32_t& taken, uint32_t& inv, unsigned& dm,
                                                int& ndefl) {
  const uint32_t lo = (uint32_t)q;
  // all ones for a live flit (inject cycles stay below 2^31), zero for an empty one
  const uint32_t lm = ~(uint32_t)((int)(q >> 32) >> 31);
  // (a free port always exists for a live flit: it has at most deg - 1 rivals.  An empty one
  // finds only bit 9, code 9, whose port field (7) and twin bit (9) nothing reads.)
  const uint32_t code = (uint32_t)__builtin_ctz(((((lo >> 3) & 31u) | 0x1E0u) & ~taken & lm) | 0x200u);
  const uint32_t port = (CODE_PORT >> (3u * code)) & 7u;
  const uint32_t twin = (uint32_t)(CODE_TWIN >> (4u * code)) & 15u;
  taken |= (1u << code) | (1u << twin);
  inv ^= (lo & 7u) << (3u * port);
  const bool defl = code - 5u < 4u;
  ndefl += defl ? 1 : 0;
  if (DEFL_MASK) dm |= defl ? (1u << ((lo & 7u) ^ 7u)) : 0u;
}

constexpr uint32_t PF_SVC = 1, PF_LOCAL = 2, PF_FILL = 4, PF_FORCED = 8, PF_DRAWN = 16;
constexpr uint32_t PF_RETRY = 32, PF_HUM = 64;  // hit under miss: the held op again; an op drawn under a miss
// LSPD: a block from memory goes into the own slice; the own slice is looked up after an L1 miss;
// this tile keeps that line's directory entry; a line read from state was out of range
constexpr uint32_t PF_FILLMEM = 128, PF_SLICE = 256, PF_DIRCORE = 512, PF_BAD = 1024;

struct Prefetch {            // loads of one cycle issued ahead of it
  uint4 r;                   // the tile's random words of the cycle
  uint4 r1;                  // ... and of the cycle after it, with its Zipf table words:
  uint32_t z_lo, z_hi;       // the op line a draw in that cycle would take is known a cycle early,
  uint32_t flags;            // PF_*: which of the cycle's memory steps happen (bits, not lane masks)
  int line_op;               // the op's line (fill or issue)
  int* set1;                 // its L1 set
  int* setR;
  int* setL;
  int u[8], vR[8], vL[8];    // L1 set of the op; L2 sets of the served request and of a local miss
  int4 nh, nm;               // hit-queue and miss-queue head nodes
  int loc_svc, loc_core;     // LSPD: the directory entries of a served directory access and of
                             // the core's own line when this tile keeps it (-1 otherwise)
};

// Random words of cycle c and the Zipf table words their op draw would use (issued, not waited).
__device__ __forceinline__ void draw_ahead(const ChipDev& C, int t, int c, Prefetch& P) {
  P.r1 = philox((uint32_t)c, (uint32_t)t, 0u, 0u, C.key0, C.key1);
  const bool priv = C.private_lines > 0 && P.r1.y >= C.shared_thr;
  const uint32_t* q = priv ? C.zp : C.zs;
  const uint32_t b = P.r1.z >> 16;
  P.z_lo = *gp(q + b);
  P.z_hi = *gp(q + b + 1);
}

// Issues every load of cycle c that does not depend on its link inputs.  The random words of c
// and their Zipf words were drawn one cycle earlier (draw_ahead); this draws those of c+1.
// VARS: `hline` is the op held by hit under miss (-1 for none), `hum` whether the chip has it.
template <bool MULTI, bool VARS, bool W48, bool LSPDB = false, bool MIGB = false>
__device__ __forceinline__ void prefetch(const ChipDev& C, int t, int c, const int4& k0, const int4& k1, const int4& k2,
                                         int hline, bool hum, int* l1_base, int* l2_base, Prefetch& P,
                                         const int4& k4 = make_int4(-1, -1, 0, 0),
                                         const int4& k5 = make_int4(-1, -1, -1, -1)) {
  const int N = C.N;
  // way counts, fixed at compile time for 4-way L1 and 8-way L2 slices (W48)
  const int w1 = W48 ? 4 : C.w1, w2 = W48 ? 8 : C.w2, w1s = W48 ? 2 : C.w1_shift, w2s = W48 ? 3 : C.w2_shift;
  P.r = P.r1;
  const bool lspd = LSPDB && C.lspd != 0;
  const bool svc = k1.x >= 0;
  const bool wake = k0.y == c;
  // LSPD (Sec. 3.2): a block from memory, or one that migrated here (Sec. 3.3), goes into the
  // own slice as it fills L1
  const bool fill_mig = MIGB && lspd && k0.x == CORE_FILL_MIG && wake;
  const bool fill_mem = (lspd && k0.x == CORE_FILL_MEM && wake) || fill_mig;
  const bool fill = (k0.x == CORE_FILL && wake) || fill_mem;
  const bool missed = k0.x == CORE_L1MISS && wake;
  const bool local = !lspd && missed && mod_n(C, (uint32_t)k0.z) == (uint32_t)t;
  // LSPD: the served message's kind, the own slice look-up (not while an eviction notice or a
  // claim is pending) and the directory entries read this cycle; a line read from state is
  // checked before it addresses the location array
  const int svc_type = lspd ? (k1.x >> 24) : Q_RA;
  const bool slice_look = lspd && missed && k4.y < 0 && (!MIGB || k5.x < 0);
  const bool bad = lspd && ((svc && (unsigned)k1.y >= (unsigned)C.lines) ||
                            ((slice_look || fill_mem) && (unsigned)k0.z >= (unsigned)C.lines));
  const int dir_of_op = C.lspd == 2 ? C.dir_center : (int)mod_n(C, (uint32_t)k0.z);
  const bool dir_core = (slice_look || fill_mig) && !bad && dir_of_op == t;
  P.loc_svc = lspd && svc && (svc_type == Q_DA || (MIGB && svc_type == Q_CLAIM)) && !bad ? *gp(&C.loc[k1.y]) : -1;
  P.loc_core = dir_core ? *gp(&C.loc[k0.z]) : -1;
  const bool retry = VARS && k0.x == CORE_IDLE && hline >= 0;
  const bool forced = k0.x == CORE_IDLE && !retry && k2.w >= 0;
  const bool drawn = k0.x == CORE_IDLE && !retry && !forced && P.r.x < C.op_thr;
  // hit under miss (Sec. 3.5): a core with a miss outstanding still draws, unless the L1 is busy
  // with the fill or an op is already held
  const bool drawn_hum = VARS && hum && k0.x != CORE_IDLE && !fill && hline < 0 && P.r.x < C.op_thr;
  P.flags = (svc ? PF_SVC : 0u) | (local ? PF_LOCAL : 0u) | (fill ? PF_FILL : 0u) | (forced ? PF_FORCED : 0u) |
            (drawn ? PF_DRAWN : 0u) | (retry ? PF_RETRY : 0u) | (drawn_hum ? PF_HUM : 0u);
  if (LSPDB)
    P.flags |= (fill_mem ? PF_FILLMEM : 0u) | (slice_look ? PF_SLICE : 0u) | (dir_core ? PF_DIRCORE : 0u) | (bad ? PF_BAD : 0u);
  // L2 set: a static home holds only its own lines (index line / N); an LSPD slice any line
  const uint32_t ixR = lspd ? (uint32_t)k1.y : div_n(C, (uint32_t)k1.y), ixL = lspd ? (uint32_t)k0.z : div_n(C, (uint32_t)k0.z);
  P.setR = l2_base + ((ixR & (uint32_t)(C.s2 - 1)) << w2s);
  P.setL = l2_base + ((ixL & (uint32_t)(C.s2 - 1)) << w2s);
  if (svc && (svc_type == Q_RA || (MIGB && svc_type == Q_ARRIVED))) set_load(P.setR, w2, P.vR);
  if (local || ((slice_look || fill_mem) && !bad)) set_load(P.setL, w2, P.vL);
  P.nh = make_int4(-1, -1, -1, -1);
  P.nm = make_int4(-1, -1, -1, -1);
  if ((unsigned)k1.z < (unsigned)N) P.nh = ld_node<MULTI>(&C.node[k1.z]);
  if ((unsigned)k2.x < (unsigned)N) P.nm = ld_node<MULTI>(&C.node[k2.x]);
  // a drawn op: Zipf rank from the table bucket of the high half of r.z, linear inside the
  // bucket by the low half; private lines follow the shared ones, private_lines per tile
  const bool priv = C.private_lines > 0 && P.r.y >= C.shared_thr;
  const int rank = (int)(P.z_lo + (uint32_t)(((unsigned long long)(P.r.z & 0xFFFFu) * (P.z_hi - P.z_lo)) >> 16));
  const int drawn_line = (priv ? C.shared_lines + t * C.private_lines : 0) + rank;
  P.line_op = retry ? hline : forced ? k2.w : ((drawn || drawn_hum) ? drawn_line : k0.z);
  P.set1 = l1_base + ((P.line_op & (C.s1 - 1)) << w1s);
  if (fill || retry || forced || drawn || drawn_hum) set_load(P.set1, w1, P.u);
  draw_ahead(C, t, c + 1, P);
}

// OPT bit 0 (FAST_PACKETS): replies may have several flits (the chip's reply_flits); without it
// the kernel is the single-flit model, compiled without the per-flit counts.  OPT bit 1
// (FAST_VARIANTS): the chip may have any of three variants, each read from the chip at run
// time: priority by deflection count (Sec. 4.2, Sec. 6.2.1; the flit rows then keep the count
// in bits 20-27 of their dst and src words, as the link slots do), hit under miss (Sec. 3.5;
// the held op rides in two more registers) and the injection register (a flit made in a
// cycle enters the network from the next one on, Sec. 6.2.1).  Without the bit they are
// compiled out.  OPT bit 2 (FAST_PIPE): the chip may have a router delay D > 1 (arrivals wait
// D-1 cycles in a per-tile pipeline in HBM before they are arbitrated).
// OPT bit 3 (FAST_WAYS48): every chip of the launch has 4-way L1 and 8-way L2 slices, so the set
// code is compiled for those way counts instead of reading them from the chip.
// OPT bit 4 (FAST_LSPD): the chip may have the LSPD directory (Sec. 3.2, Sec. 6.2.2).  Without
// migration it has two builds: for single-flit chips without variants or router delay and with
// 4/8-way caches (bit 3 alone beside it), and with bits 0-2 on and the way counts read at run time.
// OPT bit 5 (FAST_MIG): the directory with migration (Sec. 3.3), in the same two builds (bit 3
// alone beside bits 4-5, or bits 0-2 on).
// OPT bit 6 (FAST_NARROW): workgroups of at most 128 threads, with the LDS rows sized for them,
// so that four workgroups of two waves share a compute unit (base model only).
constexpr int FAST_PACKETS = 1, FAST_VARIANTS = 2, FAST_PIPE = 4, FAST_WAYS48 = 8, FAST_LSPD = 16, FAST_MIG = 32;
constexpr int FAST_NARROW = 64;
// The chip descriptor read through the constant address space from a pointer made uniform: the
// descriptor does not change while a launch runs.
__device__ __forceinline__ ChipDev desc_const(const ChipDev* p) {
  const unsigned long long u = (unsigned long long)(uintptr_t)p;
  const unsigned long long s = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
  static_assert(sizeof(ChipDev) % 4 == 0, "descriptor copied in 4-byte words");
  union Words { ChipDev d; uint32_t w[sizeof(ChipDev) / 4]; } out;
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)(uintptr_t)s;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ChipDev) / 4); ++i) out.w[i] = src[i];
  return out.d;
}
template <bool MULTI, bool DIGEST, int OPT>
__global__ void __launch_bounds__(FAST_MAX) step_fast(const LaunchEntry* __restrict__ table, int chunk,
                                                      unsigned long long* digests, int digest_base) {
  constexpr bool PACKETS = (OPT & FAST_PACKETS) != 0;
  constexpr bool VARS = (OPT & FAST_VARIANTS) != 0;
  constexpr bool PIPE = (OPT & FAST_PIPE) != 0;
  constexpr bool W48 = (OPT & FAST_WAYS48) != 0;
  constexpr bool LSPDB = (OPT & FAST_LSPD) != 0;
  constexpr bool MIGB = LSPDB && (OPT & FAST_MIG) != 0;
  constexpr int LW = (OPT & FAST_NARROW) ? 128 : FAST_MAX;  // threads the LDS rows are sized for
  __shared__ LdsStats L;
  __shared__ int s_fail;
  // [parity][row][local tile]: rows 0-3 are the input slots of ports 0-3 (written by the
  // neighbour inside the patch, or by the tile itself from a patch-edge slot), row 4 the flit
  // the tile injects, row 5 an empty flit; each output port copies the row of the flit it carries
  __shared__ int4 s_link[2][6][LW];
  const LaunchEntry e = table[blockIdx.x];
  // the checking build reads the chip descriptor as constant memory (scalar loads: the compiler
  // then keeps its fields out of vector registers, which lets two waves share a SIMD; the timed
  // build keeps the vector copy, whose arithmetic issues faster at one wave per SIMD)
  auto load_desc = [&]() -> ChipDev {
    if constexpr (DIGEST) return desc_const(e.chip);
    else return *e.chip;
  };
  const ChipDev C = load_desc();
  const int N = C.N;
  const int idl = VARS ? C.inj_delay : 0;  // 1: a reply or request made in cycle c enters from c+1
  const bool aged = VARS && (C.variants & SIM_FLAG_AGE_DEFLECT) != 0;  // counts kept and ranked
  const bool hum = VARS && (C.variants & SIM_FLAG_HIT_UNDER_MISS) != 0;  // ops drawn under a miss
  const int rd = PIPE ? C.rdelay : 1;  // router delay D: arrivals wait D-1 cycles in a pipeline
  const uint32_t wsel = C.W > 1 ? 0u : ~0u;  // prod_mask's row when the chip is one column wide
  const int negW = -C.W;
  const bool lspd = LSPDB && C.lspd != 0;  // the directory model (Sec. 3.2)
  const bool mig = MIGB && lspd && C.mig > 0;  // with migration (Sec. 3.3): N accessors per way
  const int mg = mig ? C.mig : 0;
  const uint32_t ym = LSPDB ? ~CTL_BIT : ~0u;  // an inject cycle without the LSPD control bit
  // the tile that keeps a line's directory entry
  auto dir_of = [&](int line) -> int { return C.lspd == 2 ? C.dir_center : (int)mod_n(C, (uint32_t)line); };
  const int patch = e.patch;
  const int pxi = patch % C.pgx, pyi = patch / C.pgx;
  const int x0 = pxi * C.pw, y0 = pyi * C.ph;
  const int cols = min(C.pw, C.W - x0), rows = min(C.ph, C.H - y0);
  const int ntiles = cols * rows;
  const int j = threadIdx.x;
  const bool active = j < ntiles;
  const int lx = active ? j % cols : 0, ly = active ? j / cols : 0;
  const int x = x0 + lx, y = y0 + ly, t = y * C.W + x;
  // geometry of the tile as bits of one vector register (bit p: link p exists; 4+p: the neighbour
  // is in this patch; 8+p: it is across a patch edge); re-read each cycle so the compiler keeps
  // these as bits instead of a dozen live scalar lane masks
  uint32_t geo0;
  {
    const bool a0 = active && y > 0, a1 = active && y < C.H - 1, a2 = active && x < C.W - 1, a3 = active && x > 0;
    const bool b0 = a0 && ly > 0, b1 = a1 && ly < rows - 1, b2 = a2 && lx < cols - 1, b3 = a3 && lx > 0;
    geo0 = (a0 ? 1u : 0u) | (a1 ? 2u : 0u) | (a2 ? 4u : 0u) | (a3 ? 8u : 0u) | (b0 ? 16u : 0u) | (b1 ? 32u : 0u) |
           (b2 ? 64u : 0u) | (b3 ? 128u : 0u) | ((a0 && !b0) ? 256u : 0u) | ((a1 && !b1) ? 512u : 0u) |
           ((a2 && !b2) ? 1024u : 0u) | ((a3 && !b3) ? 2048u : 0u);
  }
#define GEO(bit) (((geo >> (bit)) & 1u) != 0u)
#define GEO_BIT(g, bit) ((((g) >> (bit)) & 1u) != 0u)
  const int4 EMPTY = make_int4(-1, -1, -1, -1);
  // Patch-edge slots as byte offsets inside one parity's half of the slot array (which is
  // 4 N slots of 16 bytes): the slot each edge input is read from (0, a shared slot, where port
  // p has no patch edge) and the neighbour's slot each edge output goes to (0 where unused).
  // The half's base is the same for the whole launch, so it is kept in scalar registers and a
  // slot access needs no address arithmetic of its own.
  uint32_t ein0 = 0, ein1 = 0, ein2 = 0, ein3 = 0, eout0 = 0, eout1 = 0, eout2 = 0, eout3 = 0;
  {
    const uint32_t n16 = (uint32_t)N * 16u, t16 = (uint32_t)t * 16u, w16 = (uint32_t)C.W * 16u;
    if (GEO_BIT(geo0, 8)) { ein0 = t16; eout0 = n16 + t16 - w16; }       // north: its south input
    if (GEO_BIT(geo0, 9)) { ein1 = n16 + t16; eout1 = t16 + w16; }       // south: its north input
    if (GEO_BIT(geo0, 10)) { ein2 = 2 * n16 + t16; eout2 = 3 * n16 + t16 + 16; }  // east: its west
    if (GEO_BIT(geo0, 11)) { ein3 = 3 * n16 + t16; eout3 = 2 * n16 + t16 - 16; }  // west: its east
  }
  const unsigned long long link_u = (unsigned long long)(uintptr_t)C.link;
  const char* const link_s = reinterpret_cast<const char*>(
      (uintptr_t)(((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(link_u >> 32)) << 32) |
                  (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)link_u)));
  const uint32_t half16 = (uint32_t)N * 64u;  // bytes of one parity's half
#define EDGE_IN(par, off) reinterpret_cast<const int4*>(link_s + (size_t)((par) ? half16 : 0u) + (size_t)(off))
#define EDGE_OUT(par, off) reinterpret_cast<int4*>(const_cast<char*>(link_s) + (size_t)((par) ? half16 : 0u) + (size_t)(off))

  for (int i = threadIdx.x; i < NSTAT; i += blockDim.x) L.v[i] = 0;
  if (threadIdx.x == 0) s_fail = 0;
  s_link[0][5][j] = EMPTY;
  s_link[1][5][j] = EMPTY;
  Acc acc = {};
  const int c0 = ld_coh(&C.flags[patch * FLAG_STRIDE]);
  const int c_end = max(c0, min(min(c0 + chunk, e.stop >= 0 ? e.stop : C.stop), patch == C.halt_patch ? C.halt_cycle : INT_MAX));
  int c_done = c0;
  // pipeline entry of the current cycle (cycle mod (D-1)): the flits it holds leave this cycle,
  // and this cycle's arrivals take their place
  int pe = (PIPE && rd > 1) ? (int)((uint32_t)c0 % (uint32_t)(rd - 1)) : 0;

  int4 k0 = EMPTY, k1 = EMPTY, k2 = EMPTY;
  int fdst = -1, rcv = 0;  // forced background destination; flits of the awaited reply received
  int hline = -1, hissue = 0;  // hit under miss: the held op's line and issue cycle (none: -1, 0)
  // LSPD core words: remote-access target, pending eviction notice, directory checksum lo, hi
  int4 k4 = make_int4(-1, -1, 0, 0);
  // migration core words: pending claim (line), the block sent away, its destination (with the
  // in-transit bit until its arrival notice is served), a pending arrival notice (its source)
  int4 k5 = EMPTY;
  uint32_t geo = geo0;
  const bool i0 = GEO(4), i1 = GEO(5), i2 = GEO(6), i3 = GEO(7);
  if (active) {
    k0 = gload4(&C.core[t]);
    k1 = gload4(&C.core[N + t]);
    k2 = gload4(&C.core[2 * N + t]);
    const int4 k3 = gload4(&C.core[3 * N + t]);
    fdst = k3.x;
    rcv = k3.y;
    if (VARS) {
      hline = k3.z;
      hissue = k3.w;
    }
    if (lspd) k4 = gload4(&C.core[4 * N + t]);
    if (mig) k5 = gload4(&C.core[5 * N + t]);
    const int par = c0 & 1;
    if (i0) {
      const int4 w = gload4(&C.link[(par * 4 + 0) * N + t]);
      s_link[par][0][j] = VARS ? slot_decode_aged(w) : slot_decode(w);
    }
    if (i1) {
      const int4 w = gload4(&C.link[(par * 4 + 1) * N + t]);
      s_link[par][1][j] = VARS ? slot_decode_aged(w) : slot_decode(w);
    }
    if (i2) {
      const int4 w = gload4(&C.link[(par * 4 + 2) * N + t]);
      s_link[par][2][j] = VARS ? slot_decode_aged(w) : slot_decode(w);
    }
    if (i3) {
      const int4 w = gload4(&C.link[(par * 4 + 3) * N + t]);
      s_link[par][3][j] = VARS ? slot_decode_aged(w) : slot_decode(w);
    }
  }
  // this tile's cache arrays
  const int ways1 = W48 ? 4 : C.w1, ways2 = W48 ? 8 : C.w2;  // way counts (compile-time with W48)
  int* const l1_base = C.l1 + (size_t)(active ? t : 0) * (size_t)C.s1 * (size_t)ways1;
  int* const l2_base = C.l2 + (size_t)(active ? t : 0) * (size_t)C.s2 * (size_t)ways2;
  Prefetch P;
  if (active) {
    draw_ahead(C, t, c0, P);
    prefetch<MULTI, VARS, W48, LSPDB, MIGB>(C, t, c0, k0, k1, k2, hline, hum, l1_base, l2_base, P, k4, k5);
  }
  __syncthreads();

  for (int c = c0; c <= c_end; ++c) {
    const bool step = c < c_end;
    const bool dig = DIGEST && digests != nullptr && c > c0;  // (the watchdog runs this build without)
    if (!step && !dig) break;
    const int cur = c & 1, nxt = cur ^ 1;
    unsigned long long h = 0;
    bool ok = true;
    if (active) {
      uint32_t geo = geo0;
      asm volatile("" : "+v"(geo));
      const bool v0 = GEO(0), v1 = GEO(1), v2 = GEO(2), v3 = GEO(3);
      const bool i0 = GEO(4), i1 = GEO(5), i2 = GEO(6), i3 = GEO(7);
      const bool e0 = GEO(8), e1 = GEO(9), e2 = GEO(10), e3 = GEO(11);
      // ---- inputs of cycle c: interior from LDS, edges polled until stamped c ----------------
      // First read of the patch-edge slots, issued by every lane of the wave (a lane without
      // an edge on port p reads one shared slot instead): a fixed number of loads lets the
      // compiler wait for the prefetched words in phase one without waiting for these.
      int4 w0 = EMPTY, w1 = EMPTY, w2 = EMPTY, w3 = EMPTY;
      // with D > 1, the pipeline entry leaving this cycle (raw slot words), read ahead as well
      int4 pp0 = EMPTY, pp1 = EMPTY, pp2 = EMPTY, pp3 = EMPTY;
      if (PIPE && rd > 1 && step) {
        const int4* pq = &C.pipe[(size_t)pe * 4 * N + t];
        if (v0) pp0 = gload4(pq);
        if (v1) pp1 = gload4(pq + N);
        if (v2) pp2 = gload4(pq + 2 * N);
        if (v3) pp3 = gload4(pq + 3 * N);
      }
      if (MULTI) {
        w0 = ld_slot(EDGE_IN(cur, ein0), true);
        w1 = ld_slot(EDGE_IN(cur, ein1), true);
        w2 = ld_slot(EDGE_IN(cur, ein2), true);
        w3 = ld_slot(EDGE_IN(cur, ein3), true);
      }
      // the four input rows of this tile, read by every lane (rows of ports without an
      // in-patch neighbour hold stale words, replaced below); their wait hides behind phase one
      const int4 l0 = s_link[cur][0][j], l1 = s_link[cur][1][j], l2 = s_link[cur][2][j], l3 = s_link[cur][3][j];
      uint32_t pf = P.flags;
      asm volatile("" : "+v"(pf));
      const bool p_svc = (pf & PF_SVC) != 0, p_local = (pf & PF_LOCAL) != 0, p_fill = (pf & PF_FILL) != 0;
      const bool p_forced = (pf & PF_FORCED) != 0, p_drawn = (pf & PF_DRAWN) != 0;
      const bool p_retry = VARS && (pf & PF_RETRY) != 0, p_hum = VARS && (pf & PF_HUM) != 0;
      // the core words as they stand after cycle c-1 (the digest hashes them after the links)
      const int4 d0 = k0, d1 = k1, d2 = k2;
      const int dhl = hline, dhi = hissue;
      const int dfd = fdst, drcv = rcv;
      const int4 dk4 = k4, dk5 = k5;
      if (step) {
        // (-1 = none maps to 0; a tile index to 1..N; LSPD: the served requester without its
        // message kind, the remote-access target, and the lines the prefetch checked)
        const int who1 = LSPDB && k1.x >= 0 ? (k1.x & 0xFFFFFF) : k1.x;
        const uint32_t top = max(max(max((uint32_t)(who1 + 1), (uint32_t)(k1.w + 1)), max((uint32_t)(k2.y + 1), (uint32_t)(k1.z + 1))),
                                 max((uint32_t)(k2.x + 1), (uint32_t)(k4.x + 1)));
        // (migration: the pending claim's line, the forwarded block's destination, the notice's
        // target)
        const uint32_t top5 = MIGB ? max(k5.z >= 0 ? (uint32_t)((k5.z & ~MIG_TRANSIT) + 1) : 0u, (uint32_t)(k5.w + 1)) : 0u;
        if (top > (uint32_t)N || (LSPDB && ((P.flags & PF_BAD) || (k4.y >= 0 && k4.y >= C.lines))) ||
            (MIGB && (top5 > (uint32_t)N || (k5.x >= 0 && k5.x >= C.lines)))) {
          st_coh(C.err, 2);  // a corrupt queue index: stop rather than address memory with it
          ok = false;
        }
      }
      bool dirtyR = false, dirtyL = false, dirty1 = false;
      int node_tail = -1, node_rq = -1, node_ready = 0, node_line = 0, node_w = 0;
      int4 nh = P.nh, nm = P.nm;
      if (step && ok) {
        // phase one reads no link input: it runs while this cycle's patch-edge reads are in flight
        // ---- phase one: home L2 service, then the core (Sec. 7.1 phase one; Sec. 3.5) -------
        // appends requester rq to the hit queue (replies with the block) or the miss queue (a
        // static home's memory misses; the directory's one-flit answers); its node is stored in
        // phase three
        auto enqueue = [&](bool hitq, int rq, int ready, int word) {
          node_rq = rq;
          node_ready = ready;
          node_line = word;
          const int4 fresh = make_int4(-1, ready, word, 0);
          if (hitq) {
            if (k1.w >= 0) { node_tail = k1.w; if (k1.w == k1.z) nh.x = rq; }
            else { k1.z = rq; nh = fresh; }
            k1.w = rq;
          } else {
            if (k2.y >= 0) { node_tail = k2.y; if (k2.y == k2.x) nm.x = rq; }
            else { k2.x = rq; nm = fresh; }
            k2.y = rq;
          }
        };
        // LSPD (Sec. 3.2): a write of one of this tile's directory entries, which also moves the
        // tile's checksum of them (k4.z, k4.w)
        int fwd_line = -1, fwd_val = 0;  // the entry the service wrote, read again by the core
        auto dir_write = [&](int line, int old_owner, int owner) {
          typedef unsigned long long u64;
          u64 sum = (u64)(uint32_t)k4.z | ((u64)(uint32_t)k4.w << 32);
          if (old_owner >= 0) sum -= mix64(((u64)(uint32_t)line << 32) | (uint32_t)old_owner);
          if (owner >= 0) sum += mix64(((u64)(uint32_t)line << 32) | (uint32_t)owner);
          k4.z = (int)(uint32_t)sum;
          k4.w = (int)(uint32_t)(sum >> 32);
          *gp(&C.loc[line]) = owner;
          fwd_line = line;
          fwd_val = owner;
        };
        // migration: the access histories of the two slice sets (the ways' order, mg words a way)
        int* const histR = MIGB ? C.l2h + (size_t)(P.setR - C.l2) * mg : nullptr;
        int* const histL = MIGB ? C.l2h + (size_t)(P.setL - C.l2) * mg : nullptr;
        const int svc_type = k1.x >> 24;  // LSPD: the served message's kind (Q_*)
        if (p_svc && !lspd) {
          const int rq = k1.x, line = k1.y;
          const bool hit = set_touch(P.vR, ways2, line, true, dirtyR);
          acc.l2_hit += hit;
          acc.l2_miss += !hit;
          enqueue(hit, rq, (hit ? c : c + C.mem_lat) + idl, line);
          k1.x = -1;
          k1.y = -1;
        } else if (LSPDB && p_svc) {  // remote access, directory access, eviction notice (Sec. 3.2)
          const int who = k1.x & 0xFFFFFF, line = k1.y;
          if (svc_type == Q_RA) {  // the block is here: reply with it; gone: a trap
            const int i = way_of(P.vR, line);
            if (i >= 0) {
              acc.l2_hit++;
              int n = 0;
              if (mig) {  // Sec. 3.3: the block's list of its last accessors
                n = hist_note(histR, mg, i, who);
                hist_front(histR, mg, i);
              }
              way_front(P.vR, i);
              dirtyR = true;
              // a remote tile made most of the block's last accesses: the block moves there,
              // unless it has just moved here and this slice still waits for the directory to
              // acknowledge its claim, or another block of this slice is still on its way
              const bool claiming = k0.x == CORE_WAIT && k0.z == line;
              const bool sending = k5.z >= 0 && (k5.z & MIG_TRANSIT);
              if (mig && 2 * n > mg && !claiming && !sending) {
                k5.y = line;  // sent whole; this slice serves it until told of its arrival
                k5.z = who | MIG_TRANSIT;
                lds_add(L, SIM_ST_MIGRATE, 1);
                enqueue(true, who, c + idl, line | MIG_MARK);
              } else {
                enqueue(true, who, c + idl, line);
              }
            } else if (mig && k5.y == line) {  // Sec. 3.3: redirected to where the block went
              lds_add(L, SIM_ST_REDIRECT, 1);
              enqueue(false, who, c + idl, k5.z & ~MIG_TRANSIT);
            } else {
              lds_add(L, SIM_ST_TRAP, 1);
              enqueue(false, who, c + idl, CODE_TRAP);
            }
          } else if (MIGB && svc_type == Q_ARRIVED) {  // the block sent away has arrived: this copy goes
            if (k5.z == (who | MIG_TRANSIT)) {
              const int i = way_of(P.vR, line);
              if (i >= 0) {
                way_remove(P.vR, ways2, i);
                if (mig) hist_remove(histR, mg, ways2, i);
                dirtyR = true;
              }
              k5.z = who;
            }
          } else if (MIGB && svc_type == Q_CLAIM) {  // the directory names the block's new owner and tells it
            dir_write(line, P.loc_svc, who);
            enqueue(false, who, c + idl, CODE_ACK);
          } else if (svc_type == Q_DA) {  // the owner, or (not on chip) the asker brings it from memory
            lds_add(L, SIM_ST_DIR_ACCESS, 1);
            int code = P.loc_svc;
            if (code < 0) {
              dir_write(line, -1, who);
              lds_add(L, SIM_ST_DIR_NACK, 1);
              code = CODE_NACK;
            }
            enqueue(false, who, c + idl, code);
          } else {  // the entry names the evicting slice until its notice arrives
            dir_write(line, who, -1);
            lds_add(L, SIM_ST_DIR_EVICT, 1);
          }
          k1.x = -1;
          k1.y = -1;
        }
        // the core's slice access below sees the service's changes when both touch one set
        if (LSPDB && (pf & PF_SVC) && (pf & (PF_SLICE | PF_FILLMEM)) && (svc_type == Q_RA || (MIGB && svc_type == Q_ARRIVED)) &&
            P.setL == P.setR) {
#pragma unroll
          for (int i = 0; i < 8; ++i) P.vL[i] = P.vR[i];
          dirtyL = dirtyL || dirtyR;
          dirtyR = false;
        }
        if (p_fill) {
          bool claim = false;  // migration: the op completes when the directory has the new owner
          if (LSPDB && (pf & PF_FILLMEM)) {  // from memory (or migrated) into the local slice too;
            const int victim = way_insert(P.vL, ways2, k0.z);  // an evicted block leaves the directory
            if (mig) hist_insert(histL, mg, ways2);  // its history starts empty
            dirtyL = true;
            if (victim >= 0 && (unsigned)victim >= (unsigned)C.lines) {
              st_coh(C.err, 2);  // a corrupt slice word: stop rather than address memory with it
              ok = false;
            } else if (victim >= 0 && mig && victim == k5.y && k5.z >= 0 && (k5.z & MIG_TRANSIT)) {
              // the block on its way elsewhere leaves this slice: its new owner's claim updates
              // the directory, and requests still reaching here are redirected
            } else if (victim >= 0 && dir_of(victim) == t) {
              dir_write(victim, t, -1);
              lds_add(L, SIM_ST_DIR_EVICT, 1);
            } else if (victim >= 0) {
              k4.y = victim;  // the eviction notice goes out before the next directory access
            }
            if (MIGB && k0.x == CORE_FILL_MIG) {  // Sec. 3.3: the directory learns the new owner
              if (dir_of(k0.z) == t) {
                dir_write(k0.z, fwd_line == k0.z ? fwd_val : P.loc_core, t);
              } else {
                claim = true;
                k5.x = k0.z;
                k0.x = CORE_WAIT;
              }
            }
          }
          if (!MIGB || !claim) {
            set_touch(P.u, ways1, P.line_op, true, dirty1);
            const int lat = c - k0.w;
            acc.ops_done++;
            acc.op_lat += (unsigned long long)lat;
            acc.op_lat_max = max(acc.op_lat_max, lat);
            k0.x = CORE_IDLE;
          }
        } else if (k0.x == CORE_L1MISS && k0.y == c) {
          if (LSPDB && lspd) {  // own slice, then the directory (Sec. 3.2)
            const int i = way_of(P.vL, k0.z);
            if (!(pf & PF_SLICE)) {
              k0.y = c + 1;  // a pending eviction notice or claim goes out first
            } else if (i >= 0) {
              acc.l2_hit++;
              if (mig) {  // the local core's access
                hist_note(histL, mg, i, t);
                hist_front(histL, mg, i);
              }
              way_front(P.vL, i);
              dirtyL = true;
              k0.x = CORE_FILL;
              k0.y = c + 1;
            } else if (mig && k5.y == k0.z && k5.z >= 0 && (k5.z & MIG_TRANSIT)) {
              // this slice sent the block away and has since evicted its copy: the core waits
              // for the arrival notice before it asks for the block again (so that the notice
              // cannot remove a copy that came back to this slice)
              k0.y = c + 1;
            } else if (pf & PF_DIRCORE) {  // this tile keeps the entry: look it up at once
              lds_add(L, SIM_ST_DIR_ACCESS, 1);
              int o = fwd_line == k0.z ? fwd_val : P.loc_core;
              if (MIGB && o == t && k5.y == k0.z) {  // this slice gave the block away; the new
                o = k5.z & ~MIG_TRANSIT;             // owner's claim is still on the way
                lds_add(L, SIM_ST_REDIRECT, 1);
              }
              if (o == t) {  // this slice's own eviction (or an older migration) is still on its way: look again
                lds_add(L, SIM_ST_TRAP, 1);
                k0.y = c + 1;
              } else {
                acc.l2_miss++;
                if (o < 0) {
                  dir_write(k0.z, -1, t);
                  lds_add(L, SIM_ST_DIR_NACK, 1);
                  k0.x = CORE_FILL_MEM;
                  k0.y = c + C.mem_lat;
                } else {
                  k0.x = CORE_SEND_RA;
                  k4.x = o;
                  k0.y = c + idl;
                  acc.req_made++;
                }
              }
            } else {
              acc.l2_miss++;
              k0.x = CORE_SEND_DA;
              k0.y = c + idl;
            }
          } else if (p_local) {
            if (p_svc && P.setL == P.setR) {
#pragma unroll
              for (int i = 0; i < 8; ++i) P.vL[i] = P.vR[i];
            }
            const bool hit = set_touch(P.vL, ways2, k0.z, true, dirtyL);
            acc.l2_hit += hit;
            acc.l2_miss += !hit;
            k0.x = CORE_FILL;
            k0.y = hit ? c + 1 : c + C.mem_lat;
          } else {
            k0.x = CORE_SEND;
            acc.req_made++;
          }
        } else if (p_retry || p_forced || p_drawn) {
          const int issued = p_retry ? hissue : c;  // a held op counts from its first issue
          if (p_retry) {
            hline = -1;
            hissue = 0;
          } else {
            acc.ops_issued++;
          }
          if (p_forced) k2.w = -1;
          k0.z = P.line_op;
          k0.w = issued;
          if (set_touch(P.u, ways1, P.line_op, false, dirty1)) {
            acc.l1_hit++;
            acc.ops_done++;
            if (p_retry) {
              acc.op_lat += (unsigned long long)(c - issued);
              acc.op_lat_max = max(acc.op_lat_max, c - issued);
            }
          } else {
            acc.l1_miss++;
            k0.x = CORE_L1MISS;
            k0.y = c + C.l1_lat;
          }
        }
        if (p_hum) {  // a hit completes under the miss; a miss is held until the fill (Sec. 3.5)
          acc.ops_issued++;
          if (set_touch(P.u, ways1, P.line_op, false, dirty1)) {
            acc.l1_hit++;
            acc.ops_done++;
          } else {
            hline = P.line_op;
            hissue = c;
          }
        }

      }
      if (MULTI && (e0 | e1 | e2 | e3)) {
        int spins = 0;
        for (;;) {
          const bool p0 = e0 && !slot_has_stamp(w0, (uint32_t)c), p1 = e1 && !slot_has_stamp(w1, (uint32_t)c);
          const bool p2 = e2 && !slot_has_stamp(w2, (uint32_t)c), p3 = e3 && !slot_has_stamp(w3, (uint32_t)c);
          if (!(p0 | p1 | p2 | p3)) break;
          if ((++spins & 63) == 0 && (spins > C.spin_limit || ld_coh(C.err))) {
            note_hang(C.err);
            ok = false;
            break;
          }
          if (p0) w0 = ld_slot(EDGE_IN(cur, ein0), true);
          if (p1) w1 = ld_slot(EDGE_IN(cur, ein1), true);
          if (p2) w2 = ld_slot(EDGE_IN(cur, ein2), true);
          if (p3) w3 = ld_slot(EDGE_IN(cur, ein3), true);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // drain: every load of cycle c is in, every store of c-1 done
      // this cycle's arrivals.  The checking build hashes them, so it decodes them whole; the
      // timed build only makes dst -1 for an empty input: nothing reads the other words of an
      // empty row (keys take its sign, outputs gather only assigned rows or the empty row 5)
      auto arrival = [&](bool in, bool edge, const int4& l, const int4& w) -> int4 {
        if (DIGEST) return sel4(in, l, edge ? (VARS ? slot_decode_aged(w) : slot_decode(w)) : EMPTY);
        const uint32_t keep = VARS ? STAMP_OFF : TILE_BITS_MASK;  // (the count rides along)
        const bool live = edge && ((uint32_t)w.x & TILE_BITS_MASK) != TILE_BITS_MASK;
        return make_int4(in ? l.x : (live ? (int)((uint32_t)w.x & keep) : -1), in ? l.y : w.y,
                         in ? l.z : (int)((uint32_t)w.z & keep), in ? l.w : w.w);
      };
      const int4 a0 = arrival(i0, e0, l0, w0), a1 = arrival(i1, e1, l1, w1);
      const int4 a2 = arrival(i2, e2, l2, w2), a3 = arrival(i3, e3, l3, w3);
      // this cycle's arbitration inputs: the arrivals, or with D > 1 the flits that arrived D-1
      // cycles ago, leaving the pipeline now
      const bool piped = PIPE && rd > 1 && step;
      const int4 f0 = piped ? (v0 ? slot_decode_aged(pp0) : EMPTY) : a0;
      const int4 f1 = piped ? (v1 ? slot_decode_aged(pp1) : EMPTY) : a1;
      const int4 f2 = piped ? (v2 ? slot_decode_aged(pp2) : EMPTY) : a2;
      const int4 f3 = piped ? (v3 ? slot_decode_aged(pp3) : EMPTY) : a3;
      // every input row now holds this cycle's input (a patch-edge flit, or empty where there
      // is no link; an in-patch row is rewritten with what it held, or with D > 1 with the
      // pipeline's output)
      s_link[cur][0][j] = f0;
      s_link[cur][1][j] = f1;
      s_link[cur][2][j] = f2;
      s_link[cur][3][j] = f3;

      if (dig) {  // state owned by t after cycle c-1: its arrivals, core words and pipeline
        const int4 g0 = VARS ? row_clean(a0) : a0, g1 = VARS ? row_clean(a1) : a1;
        const int4 g2 = VARS ? row_clean(a2) : a2, g3 = VARS ? row_clean(a3) : a3;
        h = mix64(((unsigned long long)(uint32_t)(c - 1) << 32) | (uint32_t)t);
        h = mix_pair(h, g0.x, g0.y); h = mix_pair(h, g0.z, g0.w);
        h = mix_pair(h, g1.x, g1.y); h = mix_pair(h, g1.z, g1.w);
        h = mix_pair(h, g2.x, g2.y); h = mix_pair(h, g2.z, g2.w);
        h = mix_pair(h, g3.x, g3.y); h = mix_pair(h, g3.z, g3.w);
        h = mix_pair(h, d0.x, d0.y); h = mix_pair(h, d0.z, d0.w);
        h = mix_pair(h, d1.x, d1.y); h = mix_pair(h, d1.z, d1.w);
        h = mix_pair(h, d2.x, d2.y);
        h = mix_pair(h, d2.z, 0);
        h = mix_pair(h, 0, 0);
        h = mix_pair(h, d2.w, dfd);
        h = mix_pair(h, drcv, 0);
        h = mix_pair(h, dhl, dhi);  // the op held by hit under miss (-1, 0: none)
        h = mix_pair(h, dk4.x, dk4.y);  // LSPD: remote-access target, pending eviction notice
        h = mix_pair(h, dk4.z, dk4.w);  // and the directory checksum (without LSPD: -1, -1, 0, 0)
        h = mix_pair(h, dk5.x, dk5.y);  // migration: claim, forwarded block,
        h = mix_pair(h, dk5.z, dk5.w);  // its destination, arrival notice (all -1 without)
        if (aged)  // the arrivals' deflection counts
          h = mix_pair(h, (int)(row_age(a0) | (row_age(a1) << 16)), (int)(row_age(a2) | (row_age(a3) << 16)));
        if (PIPE && rd > 1) {  // stage st: the flits that leave the pipeline in cycle c-1+st
          int pst = pe;
          for (int st = 1; st < rd; ++st) {
            const int4* pq = &C.pipe[(size_t)pst * 4 * N + t];
            const int4 x0 = v0 ? gload4(pq) : EMPTY, x1 = v1 ? gload4(pq + N) : EMPTY;
            const int4 x2 = v2 ? gload4(pq + 2 * N) : EMPTY, x3 = v3 ? gload4(pq + 3 * N) : EMPTY;
            const int4 y0 = v0 ? slot_decode(x0) : EMPTY, y1 = v1 ? slot_decode(x1) : EMPTY;
            const int4 y2 = v2 ? slot_decode(x2) : EMPTY, y3 = v3 ? slot_decode(x3) : EMPTY;
            h = mix_pair(h, y0.x, y0.y); h = mix_pair(h, y0.z, y0.w);
            h = mix_pair(h, y1.x, y1.y); h = mix_pair(h, y1.z, y1.w);
            h = mix_pair(h, y2.x, y2.y); h = mix_pair(h, y2.z, y2.w);
            h = mix_pair(h, y3.x, y3.y); h = mix_pair(h, y3.z, y3.w);
            if (aged) {
              const uint32_t b0 = v0 ? slot_age(x0) : 0u, b1 = v1 ? slot_age(x1) : 0u;
              const uint32_t b2 = v2 ? slot_age(x2) : 0u, b3 = v3 ? slot_age(x3) : 0u;
              h = mix_pair(h, (int)(b0 | (b1 << 16)), (int)(b2 | (b3 << 16)));
            }
            pst = pst + 1 == rd - 1 ? 0 : pst + 1;
          }
        }
      }
      if (step && ok) {
        // ---- phase two: injection, then oldest-first arbitration ----------------------------
        const int arrivals = (f0.x >= 0) + (f1.x >= 0) + (f2.x >= 0) + (f3.x >= 0);
        const int deg = (int)v0 + (int)v1 + (int)v2 + (int)v3;
        int cls = -1;
        // (LSPD: the miss queue holds one-flit answers, and the core's own flit is a pending
        // eviction notice, a directory access or a remote access)
        // (migration: an arrival notice or a claim as well)
        const bool own = LSPDB && lspd ? (k4.y >= 0 || (MIGB && (k5.w >= 0 || k5.x >= 0)) ||
                                          ((k0.x == CORE_SEND_DA || k0.x == CORE_SEND_RA) && k0.y <= c))
                                       : (k0.x == CORE_SEND && (!VARS || k0.y + idl <= c));
        if (k2.x >= 0 && nm.y <= c) cls = 0;
        else if (k1.z >= 0 && (!VARS || nh.y <= c)) cls = 1;
        else if (own) cls = 2;
        else if (fdst >= 0) cls = 3;
        else if (k2.z > 0) cls = 4;
        if (cls >= 0 && arrivals >= deg) {
          acc.inj_blocked++;
          cls = -1;
        }
        int4 fi = EMPTY;
        if (cls >= 0) {
          fi.y = c;
          fi.z = t;
          if (LSPDB && lspd && cls == 0) {  // the directory's answer or a trap: one flit, control bit
            fi.x = k2.x;
            fi.y = (int)((uint32_t)c | CTL_BIT);
            fi.w = (KIND_REPLY << 30) | (nm.z + CODE_BASE);
            k2.x = nm.x;
            if (nm.x < 0) k2.y = -1;
            acc.inj_reply++;
          } else if (LSPDB && lspd && cls == 2) {
            if (k4.y >= 0) {  // eviction notice to the block's directory tile
              fi.x = dir_of(k4.y);
              fi.y = (int)((uint32_t)c | CTL_BIT);
              fi.w = (KIND_DIR << 30) | k4.y;
              k4.y = -1;
            } else if (MIGB && k5.w >= 0) {  // Sec. 3.3: the migrated block has arrived; its source drops its copy
              fi.x = k5.w;
              fi.y = (int)((uint32_t)c | CTL_BIT);
              fi.w = KIND_REQ << 30;
              k5.w = -1;
            } else if (MIGB && k5.x >= 0) {  // a migrated block's new owner, to its directory tile
              fi.x = dir_of(k5.x);
              fi.y = (int)((uint32_t)c | CTL_BIT);
              fi.w = (KIND_BG << 30) | k5.x;
              k5.x = -1;
            } else if (k0.x == CORE_SEND_DA) {  // directory access
              fi.x = dir_of(k0.z);
              fi.w = (KIND_DIR << 30) | k0.z;
              k0.x = CORE_WAIT;
            } else {  // remote access at the owner
              fi.x = k4.x;
              fi.w = (KIND_REQ << 30) | k0.z;
              k4.x = -1;
              k0.x = CORE_WAIT;
            }
            acc.inj_req++;
          } else if (cls <= 1) {  // a flit of the head's reply; the head is popped with the last one
            const int4 hd = cls == 0 ? nm : nh;
            fi.x = cls == 0 ? k2.x : k1.z;
            const int sent = hd.w + 1;
            // a migrating block (Sec. 3.3, Table 1) goes as MIG_FLITS answer flits
            const bool mig_pk = MIGB && lspd && (hd.z & MIG_MARK);
            const int len = mig_pk ? MIG_FLITS : C.reply_flits;
            const bool last = (!PACKETS && !mig_pk) || sent >= len;  // (a single-flit build still sends a block whole)
            if (last) {
              if (cls == 0) { k2.x = hd.x; if (hd.x < 0) k2.y = -1; }
              else { k1.z = hd.x; if (hd.x < 0) k1.w = -1; }
            }
            // the sent count goes to the head's node; a node appended this cycle is written
            // whole with phase one's stores, so its count rides with that store
            if ((PACKETS || mig_pk) && len > 1) {
              if (fi.x == node_rq) node_w = last ? 0 : sent;
              else st_i<MULTI>(reinterpret_cast<int*>(&C.node[fi.x]) + 3, last ? 0 : sent);
            }
            fi.w = (KIND_REPLY << 30) | hd.z;
            if (mig_pk) {
              fi.w = (KIND_REPLY << 30) | (CODE_MIG + CODE_BASE);
              fi.y = (int)((uint32_t)c | CTL_BIT);
            }
            acc.reply_sent += last && !mig_pk;
            acc.inj_reply++;
          } else if (cls == 2) {
            fi.x = (int)mod_n(C, (uint32_t)k0.z);
            fi.w = (KIND_REQ << 30) | k0.z;
            k0.x = CORE_WAIT;
            acc.inj_req++;
          } else {
            if (cls == 3) {
              fi.x = fdst;
              fdst = -1;
            } else {
              const uint4 r2 = philox((uint32_t)c, (uint32_t)t, 1u, 0u, C.key0, C.key1);
              const int d = (int)__umulhi(r2.x, (uint32_t)(N - 1));
              fi.x = d + (d >= t);
              k2.z -= 1;
            }
            fi.w = (int)(KIND_BG << 30);
            acc.inj_bg++;
          }
        }
        // sort keys: (inject cycle, source), then the flit's productive ports as a 5-bit mask
        // (prod_mask) and its input index i as i ^ 7 in the low 8 bits (sources take 20 bits;
        // (inject cycle, source) is unique per flit, so the low bits never decide the order);
        // all ones for an empty input, which sorts last
        typedef unsigned long long u64;
        // (with deflection counts, the source and destination words carry the count in bits
        // 20-27, masked off here; the count itself is a first key word, most deflected first)
#define SRCW(f) (VARS ? ((uint32_t)(f).z & TILE_BITS_MASK) : (uint32_t)(f).z)
#define DSTW(f) (VARS ? (int)((uint32_t)(f).x & TILE_BITS_MASK) : (f).x)
#define PM(f) prod_mask(DSTW(f), x - 1, y - 1, negW, C.w_magic, wsel)
        // (the masks are computed for every input, empty or not, so that no branch is taken here)
        const uint32_t m0 = PM(f0), m1 = PM(f1), m2 = PM(f2), m3 = PM(f3), m4 = PM(fi);
        // (an empty input's dst is -1: its sign makes both halves of the key all ones, no branch)
#define SKEY(f, m, i) ((u64)(((uint32_t)(f).y & ym) | (uint32_t)((f).x >> 31)) << 32 | \
                       (u64)((SRCW(f) << 8) | ((m) << 3) | (uint32_t)((i) ^ 7) | (uint32_t)((f).x >> 31)))
        u64 q0 = SKEY(f0, m0, 0), q1 = SKEY(f1, m1, 1), q2 = SKEY(f2, m2, 2), q3 = SKEY(f3, m3, 3), q4 = SKEY(fi, m4, 4);
#undef SKEY
#undef PM
#undef DSTW
#undef SRCW
#define AKEY(f) ((f).x < 0 ? ~0u : (uint32_t)AGE_MAX - row_age(f))
        uint32_t ak0 = 0, ak1 = 0, ak2 = 0, ak3 = 0, ak4 = 0;
        if (aged) { ak0 = AKEY(f0); ak1 = AKEY(f1); ak2 = AKEY(f2); ak3 = AKEY(f3); ak4 = AKEY(fi); }
#undef AKEY
#define CSWAP(a, b)                                                            \
  {                                                                            \
    const bool sw = VARS ? (ak##b < ak##a || (ak##b == ak##a && q##b < q##a)) : q##b < q##a; \
    const u64 qa = sw ? q##b : q##a, qb = sw ? q##a : q##b;                    \
    q##a = qa; q##b = qb;                                                      \
    if (VARS) { const uint32_t xa = sw ? ak##b : ak##a, xb = sw ? ak##a : ak##b; ak##a = xa; ak##b = xb; } \
  }
        CSWAP(0, 1) CSWAP(3, 4) CSWAP(2, 4) CSWAP(2, 3) CSWAP(1, 4) CSWAP(0, 3) CSWAP(0, 2) CSWAP(1, 3) CSWAP(1, 2)
#undef CSWAP
        s_link[cur][4][j] = fi;
        // ports off the mesh start out taken (bits 5-8: north, south, east, west)
        uint32_t taken = (v0 ? 0u : 32u) | (v1 ? 0u : 64u) | (v2 ? 0u : 128u) | (v3 ? 0u : 256u);
        unsigned dm = 0;
        uint32_t inv = 0x7FFFu;
        int ndefl = 0;
        arb_assign_mask<VARS>(q0, taken, inv, dm, ndefl);
        arb_assign_mask<VARS>(q1, taken, inv, dm, ndefl);
        arb_assign_mask<VARS>(q2, taken, inv, dm, ndefl);
        arb_assign_mask<VARS>(q3, taken, inv, dm, ndefl);
        arb_assign_mask<VARS>(q4, taken, inv, dm, ndefl);
        {  // every live flit moves over a link except the one ejected
          const int nlive = (f0.x >= 0) + (f1.x >= 0) + (f2.x >= 0) + (f3.x >= 0) + (fi.x >= 0);
          acc.trav += nlive - (int)(taken & 1u);
          acc.defl += ndefl;
          if (DIGEST && C.watch_age > 0) {  // watchdog (debug mode, checking build only): every
            // live flit took exactly one port (bits 0-4 of taken name the ports used, eject
            // included), and none is older than the bound (the oldest flit always advances)
            const uint32_t cu = (uint32_t)c;
            uint32_t oldest = 0;
            if (f0.x >= 0) oldest = max(oldest, cu - ((uint32_t)f0.y & ym));
            if (f1.x >= 0) oldest = max(oldest, cu - ((uint32_t)f1.y & ym));
            if (f2.x >= 0) oldest = max(oldest, cu - ((uint32_t)f2.y & ym));
            if (f3.x >= 0) oldest = max(oldest, cu - ((uint32_t)f3.y & ym));
            if (__builtin_popcount(taken & 31u) != nlive) {
              st_coh(C.err, ERR_ROUTER);
              ok = false;
            } else if (oldest > (uint32_t)C.watch_age) {
              st_coh(C.err, ERR_WATCHDOG);
              ok = false;
            }
          }
        }

        if (PIPE && rd > 1) {  // this cycle's arrivals enter the pipeline (stamped, as on the links)
          int4* pq = &C.pipe[(size_t)pe * 4 * N + t];
          if (v0) gstore4(pq, slot_encode(a0, (uint32_t)c));
          if (v1) gstore4(pq + N, slot_encode(a1, (uint32_t)c));
          if (v2) gstore4(pq + 2 * N, slot_encode(a2, (uint32_t)c));
          if (v3) gstore4(pq + 3 * N, slot_encode(a3, (uint32_t)c));
        }
        // ---- phase three: link outputs (patch edges first: neighbours poll for them), ejection,
        // then the next cycle's loads
#define out_for(p) s_link[cur][min((inv >> (3 * (p))) & 7u, 5u)][j]
        // the five gathers first (one LDS round trip), then the stores
        int4 o0 = out_for(0), o1 = out_for(1), o2 = out_for(2), o3 = out_for(3);
        const int4 oe = out_for(4);
        if (aged && dm) {  // a deflected flit leaves with one more deflection (Sec. 6.2.1)
          auto bump = [&](int4& o, unsigned p) {
            const unsigned i = (inv >> (3 * p)) & 7u;
            if (i > 4u || !((dm >> i) & 1u)) return;
            uint32_t a = row_age(o) + 1u;
            if (a > (uint32_t)AGE_MAX) {
              st_coh(C.err, 4);  // a flit deflected 65,536 times: reported as an invariant failure
              a = (uint32_t)AGE_MAX;
            }
            const uint32_t keep = ~(0xFFu << AGE_SHIFT);
            o.x = (int)(((uint32_t)o.x & keep) | ((a & 0xFFu) << AGE_SHIFT));
            o.z = (int)(((uint32_t)o.z & keep) | ((a >> 8) << AGE_SHIFT));
          };
          bump(o0, 0);
          bump(o1, 1);
          bump(o2, 2);
          bump(o3, 3);
        }
        const uint32_t ns = (uint32_t)(c + 1);
        if (v0 && !i0) st_slot(EDGE_OUT(nxt, eout0), slot_encode_row(o0, ns), MULTI);
        if (v1 && !i1) st_slot(EDGE_OUT(nxt, eout1), slot_encode_row(o1, ns), MULTI);
        if (v2 && !i2) st_slot(EDGE_OUT(nxt, eout2), slot_encode_row(o2, ns), MULTI);
        if (v3 && !i3) st_slot(EDGE_OUT(nxt, eout3), slot_encode_row(o3, ns), MULTI);
        // inside the patch: the neighbour's input slot opp(p) in LDS
        if (i0) s_link[nxt][1][j - cols] = o0;
        if (i1) s_link[nxt][0][j + cols] = o1;
        if (i2) s_link[nxt][3][j + 1] = o2;
        if (i3) s_link[nxt][2][j - 1] = o3;
        // phase one's stores: issued before the next cycle's loads of the same sets and nodes
        if (dirtyR) set_store(P.setR, ways2, P.vR);
        if (dirtyL) set_store(P.setL, ways2, P.vL);
        if (dirty1) set_store(P.set1, ways1, P.u);
        if (node_rq >= 0) {
          st_node<MULTI>(&C.node[node_rq], make_int4(-1, node_ready, node_line, node_w));
          if (node_tail >= 0) st_i<MULTI>(reinterpret_cast<int*>(&C.node[node_tail]), node_rq);
        }
        if (oe.x >= 0) {
          const int kind = (int)((uint32_t)oe.w >> 30);
          const bool ctl = LSPDB && ((uint32_t)oe.y & CTL_BIT);
          const int lat = c - (int)((uint32_t)oe.y & ym);
          const unsigned long long ulat = (unsigned long long)lat;
          // directory messages and ownership claims count as requests
          const bool as_req = kind == KIND_REQ || (LSPDB && kind == KIND_DIR) || (MIGB && kind == KIND_BG && ctl);
          const bool as_bg = kind == KIND_BG && !(MIGB && ctl);
          acc.ej_req += as_req;
          acc.ej_reply += kind == KIND_REPLY;
          acc.ej_bg += as_bg;
          acc.lat_req += as_req ? ulat : 0ull;
          acc.lat_reply += kind == KIND_REPLY ? ulat : 0ull;
          acc.lat_bg += as_bg ? ulat : 0ull;
          acc.lat_max = max(acc.lat_max, lat);
          lds_add(L, SIM_ST_HIST + min(15, 31 - __builtin_clz((unsigned)max(lat, 1))), 1);
          if (MIGB && kind == KIND_REQ && ctl) {  // migration: the block this slice sent has arrived
            k1.x = (int)((uint32_t)oe.z & TILE_BITS_MASK) | (Q_ARRIVED << 24);
            k1.y = k5.y;  // the block it sent (one at a time)
          } else if (kind == KIND_REQ) {
            acc.req_recv++;
            k1.x = VARS ? (int)((uint32_t)oe.z & TILE_BITS_MASK) : oe.z;
            k1.y = oe.w & LINE_MASK;
          } else if (MIGB && kind == KIND_BG && ctl) {  // migration: the new owner's claim
            k1.x = (int)((uint32_t)oe.z & TILE_BITS_MASK) | (Q_CLAIM << 24);
            k1.y = oe.w & LINE_MASK;
          } else if (LSPDB && kind == KIND_DIR) {  // directory access or (control bit) eviction notice
            k1.x = (int)((uint32_t)oe.z & TILE_BITS_MASK) | ((ctl ? Q_EV : Q_DA) << 24);
            k1.y = oe.w & LINE_MASK;
          } else if (LSPDB && kind == KIND_REPLY && ctl) {  // the directory's answer or a trap
            const int code = (oe.w & LINE_MASK) - CODE_BASE;
            if (MIGB && code == CODE_MIG) {  // a flit of the block migrating here; the last one fills it in
              rcv += 1;
              if (rcv >= MIG_FLITS) {  // the whole block is in; its source is told (Sec. 3.3)
                rcv = 0;
                k5.w = (int)((uint32_t)oe.z & TILE_BITS_MASK);
                k0.x = CORE_FILL_MIG;
                k0.y = c + 1;
              }
            } else if (MIGB && code == CODE_ACK) {  // the directory names this slice: L1 fill, op complete
              k0.x = CORE_FILL;
              k0.y = c + 1;
            } else if (code == CODE_NACK) {  // not on chip: from memory into the local slice
              k0.x = CORE_FILL_MEM;
              k0.y = c + C.mem_lat;
            } else if (code == CODE_TRAP || code == t) {  // stale entry: ask the directory again
              if (code == t) lds_add(L, SIM_ST_TRAP, 1);
              k0.x = CORE_SEND_DA;
              k0.y = c + 1;
            } else {  // the owner: a remote access to it
              k0.x = CORE_SEND_RA;
              k0.y = c + 1;
              k4.x = code;
              acc.req_made++;
            }
          } else if (kind == KIND_REPLY) {  // a flit of the block; the last one completes it
            rcv += PACKETS ? 1 : 0;
            if (!PACKETS || rcv >= C.reply_flits) {
              rcv = 0;
              acc.reply_recv++;
              k0.x = CORE_FILL;
              k0.y = c + 1;
            }
          }
        }
        if (N > 1 && P.r.w < C.bg_thr) {
          k2.z += 1;
          acc.bg_gen++;
        }
        if (c + 1 < c_end)
          prefetch<MULTI, VARS, W48, LSPDB, MIGB>(C, t, c + 1, k0, k1, k2, hline, hum, l1_base, l2_base, P, k4, k5);
#undef out_for
      }
    }
    if (dig) {
      h = wave_sum(h);
      if ((threadIdx.x & 63) == 0) atomicAdd(&digests[c - 1 - digest_base], h);
    }
    if (!ok) s_fail = 1;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only: this wave's LDS slot writes are done
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (s_fail) break;
    if (step) {
      c_done = c + 1;
      if (PIPE && rd > 1) pe = pe + 1 == rd - 1 ? 0 : pe + 1;
    }
  }

  // ---- write back: core words, interior slots of cycle c_done (stamped), flag, counters ----
  if (active) {
    gstore4(&C.core[t], k0);
    gstore4(&C.core[N + t], k1);
    gstore4(&C.core[2 * N + t], k2);
    gstore4(&C.core[3 * N + t], make_int4(fdst, rcv, hline, hissue));
    if (lspd) gstore4(&C.core[4 * N + t], k4);
    if (mig) gstore4(&C.core[5 * N + t], k5);
    const int par = c_done & 1;
    if (i0) gstore4(&C.link[(par * 4 + 0) * N + t], slot_encode(s_link[par][0][j], (uint32_t)c_done));
    if (i1) gstore4(&C.link[(par * 4 + 1) * N + t], slot_encode(s_link[par][1][j], (uint32_t)c_done));
    if (i2) gstore4(&C.link[(par * 4 + 2) * N + t], slot_encode(s_link[par][2][j], (uint32_t)c_done));
    if (i3) gstore4(&C.link[(par * 4 + 3) * N + t], slot_encode(s_link[par][3][j], (uint32_t)c_done));
  }
  if (threadIdx.x == 0) st_coh(&C.flags[patch * FLAG_STRIDE], c_done);
  flush_counters(acc, L, C, patch, c0, c_done);
#undef GEO
#undef GEO_BIT
#undef EDGE_IN
#undef EDGE_OUT
}

// ---- small utility kernels (no memsets: these also record safely into graphs) -----------------
__global__ void fill_i32(int32_t* p, int32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_u64(unsigned long long* p, unsigned long long v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void set_stop(ChipDev* d, int stop) { d->stop = stop; }
// Launch tables are written on the device from a list of chips passed by value (no host
// staging buffer; a table upload is then one small kernel, also inside a captured graph).
constexpr int LIST_CHIPS = 96;  // chips per list (kernel arguments stay well under 4 KB)
struct ChipList {
  int32_t count;
  int32_t first[LIST_CHIPS];  // first table entry of each chip
  int32_t stop[LIST_CHIPS];   // cycle each chip stops at (-1: the chip's own descriptor says)
  ChipDev* chip[LIST_CHIPS];
};
// workgroup k writes the entries of chip k: one per patch, in patch order
__global__ void fill_table(LaunchEntry* table, ChipList L) {
  const int k = blockIdx.x;
  if (k >= L.count) return;
  ChipDev* d = L.chip[k];
  const int np = d->n_patches;
  for (int p = threadIdx.x; p < np; p += blockDim.x) table[L.first[k] + p] = LaunchEntry{d, p, L.stop[k]};
}
// out[base + k] = error word of chip k
__global__ void gather_errors(int32_t* out, int base, ChipList L) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L.count) out[base + k] = *L.chip[k]->err;
}
// link slots of a fresh (or reloaded) chip at cycle c: every slot empty; parity c&1 holds the
// inputs of cycle c, the other parity is stamped c-1 so that it cannot pass for cycle c+1
__global__ void init_links(int4* link, int N, int c) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 8 * N; i += gridDim.x * blockDim.x) {
    const int par = i / (4 * N);
    link[i] = slot_encode(make_int4(-1, -1, -1, -1), (uint32_t)(par == (c & 1) ? c : c - 1));
  }
}
// core words of a fresh chip: state idle, bg 0, everything else -1
__global__ void init_core(int4* core, int4* node, int N) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < N; t += gridDim.x * blockDim.x) {
    core[t] = make_int4(CORE_IDLE, -1, -1, -1);
    core[N + t] = make_int4(-1, -1, -1, -1);
    core[2 * N + t] = make_int4(-1, -1, 0, -1);
    core[3 * N + t] = make_int4(-1, 0, -1, 0);  // forced background destination, reply flits received, held op
    core[4 * N + t] = make_int4(-1, -1, 0, 0);  // remote-access target, pending eviction, directory checksum
    core[5 * N + t] = make_int4(-1, -1, -1, -1);  // pending claim, forwarded line and destination, spare
    node[t] = make_int4(-1, -1, -1, 0);
  }
}

int g_last_hip = 0;

}  // namespace

// ============================== host runtime ====================================================
struct sim_chip {
  sim_config cfg;
  ChipDev hd;         // host copy of the device descriptor
  ChipDev* dd;        // device descriptor
  char* base;
  size_t bytes;
  hipStream_t stream;
  int64_t cycle;
  int32_t block, chunk;
  bool fast;               // every patch fits its workgroup: one tile per thread (step_fast)
  bool use_fast;           // allow step_fast (tests compare both kernels)
  bool narrow;             // step_fast's build for workgroups of at most 128 threads (FAST_NARROW)
  LaunchEntry* table_dev;  // max_patches entries
};

// A launch group: consecutive chips whose workgroups are launched together.  Chips cut into
// several patches wait on each other's edges, so a group that holds such a chip is kept within
// the number of workgroups the device can hold at once; groups run one after the other.
struct sim_launch_group {
  int32_t first_chip, n_chips;
  int64_t first_entry, n_entries;
  bool multi;
};

struct sim_group {
  std::vector<sim_chip*> slots;      // chip of each slot; nullptr = free
  int32_t block;                     // threads per workgroup of every launch
  int32_t max_chips;                 // capacity of the caller's workspace
  int64_t max_entries;
  hipStream_t stream;
  LaunchEntry* table_dev;            // workspace: [max_entries] launch entries
  int32_t* err_dev;                  // workspace: [max_chips] error words gathered after a step
  // derived from the members, rebuilt after simb_add / simb_remove
  bool dirty;
  std::vector<int32_t> members;      // occupied slots in table order
  std::vector<int32_t> first_entry;  // first table entry of each member
  std::vector<sim_launch_group> groups;
  bool fast;
  int opt;                           // FAST_* bits some member needs (multi-flit replies, variants, router delay)
  int var;                           // general-kernel build: 1 a variant or router delay > 1, 2 the directory
  int64_t n_entries;
  // one chunk of every launch group, as a graph of kernel nodes (simb_set_graph)
  bool use_graph;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int32_t graph_chunk;
};

namespace {

#define HIPCHECK(x)                          \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) {                  \
      g_last_hip = (int)e_;                  \
      return SIM_EHIP;                       \
    }                                        \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
bool pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }
bool ways_ok(int32_t w) { return w == 1 || w == 2 || w == 4 || w == 8; }

bool config_ok(const sim_config* c) {
  if (!c || c->width < 1 || c->height < 1 || c->width > 2048 || c->height > 2048) return false;
  const int64_t N = (int64_t)c->width * c->height;
  if (N >= (1 << 20)) return false;  // tile indices take 20 bits in a slot word, all ones = empty
  if (!pow2(c->l1_sets) || !ways_ok(c->l1_ways) || !pow2(c->l2_sets) || !ways_ok(c->l2_ways)) return false;
  if (c->l1_lat < 1 || c->mem_lat < 1 || c->shared_lines < 1 || c->private_lines < 0) return false;
  if (c->reply_flits < 0 || c->reply_flits > 16) return false;
  if (c->flags & ~VARIANT_FLAGS) return false;
  if (c->router_delay < 0 || c->router_delay > 8) return false;
  if ((c->flags & SIM_FLAG_LSPD_CENTRAL) && !(c->flags & SIM_FLAG_LSPD)) return false;
  if (c->mig_threshold < 0 || c->mig_threshold > MIG_MAX || (c->mig_threshold && !(c->flags & SIM_FLAG_LSPD))) return false;
  if ((int64_t)c->shared_lines + N * c->private_lines > (int64_t)LINE_MASK + 1) return false;
  return true;
}

struct Layout {
  size_t desc, link, pipe, core, node, loc, l1, l2, l2h, zs, zp, flags, table, stats, err, total;
};
size_t lspd_lines(const sim_config* c) {  // location-array entries (0 without the directory)
  return (c->flags & SIM_FLAG_LSPD) ? (size_t)c->shared_lines + (size_t)c->width * c->height * c->private_lines : 0;
}
int router_delay(const sim_config* c) { return c->router_delay > 0 ? c->router_delay : 1; }
// which build of the general kernel a chip needs: 0 base model, 1 variants / router delay, 2 directory
int kernel_level(const ChipDev& d) { return d.lspd ? 2 : (d.variants != 0 || d.rdelay > 1) ? 1 : 0; }
// OPT bits of the one-tile-per-thread kernel a chip needs
// variants the one-tile-per-thread kernel carries, with any router delay
constexpr int32_t FAST_FLAGS = SIM_FLAG_AGE_DEFLECT | SIM_FLAG_HIT_UNDER_MISS | SIM_FLAG_INJECT_DELAY;
// whether a chip may run on the one-tile-per-thread kernel: any of those variants, and the LSPD
// directory with or without migration
bool fast_model(const sim_config* c) {
  const int32_t carried = FAST_FLAGS | SIM_FLAG_LSPD | SIM_FLAG_LSPD_CENTRAL;
  return (c->flags & VARIANT_FLAGS & ~carried) == 0;
}
// (FAST_WAYS48 is set only when every chip of a launch has the 4/8-way geometry: see batch_kind)
int fast_opt(const ChipDev& d) {
  return (d.lspd ? FAST_LSPD : 0) | (d.mig ? FAST_MIG : 0) | (d.reply_flits > 1 ? FAST_PACKETS : 0) | ((d.variants & FAST_FLAGS) ? FAST_VARIANTS : 0) |
         (d.rdelay > 1 ? FAST_PIPE : 0) | ((d.w1 == 4 && d.w2 == 8) ? FAST_WAYS48 : 0);
}

int max_patches(const sim_config* c) { return (int)std::min<int64_t>(MAX_PATCHES, (int64_t)c->width * c->height); }

Layout layout(const sim_config* c) {
  Layout L{};
  const size_t N = (size_t)c->width * c->height;
  const size_t maxp = (size_t)max_patches(c);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  L.desc = take(sizeof(ChipDev));
  L.link = take(2 * 4 * N * sizeof(int4));
  L.pipe = take((size_t)(router_delay(c) - 1) * 4 * N * sizeof(int4));
  L.core = take(6 * N * sizeof(int4));
  L.loc = take(lspd_lines(c) * sizeof(int32_t));
  L.node = take(N * sizeof(int4));
  L.l1 = take(N * c->l1_sets * c->l1_ways * sizeof(int32_t));
  L.l2 = take(N * c->l2_sets * c->l2_ways * sizeof(int32_t));
  L.l2h = take(c->mig_threshold > 0 ? N * c->l2_sets * c->l2_ways * c->mig_threshold * sizeof(int32_t) : 0);
  L.zs = take((ZIPF_K + 1) * sizeof(uint32_t));
  L.zp = take((ZIPF_K + 1) * sizeof(uint32_t));
  L.flags = take(maxp * FLAG_STRIDE * sizeof(int32_t));
  L.table = take(maxp * sizeof(LaunchEntry));
  L.stats = take(NSTAT * sizeof(unsigned long long));
  L.err = take(256);
  L.total = o;
  return L;
}

// host copies of the slot encoding (dump and load); *age = the flit's deflection count
void host_decode(const int4& w, int32_t* out, int32_t* age) {
  const uint32_t d = (uint32_t)w.x & TILE_BITS_MASK;
  *age = 0;
  if (d == TILE_BITS_MASK) { out[0] = out[1] = out[2] = out[3] = -1; return; }
  out[0] = (int32_t)d; out[1] = w.y; out[2] = (int32_t)((uint32_t)w.z & TILE_BITS_MASK); out[3] = w.w;
  *age = (int32_t)((((uint32_t)w.x >> AGE_SHIFT) & 0xFFu) | ((((uint32_t)w.z >> AGE_SHIFT) & 0xFFu) << 8));
}
int4 host_encode(const int32_t* f, uint32_t stamp, int32_t age) {
  const uint32_t s = (stamp & STAMP_MASK) << STAMP_SHIFT;
  if (f[0] < 0) return make_int4((int)(TILE_BITS_MASK | s), -1, (int)(TILE_BITS_MASK | s), -1);
  const uint32_t lo = ((uint32_t)age & 0xFFu) << AGE_SHIFT, hi = (((uint32_t)age >> 8) & 0xFFu) << AGE_SHIFT;
  return make_int4((int)((uint32_t)f[0] | lo | s), f[1], (int)((uint32_t)f[2] | hi | s), f[3]);
}

int launch_grid_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  if (!n) return SIM_OK;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_i32, dim3(blocks), dim3(256), 0, s, p, v, n);
  HIPCHECK(hipGetLastError());
  return SIM_OK;
}
int launch_grid_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s) {
  if (!n) return SIM_OK;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_u64, dim3(blocks), dim3(256), 0, s, p, v, n);
  HIPCHECK(hipGetLastError());
  return SIM_OK;
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    cus = prop.multiProcessorCount;
  }
  return cus;
}

// the one-tile-per-thread kernel's build for the given OPT bits (FAST_*)
template <bool MULTI, bool DIGEST>
const void* fast_build(int opt) {
  if ((opt & FAST_NARROW) && (opt & ~(FAST_NARROW | FAST_WAYS48)) == 0)
    return (opt & FAST_WAYS48) ? reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, FAST_NARROW | FAST_WAYS48>)
                               : reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, FAST_NARROW>);
  if ((opt & (FAST_MIG | 7)) == FAST_MIG && (opt & FAST_WAYS48))
    return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, FAST_MIG | FAST_LSPD | FAST_WAYS48>);
  if (opt & FAST_MIG) return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, FAST_MIG | FAST_LSPD | 7>);
  if ((opt & (FAST_LSPD | 7)) == FAST_LSPD && (opt & FAST_WAYS48))
    return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, FAST_LSPD | FAST_WAYS48>);
  if (opt & FAST_LSPD) return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, FAST_LSPD | 7>);
  switch (opt & 15) {
    case 0: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 0>);
    case 1: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 1>);
    case 2: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 2>);
    case 3: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 3>);
    case 4: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 4>);
    case 5: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 5>);
    case 6: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 6>);
    case 7: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 7>);
    case 8: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 8>);
    case 9: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 9>);
    case 10: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 10>);
    case 11: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 11>);
    case 12: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 12>);
    case 13: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 13>);
    case 14: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 14>);
    default: return reinterpret_cast<const void*>(step_fast<MULTI, DIGEST, 15>);
  }
}
const void* multi_kernel(bool fast, bool digest = false, int opt = 0, int var = 0) {
  if (!fast) return var == 2 ? reinterpret_cast<const void*>(step_kernel<true, 2>)
                    : var == 1 ? reinterpret_cast<const void*>(step_kernel<true, 1>)
                               : reinterpret_cast<const void*>(step_kernel<true, 0>);
  return digest ? fast_build<true, true>(opt) : fast_build<true, false>(opt);
}
// how many workgroups of `block` threads of the multi-patch kernel of one kind (the general
// kernel's build `var`, or the one-tile-per-thread build for OPT bits `opt`) the device holds at
// once; with `digests`, the lower of its builds with and without them, as a single chip may
// ask for either (batches launch the build without); 0 if the runtime cannot tell
int resident_limit(int block, bool fast, int opt, int var, bool digests) {
  int lo = INT_MAX;
  for (int dig = 0; dig < (fast && digests ? 2 : 1); ++dig) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, multi_kernel(fast, dig != 0, opt, var), block, 0) !=
        hipSuccess)
      return 0;
    lo = std::min(lo, per_cu);
  }
  return lo * device_cus();
}
// Whether a chip cut into np patches of `block` threads can be resident at once on the kernel it
// would run (fast: one tile per thread); when the usual build cannot hold them, a base-model
// chip of workgroups of at most 128 threads may use the narrow build (*narrow), which can.
int fit_mapping(const sim_chip* h, int np, int block, bool fast, bool* narrow) {
  *narrow = false;
  if (np <= 1) return SIM_OK;
  const int opt = fast_opt(h->hd), var = kernel_level(h->hd);
  if (np <= resident_limit(block, fast, opt, var, true)) return SIM_OK;
  if (fast && block <= 128 && (opt & ~FAST_WAYS48) == 0 && np <= resident_limit(block, true, opt | FAST_NARROW, var, true)) {
    *narrow = true;
    return SIM_OK;
  }
  return SIM_EINVAL;
}

int upload_desc(sim_chip* h) {
  HIPCHECK(hipMemcpyAsync(h->dd, &h->hd, sizeof(ChipDev), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

static int block_for(int tiles) { return tiles <= 64 ? 64 : tiles <= 128 ? 128 : tiles <= 192 ? 192 : 256; }

// Default mapping: one workgroup for small chips; otherwise one tile per thread in strips of one
// row per workgroup of one or two waves (a row cut into equal strips of at most 128 tiles; up to
// 256 tiles of whole rows below 64 columns), as long as every strip can be resident at once on
// the chip's own build; otherwise square-ish patches, about one per compute unit.
void default_mapping(const sim_chip* hc, int32_t* pw, int32_t* ph, int32_t* block) {
  const sim_config* c = &hc->cfg;
  const int N = c->width * c->height;
  if (N <= 1024) {
    *pw = c->width;
    *ph = c->height;
    *block = N <= 64 ? 64 : 256;
    return;
  }
  {
    const int k = (c->width + 127) / 128;  // strips per row
    const int w = (c->width + k - 1) / k;
    const int h = c->width < 64 ? std::min(c->height, 256 / c->width) : 1;
    const int np = ((c->width + w - 1) / w) * ((c->height + h - 1) / h);
    bool narrow = false;
    if (np <= hc->hd.max_patches && fit_mapping(hc, np, block_for(w * h), hc->use_fast, &narrow) == SIM_OK) {
      *pw = w;
      *ph = h;
      *block = block_for(w * h);
      return;
    }
  }
  const int target = device_cus();
  int side = 1;
  while ((int64_t)((c->width + side - 1) / side) * ((c->height + side - 1) / side) > target) side++;
  *pw = std::min(side, c->width);
  *ph = std::min(side, c->height);
  *block = block_for((*pw) * (*ph));
}

int apply_mapping(sim_chip* h, int32_t pw, int32_t ph, int32_t block) {
  if (pw < 1 || ph < 1 || block < 64 || block > 256 || block % 64) return SIM_EINVAL;
  pw = std::min(pw, h->cfg.width);
  ph = std::min(ph, h->cfg.height);
  const int pgx = (h->cfg.width + pw - 1) / pw, pgy = (h->cfg.height + ph - 1) / ph;
  const int np = pgx * pgy;
  if (np > h->hd.max_patches) return SIM_EINVAL;
  bool narrow = false;
  if (fit_mapping(h, np, block, pw * ph <= block && h->use_fast, &narrow)) return SIM_EINVAL;
  h->narrow = narrow;
  h->hd.pw = pw;
  h->hd.ph = ph;
  h->hd.pgx = pgx;
  h->hd.pgy = pgy;
  h->hd.n_patches = np;
  h->block = block;
  h->fast = pw * ph <= block;
  // every patch's flag records the chip's cycle
  int rc = launch_grid_fill_i32(h->hd.flags, (int32_t)h->cycle, (size_t)h->hd.max_patches * FLAG_STRIDE, h->stream);
  if (rc) return rc;
  HIPCHECK(hipMemcpyAsync(h->dd, &h->hd, sizeof(ChipDev), hipMemcpyHostToDevice, h->stream));
  ChipList one{};
  one.count = 1;
  one.first[0] = 0;
  one.stop[0] = -1;
  one.chip[0] = h->dd;
  hipLaunchKernelGGL(fill_table, dim3(1), dim3(256), 0, h->stream, h->table_dev, one);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

// fast: every patch has at most `block` tiles (one tile per thread: step_fast)
// opt: FAST_PACKETS when some chip of the table has multi-flit replies (the kernel then reads
// each chip's count), FAST_VARIANTS when some chip has a variant the kernel carries, FAST_PIPE
// when some chip has a router delay
// checking: run the checking build of the one-tile-per-thread kernel even without digests (the
// watchdog's checks live there)
int launch_entries(const LaunchEntry* table, int64_t n, bool multi, bool fast, int block, int chunk,
                   unsigned long long* digests, int digest_base, hipStream_t s, int opt, int var, bool checking = false) {
  if (n <= 0) return SIM_OK;
  const bool chk = digests != nullptr || checking;
  if (multi) {
    void* args[] = {(void*)&table, (void*)&chunk, (void*)&digests, (void*)&digest_base};
    HIPCHECK(hipLaunchCooperativeKernel(multi_kernel(fast, chk, opt, var), dim3((unsigned)n), dim3(block), args, 0, s));
  } else if (fast) {
    void* args[] = {(void*)&table, (void*)&chunk, (void*)&digests, (void*)&digest_base};
    HIPCHECK(hipLaunchKernel(chk ? fast_build<false, true>(opt) : fast_build<false, false>(opt), dim3((unsigned)n),
                             dim3(block), args, 0, s));
  } else {
    const dim3 g((unsigned)n), b(block);
    if (var == 2) hipLaunchKernelGGL((step_kernel<false, 2>), g, b, 0, s, table, chunk, digests, digest_base);
    else if (var == 1) hipLaunchKernelGGL((step_kernel<false, 1>), g, b, 0, s, table, chunk, digests, digest_base);
    else hipLaunchKernelGGL((step_kernel<false, 0>), g, b, 0, s, table, chunk, digests, digest_base);
    HIPCHECK(hipGetLastError());
  }
  return SIM_OK;
}

}  // namespace

extern "C" {

const char* sim_strerror(int code) {
  switch (code) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument or shape";
    case SIM_ENOMEM: return "device buffer too small";
    case SIM_EHIP: return "HIP runtime error";
    case SIM_EINVARIANT: return "invariant violated";
    case SIM_EBUSY: return "busy";
    case SIM_EHANG: return "cross-workgroup wait timed out";
    case SIM_ELIVELOCK: return "a flit outlived the watchdog's age bound";
    default: return "unknown error";
  }
}

int sim_last_hip_error(void) { return g_last_hip; }

int sim_div_constants(int32_t width, int32_t tiles, uint32_t* out) {
  if (!out || width < 1 || tiles < 1) return SIM_EINVAL;
  // tile / W = umulhi(tile, ceil(2^32 / W)) for tile < 2^20
  out[0] = width > 1 ? (uint32_t)((0x100000000ull + (uint64_t)width - 1) / (uint64_t)width) : 0u;
  out[1] = 0;
  if (tiles > 1) {
    // line / N = umulhi(line, ceil(2^(32+k) / N)) >> k for line < 2^30, k = floor(log2 N) - 1
    const int k = 30 - __builtin_clz((unsigned)tiles);
    out[2] = (uint32_t)(((1ull << (32 + k)) + (uint64_t)tiles - 1) / (uint64_t)tiles);
    out[3] = (uint32_t)k;
  } else {
    out[2] = 0;
    out[3] = 0;
  }
  return SIM_OK;
}

size_t sim_state_bytes(const sim_config* cfg) {
  if (!config_ok(cfg)) return 0;
  return layout(cfg).total;
}

int sim_create(const sim_config* cfg, const uint32_t* zs, const uint32_t* zp, int32_t zk, void* dev_mem, size_t bytes,
               void* stream, sim_t** out) {
  if (!out) return SIM_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg) || !zs || zk != ZIPF_K || (cfg->private_lines > 0 && !zp) || !dev_mem) return SIM_EINVAL;
  // a quantile table must not decrease and must stay inside its region (ranks below its size)
  auto table_ok = [](const uint32_t* q, int32_t lines) {
    for (int i = 0; i < ZIPF_K; ++i)
      if (q[i] > q[i + 1]) return false;
    return q[ZIPF_K] <= (uint32_t)lines;
  };
  if (!table_ok(zs, cfg->shared_lines) || (cfg->private_lines > 0 && !table_ok(zp, cfg->private_lines))) return SIM_EINVAL;
  const Layout Lo = layout(cfg);
  if (bytes < Lo.total) return SIM_ENOMEM;
  if (reinterpret_cast<uintptr_t>(dev_mem) % 256) return SIM_EINVAL;
  sim_chip* h = new (std::nothrow) sim_chip();
  if (!h) return SIM_ENOMEM;
  h->cfg = *cfg;
  h->base = static_cast<char*>(dev_mem);
  h->bytes = bytes;
  h->stream = static_cast<hipStream_t>(stream);
  h->cycle = 0;
  h->chunk = 1000;
  h->use_fast = fast_model(cfg);
  const int N = cfg->width * cfg->height;
  ChipDev& d = h->hd;
  d.W = cfg->width;
  d.H = cfg->height;
  d.N = N;
  d.key0 = cfg->seed_lo;
  d.key1 = cfg->seed_hi;
  d.op_thr = cfg->op_thr;
  d.shared_thr = cfg->shared_thr;
  d.bg_thr = cfg->bg_thr;
  {
    uint32_t dc[4];
    sim_div_constants(cfg->width, N, dc);
    d.w_magic = dc[0];
    d.n_magic = dc[2];
    d.n_shift = dc[3];
  }
  d.spin_limit = SPIN_LIMIT;
  d.watch_age = 0;
  d.halt_patch = -1;
  d.halt_cycle = 0;
  d.w1_shift = __builtin_ctz((unsigned)cfg->l1_ways);
  d.w2_shift = __builtin_ctz((unsigned)cfg->l2_ways);
  d.s1 = cfg->l1_sets;
  d.w1 = cfg->l1_ways;
  d.s2 = cfg->l2_sets;
  d.w2 = cfg->l2_ways;
  d.l1_lat = cfg->l1_lat;
  d.mem_lat = cfg->mem_lat;
  d.reply_flits = cfg->reply_flits > 0 ? cfg->reply_flits : 1;
  d.variants = cfg->flags;
  d.inj_delay = (cfg->flags & SIM_FLAG_INJECT_DELAY) ? 1 : 0;
  d.rdelay = router_delay(cfg);
  d.lspd = (cfg->flags & SIM_FLAG_LSPD) ? ((cfg->flags & SIM_FLAG_LSPD_CENTRAL) ? 2 : 1) : 0;
  d.dir_center = (cfg->height / 2) * cfg->width + cfg->width / 2;
  d.lines = (int32_t)lspd_lines(cfg);
  d.mig = cfg->mig_threshold;
  d.shared_lines = cfg->shared_lines;
  d.private_lines = cfg->private_lines;
  d.stop = 0;
  d.max_patches = max_patches(cfg);
  d.link = reinterpret_cast<int4*>(h->base + Lo.link);
  d.pipe = reinterpret_cast<int4*>(h->base + Lo.pipe);
  d.loc = reinterpret_cast<int32_t*>(h->base + Lo.loc);
  d.l2h = reinterpret_cast<int32_t*>(h->base + Lo.l2h);
  d.core = reinterpret_cast<int4*>(h->base + Lo.core);
  d.node = reinterpret_cast<int4*>(h->base + Lo.node);
  d.l1 = reinterpret_cast<int32_t*>(h->base + Lo.l1);
  d.l2 = reinterpret_cast<int32_t*>(h->base + Lo.l2);
  d.zs = reinterpret_cast<const uint32_t*>(h->base + Lo.zs);
  d.zp = reinterpret_cast<const uint32_t*>(h->base + Lo.zp);
  d.flags = reinterpret_cast<int32_t*>(h->base + Lo.flags);
  d.stats = reinterpret_cast<unsigned long long*>(h->base + Lo.stats);
  d.err = reinterpret_cast<int32_t*>(h->base + Lo.err);
  h->dd = reinterpret_cast<ChipDev*>(h->base + Lo.desc);
  h->table_dev = reinterpret_cast<LaunchEntry*>(h->base + Lo.table);
  int rc = SIM_OK;
  auto fail = [&](int code) { delete h; return code; };
  hipLaunchKernelGGL(init_links, dim3(std::min((8 * N + 255) / 256, 4096)), dim3(256), 0, h->stream, d.link, N, 0);
  if (hipGetLastError() != hipSuccess) return fail(SIM_EHIP);
  hipLaunchKernelGGL(init_core, dim3(std::min((N + 255) / 256, 4096)), dim3(256), 0, h->stream, d.core, d.node, N);
  if (hipGetLastError() != hipSuccess) return fail(SIM_EHIP);
  if ((rc = launch_grid_fill_i32(reinterpret_cast<int32_t*>(d.pipe), -1, (size_t)(d.rdelay - 1) * 4 * N * 4, h->stream)))
    return fail(rc);
  if ((rc = launch_grid_fill_i32(d.loc, -1, lspd_lines(cfg), h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_i32(d.l2h, -1, cfg->mig_threshold > 0 ? (size_t)N * cfg->l2_sets * cfg->l2_ways * cfg->mig_threshold : 0, h->stream)))
    return fail(rc);
  if ((rc = launch_grid_fill_i32(d.l1, -1, (size_t)N * cfg->l1_sets * cfg->l1_ways, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_i32(d.l2, -1, (size_t)N * cfg->l2_sets * cfg->l2_ways, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_u64(d.stats, 0, NSTAT, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_i32(d.err, 0, 1, h->stream))) return fail(rc);
  if (hipMemcpyAsync(const_cast<uint32_t*>(d.zs), zs, (ZIPF_K + 1) * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(SIM_EHIP);
  if (hipMemcpyAsync(const_cast<uint32_t*>(d.zp), zp ? zp : zs, (ZIPF_K + 1) * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(SIM_EHIP);
  int32_t pw, ph, block;
  default_mapping(h, &pw, &ph, &block);
  if ((rc = apply_mapping(h, pw, ph, block))) return fail(rc);
  *out = h;
  return SIM_OK;
}

int64_t sim_cycle(const sim_t* h) { return h ? h->cycle : -1; }

int sim_set_launch(sim_t* h, int32_t pw, int32_t ph, int32_t block, int32_t chunk) {
  if (!h) return SIM_EINVAL;
  if (chunk < 0) return SIM_EINVAL;
  if (chunk) h->chunk = chunk;
  return apply_mapping(h, pw ? pw : h->hd.pw, ph ? ph : h->hd.ph, block ? block : h->block);
}

int sim_set_kernel(sim_t* h, int32_t generic_only) {
  if (!h) return SIM_EINVAL;
  const bool use_fast = !generic_only && fast_model(&h->cfg);
  const int np = h->hd.n_patches;
  bool narrow = false;
  if (fit_mapping(h, np, h->block, h->fast && use_fast, &narrow)) return SIM_EINVAL;
  h->use_fast = use_fast;
  h->narrow = narrow;
  return SIM_OK;
}

int sim_get_launch(const sim_t* h, int32_t* pw, int32_t* ph, int32_t* block, int32_t* chunk) {
  if (!h) return SIM_EINVAL;
  if (pw) *pw = h->hd.pw;
  if (ph) *ph = h->hd.ph;
  if (block) *block = h->block;
  if (chunk) *chunk = h->chunk;
  return SIM_OK;
}

static int check_err(sim_t* h) {
  int32_t err = 0;
  HIPCHECK(hipMemcpyAsync(&err, h->hd.err, sizeof err, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return err == 0 ? SIM_OK : err == 1 ? SIM_EHANG : err == ERR_WATCHDOG ? SIM_ELIVELOCK : SIM_EINVARIANT;
}

int sim_step(sim_t* h, int64_t n, uint64_t* dev_digests) {
  if (!h || n < 0 || h->cycle + n > 0x7FFFFFFFll) return SIM_EINVAL;
  if (!n) return SIM_OK;
  const int np = h->hd.n_patches;
  hipLaunchKernelGGL(set_stop, dim3(1), dim3(1), 0, h->stream, h->dd, (int)(h->cycle + n));
  HIPCHECK(hipGetLastError());
  unsigned long long* dig = reinterpret_cast<unsigned long long*>(dev_digests);
  if (dig) {
    int rc = launch_grid_fill_u64(dig, 0, (size_t)n, h->stream);
    if (rc) return rc;
  }
  const int launches = (int)((n + h->chunk - 1) / h->chunk);
  for (int i = 0; i < launches; ++i) {
    int rc = launch_entries(h->table_dev, np, np > 1, h->fast && h->use_fast, h->block, h->chunk, dig, (int)h->cycle, h->stream,
                            fast_opt(h->hd) | (h->narrow ? FAST_NARROW : 0), kernel_level(h->hd), h->hd.watch_age > 0);
    if (rc) return rc;
  }
  h->cycle += n;
  return SIM_OK;
}

int sim_sync(sim_t* h) {
  if (!h) return SIM_EINVAL;
  return check_err(h);
}

int sim_stats(sim_t* h, sim_stats_t* out) {
  if (!h || !out) return SIM_EINVAL;
  HIPCHECK(hipMemcpyAsync(out->v, h->hd.stats, sizeof out->v, hipMemcpyDeviceToHost, h->stream));
  return check_err(h);
}

size_t sim_dump_words(const sim_t* h) {
  if (!h) return 0;
  const size_t N = (size_t)h->hd.N;
  return 16 + N * 16 + N * CORE_RECORD + N * h->hd.s1 * h->hd.w1 + N * h->hd.s2 * h->hd.w2 + 2 * NSTAT + N * 4 +
         (size_t)(h->hd.rdelay - 1) * N * 20 + (size_t)h->hd.lines + (size_t)N * h->hd.s2 * h->hd.w2 * h->hd.mig;
}

int sim_dump(sim_t* h, int32_t* buf, size_t words) {
  if (!h || !buf || words < sim_dump_words(h)) return SIM_EINVAL;
  const size_t N = (size_t)h->hd.N;
  const int par = (int)(h->cycle & 1);
  std::vector<int4> link(4 * N), core(6 * N), node(N);
  HIPCHECK(hipMemcpyAsync(link.data(), h->hd.link + (size_t)par * 4 * N, 4 * N * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(core.data(), h->hd.core, 6 * N * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(node.data(), h->hd.node, N * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
  size_t o = 16;
  const size_t n1 = N * h->hd.s1 * h->hd.w1, n2 = N * h->hd.s2 * h->hd.w2;
  int32_t* l1 = buf + 16 + N * (16 + CORE_RECORD);
  int32_t* l2 = l1 + n1;
  HIPCHECK(hipMemcpyAsync(l1, h->hd.l1, n1 * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(l2, h->hd.l2, n2 * 4, hipMemcpyDeviceToHost, h->stream));
  unsigned long long st[NSTAT];
  HIPCHECK(hipMemcpyAsync(st, h->hd.stats, sizeof st, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  const int32_t hdr[16] = {0x4E4F4353, DUMP_VERSION, h->hd.W, h->hd.H, (int32_t)(uint32_t)h->cycle,
                           (int32_t)(h->cycle >> 32), h->hd.s1, h->hd.w1, h->hd.s2, h->hd.w2, h->hd.reply_flits,
                           CORE_RECORD, h->hd.variants, h->hd.rdelay, h->hd.lspd, h->hd.mig};
  std::memcpy(buf, hdr, sizeof hdr);
  int32_t* ages = buf + 16 + N * (16 + CORE_RECORD) + n1 + n2 + 2 * NSTAT;
  for (size_t t = 0; t < N; ++t)
    for (int p = 0; p < 4; ++p) host_decode(link[p * N + t], buf + o + t * 16 + p * 4, ages + t * 4 + p);
  o += N * 16;
  for (size_t t = 0; t < N; ++t) {
    const int4 k0 = core[t], k1 = core[N + t], k2 = core[2 * N + t], k3 = core[3 * N + t], k4 = core[4 * N + t];
    const int4 k5 = core[5 * N + t], nd = node[t];
    const int32_t rec[CORE_RECORD] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w, k2.x, k2.y, k2.z, nd.x, nd.y, nd.z,
                                      k2.w, k3.x, k3.y, nd.w, k3.z, k3.w, k4.x, k4.y, k4.z, k4.w, k5.x, k5.y, k5.z, k5.w};
    std::memcpy(buf + o + t * CORE_RECORD, rec, sizeof rec);
  }
  o += N * CORE_RECORD + n1 + n2;
  for (int i = 0; i < NSTAT; ++i) {
    buf[o++] = (int32_t)(uint32_t)st[i];
    buf[o++] = (int32_t)(st[i] >> 32);
  }
  o += N * 4;  // slot deflection counts, written above
  const int D = h->hd.rdelay;
  if (D > 1) {  // pipeline stages k = 1..D-1: ring entry (cycle + k - 1) mod (D-1)
    std::vector<int4> pipe((size_t)(D - 1) * 4 * N);
    HIPCHECK(hipMemcpyAsync(pipe.data(), h->hd.pipe, pipe.size() * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    int32_t* pa = buf + o + (size_t)(D - 1) * N * 16;
    for (int k = 1; k < D; ++k) {
      const size_t ring = (size_t)((h->cycle + k - 1) % (D - 1));
      for (size_t t = 0; t < N; ++t)
        for (int p = 0; p < 4; ++p)
          host_decode(pipe[(ring * 4 + p) * N + t], buf + o + ((size_t)(k - 1) * N + t) * 16 + p * 4,
                      pa + ((size_t)(k - 1) * N + t) * 4 + p);
    }
  }
  o += (size_t)(D - 1) * N * 20;
  if (h->hd.lines) {  // LSPD location array
    HIPCHECK(hipMemcpyAsync(buf + o, h->hd.loc, (size_t)h->hd.lines * 4, hipMemcpyDeviceToHost, h->stream));
    o += (size_t)h->hd.lines;
  }
  if (h->hd.mig)  // migration: the last `mig` accessors of every L2 way, most recent first
    HIPCHECK(hipMemcpyAsync(buf + o, h->hd.l2h, N * h->hd.s2 * h->hd.w2 * h->hd.mig * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

int sim_load(sim_t* h, const int32_t* buf, size_t words) {
  if (!h || !buf || words < sim_dump_words(h)) return SIM_EINVAL;
  if (buf[0] != 0x4E4F4353 || buf[1] != DUMP_VERSION || buf[2] != h->hd.W || buf[3] != h->hd.H ||
      buf[6] != h->hd.s1 || buf[7] != h->hd.w1 || buf[8] != h->hd.s2 || buf[9] != h->hd.w2 ||
      buf[10] != h->hd.reply_flits || buf[11] != CORE_RECORD || buf[12] != h->hd.variants ||
      buf[13] != h->hd.rdelay || buf[14] != h->hd.lspd || buf[15] != h->hd.mig)
    return SIM_EINVAL;
  const size_t N = (size_t)h->hd.N;
  const size_t n1 = N * h->hd.s1 * h->hd.w1, n2 = N * h->hd.s2 * h->hd.w2;
  const int32_t* ages = buf + 16 + N * (16 + CORE_RECORD) + n1 + n2 + 2 * NSTAT;
  const bool aged = h->hd.variants & SIM_FLAG_AGE_DEFLECT;
  const int64_t cyc = (int64_t)(((uint64_t)(uint32_t)buf[5] << 32) | (uint32_t)buf[4]);
  if (cyc < 0 || cyc > 0x7FFFFFFF) return SIM_EINVAL;
  std::vector<int4> link(4 * N), core(6 * N), node(N);
  size_t o = 16;
  for (size_t t = 0; t < N; ++t)
    for (int p = 0; p < 4; ++p) {
      const int32_t* w = buf + o + t * 16 + p * 4;
      const int32_t a = ages[t * 4 + p];
      if (w[0] >= (int32_t)N || w[2] >= (int32_t)N || (w[0] >= 0 && w[2] < 0)) return SIM_EINVAL;
      if (a < 0 || a > AGE_MAX || (a && (!aged || w[0] < 0))) return SIM_EINVAL;
      link[p * N + t] = host_encode(w, (uint32_t)cyc, a);
    }
  o += N * 16;
  for (size_t t = 0; t < N; ++t) {
    const int32_t* r = buf + o + t * CORE_RECORD;
    core[t] = make_int4(r[0], r[1], r[2], r[3]);
    core[N + t] = make_int4(r[4], r[5], r[6], r[7]);
    core[2 * N + t] = make_int4(r[8], r[9], r[10], r[14]);
    // a held op exists only with hit under miss (the base kernel keeps none)
    if (r[18] >= 0 && !(h->hd.variants & SIM_FLAG_HIT_UNDER_MISS)) return SIM_EINVAL;
    // the directory's words: a target and a pending eviction only with LSPD
    if (!h->hd.lspd && (r[20] != -1 || r[21] != -1 || r[22] != 0 || r[23] != 0)) return SIM_EINVAL;
    if (r[20] < -1 || r[20] >= (int32_t)N || r[21] < -1 || r[21] >= h->hd.lines) return SIM_EINVAL;
    // migration words: a claim and a forwarding pointer only with migration
    if (!h->hd.mig && (r[24] != -1 || r[25] != -1 || r[26] != -1 || r[27] != -1)) return SIM_EINVAL;
    // (a forwarding destination carries MIG_TRANSIT while its block is on the way)
    const int32_t fwd = r[26] >= 0 ? (r[26] & ~MIG_TRANSIT) : r[26];
    if (r[24] < -1 || r[24] >= h->hd.lines || r[25] < -1 || r[25] >= h->hd.lines || fwd < -1 ||
        fwd >= (int32_t)N || r[27] < -1 || r[27] >= (int32_t)N)
      return SIM_EINVAL;
    core[3 * N + t] = make_int4(r[15], r[16], r[18], r[19]);
    core[4 * N + t] = make_int4(r[20], r[21], r[22], r[23]);
    core[5 * N + t] = make_int4(r[24], r[25], r[26], r[27]);
    node[t] = make_int4(r[11], r[12], r[13], r[17]);
  }
  o += N * CORE_RECORD;
  // pipeline stages (router delay > 1), validated before anything is copied: stage k goes to
  // ring entry (cycle + k - 1) mod (D-1)
  const int D = h->hd.rdelay;
  std::vector<int4> pipe((size_t)(D - 1) * 4 * N);
  {
    const int32_t* pw = buf + 16 + N * (16 + CORE_RECORD) + n1 + n2 + 2 * NSTAT + N * 4;
    const int32_t* pa = pw + (size_t)(D - 1) * N * 16;
    for (int k = 1; k < D; ++k) {
      const size_t ring = (size_t)((cyc + k - 1) % (D - 1));
      for (size_t t = 0; t < N; ++t)
        for (int p = 0; p < 4; ++p) {
          const int32_t* w = pw + ((size_t)(k - 1) * N + t) * 16 + p * 4;
          const int32_t a = pa[((size_t)(k - 1) * N + t) * 4 + p];
          if (w[0] >= (int32_t)N || w[2] >= (int32_t)N || (w[0] >= 0 && w[2] < 0)) return SIM_EINVAL;
          if (a < 0 || a > AGE_MAX || (a && (!aged || w[0] < 0))) return SIM_EINVAL;
          pipe[(ring * 4 + p) * N + t] = host_encode(w, 0u, a);
        }
    }
  }
  // LSPD location array: owners in range
  const int32_t* locw = buf + 16 + N * (16 + CORE_RECORD) + n1 + n2 + 2 * NSTAT + N * 4 + (size_t)(D - 1) * N * 20;
  for (int32_t i = 0; i < h->hd.lines; ++i)
    if (locw[i] < -1 || locw[i] >= (int32_t)N) return SIM_EINVAL;
  const int par = (int)(cyc & 1);
  HIPCHECK(hipMemcpyAsync(h->hd.link + (size_t)par * 4 * N, link.data(), 4 * N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  // the other parity: empty, stamped cyc-1 (it is rewritten during cycle cyc)
  std::vector<int4> other(4 * N, host_encode(std::vector<int32_t>{-1, -1, -1, -1}.data(), (uint32_t)(cyc - 1), 0));
  HIPCHECK(hipMemcpyAsync(h->hd.link + (size_t)(par ^ 1) * 4 * N, other.data(), 4 * N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  int rc = SIM_OK;
  HIPCHECK(hipMemcpyAsync(h->hd.core, core.data(), 6 * N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hd.node, node.data(), N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hd.l1, buf + o, n1 * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hd.l2, buf + o + n1, n2 * 4, hipMemcpyHostToDevice, h->stream));
  o += n1 + n2;
  unsigned long long st[NSTAT];
  for (int i = 0; i < NSTAT; ++i) st[i] = (unsigned long long)(uint32_t)buf[o + 2 * i] | ((unsigned long long)(uint32_t)buf[o + 2 * i + 1] << 32);
  HIPCHECK(hipMemcpyAsync(h->hd.stats, st, sizeof st, hipMemcpyHostToDevice, h->stream));
  if (D > 1) HIPCHECK(hipMemcpyAsync(h->hd.pipe, pipe.data(), pipe.size() * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  if (h->hd.lines) HIPCHECK(hipMemcpyAsync(h->hd.loc, locw, (size_t)h->hd.lines * 4, hipMemcpyHostToDevice, h->stream));
  if (h->hd.mig)
    HIPCHECK(hipMemcpyAsync(h->hd.l2h, locw + h->hd.lines, N * h->hd.s2 * h->hd.w2 * h->hd.mig * 4, hipMemcpyHostToDevice, h->stream));
  h->cycle = cyc;
  if ((rc = launch_grid_fill_i32(h->hd.flags, (int32_t)cyc, (size_t)h->hd.max_patches * FLAG_STRIDE, h->stream))) return rc;
  // the restored state is whole: an error recorded for the state it replaces no longer applies
  if ((rc = launch_grid_fill_i32(h->hd.err, 0, 1, h->stream))) return rc;
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

int sim_force_op(sim_t* h, int32_t tile, int32_t line) {
  if (!h || tile < 0 || tile >= h->hd.N || line < 0 || line > LINE_MASK) return SIM_EINVAL;
  int4 k2;
  HIPCHECK(hipMemcpyAsync(&k2, h->hd.core + 2 * (size_t)h->hd.N + tile, sizeof k2, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  k2.w = line;
  HIPCHECK(hipMemcpyAsync(h->hd.core + 2 * (size_t)h->hd.N + tile, &k2, sizeof k2, hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

int sim_force_bg(sim_t* h, int32_t tile, int32_t dst) {
  if (!h || tile < 0 || tile >= h->hd.N || dst < 0 || dst >= h->hd.N || dst == tile) return SIM_EINVAL;
  const int32_t d = dst;  // the forced destination word only (the reply-flit count beside it stays)
  HIPCHECK(hipMemcpyAsync(reinterpret_cast<int32_t*>(h->hd.core + 3 * (size_t)h->hd.N + tile), &d, sizeof d,
                          hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

int sim_force_hang(sim_t* h, int32_t patch, int32_t cycle, int32_t polls) {
  if (!h || polls < 0 || patch < -1 || patch >= h->hd.n_patches || cycle < 0) return SIM_EINVAL;
  h->hd.spin_limit = polls ? polls : SPIN_LIMIT;
  h->hd.halt_patch = patch;
  h->hd.halt_cycle = cycle;
  return upload_desc(h);
}

int sim_set_watchdog(sim_t* h, int32_t max_age) {
  if (!h || max_age < 0) return SIM_EINVAL;
  h->hd.watch_age = max_age;
  return upload_desc(h);
}

int sim_set_rates(sim_t* h, uint32_t op_thr, uint32_t bg_thr) {
  if (!h) return SIM_EINVAL;
  h->hd.op_thr = op_thr;
  h->hd.bg_thr = bg_thr;
  h->cfg.op_thr = op_thr;
  h->cfg.bg_thr = bg_thr;
  return upload_desc(h);
}

int sim_destroy(sim_t* h) {
  if (!h) return SIM_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return SIM_OK;
}

// ---- batches ------------------------------------------------------------------------------------
size_t simb_state_bytes(int32_t max_chips, int64_t max_patches) {
  if (max_chips < 1 || max_patches < max_chips || max_patches > 0x7FFFFFFF) return 0;
  return align_up((size_t)max_patches * sizeof(LaunchEntry), 256) + align_up((size_t)max_chips * sizeof(int32_t), 256);
}

}  // extern "C"

namespace {

// The kernel that runs a launch group of a batch.
const void* batch_kernel(bool multi, bool fast, int opt, int var) {
  if (multi) return multi_kernel(fast, false, opt, var);
  if (fast) return fast_build<false, false>(opt);
  return var == 2 ? reinterpret_cast<const void*>(step_kernel<false, 2>)
         : var == 1 ? reinterpret_cast<const void*>(step_kernel<false, 1>)
                    : reinterpret_cast<const void*>(step_kernel<false, 0>);
}

// Which kernel a set of chips runs on in a batch of `block`-thread workgroups.
struct BatchKind {
  bool fast, multi;
  int opt, var;
};
template <class ChipAt>
BatchKind batch_kind(ChipAt chip_at, int n, int block) {
  BatchKind k{true, false, 0, 0};
  bool w48 = true;  // every chip has the 4/8-way geometry
  for (int i = 0; i < n; ++i) {
    const sim_chip* h = chip_at(i);
    k.fast = k.fast && h->use_fast && h->hd.pw * h->hd.ph <= block;
    k.multi = k.multi || h->hd.n_patches > 1;
    const int o = fast_opt(h->hd);
    k.opt |= o & ~FAST_WAYS48;
    w48 = w48 && (o & FAST_WAYS48);
    k.var = std::max(k.var, kernel_level(h->hd));
  }
  if (w48 && n > 0) k.opt |= FAST_WAYS48;
  return k;
}

// Cuts chips 0..n-1 (in order) into launch groups: a group that holds a chip of several
// patches stays within `limit` workgroups, the number the device holds at once.  Calls
// emit(group) for each group; returns SIM_EINVAL if one chip alone exceeds the limit.
template <class ChipAt, class Emit>
int plan_groups(ChipAt chip_at, int n, int limit, Emit emit) {
  sim_launch_group cur{0, 0, 0, 0, false};
  int64_t e = 0;
  for (int i = 0; i < n; ++i) {
    const int np = chip_at(i)->hd.n_patches;
    if (np > 1 && np > limit) return SIM_EINVAL;
    const bool m = cur.multi || np > 1;
    if (cur.n_chips > 0 && m && cur.n_entries + np > limit) {
      emit(cur);
      cur = sim_launch_group{i, 0, e, 0, false};
    }
    cur.n_chips++;
    cur.n_entries += np;
    cur.multi = cur.multi || np > 1;
    e += np;
  }
  if (cur.n_chips > 0) emit(cur);
  return SIM_OK;
}

// Writes the launch-table entries of chips [k0, k0 + count) (first entries first[], stop
// cycles stop[]) on the stream, LIST_CHIPS chips per kernel.
template <class ChipAt, class FirstAt, class StopAt>
int write_table(LaunchEntry* table, ChipAt chip_at, FirstAt first_at, StopAt stop_at, int n, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += LIST_CHIPS) {
    ChipList L{};
    L.count = std::min(LIST_CHIPS, n - k0);
    for (int k = 0; k < L.count; ++k) {
      L.chip[k] = chip_at(k0 + k)->dd;
      L.first[k] = first_at(k0 + k);
      L.stop[k] = stop_at(k0 + k);
    }
    hipLaunchKernelGGL(fill_table, dim3(L.count), dim3(64), 0, s, table, L);
    HIPCHECK(hipGetLastError());
  }
  return SIM_OK;
}

// Gathers the error words of chips 0..n-1 into err_dev, copies them to err_host and returns
// the worst status (synchronises the stream).
template <class ChipAt>
int gather_status(int32_t* err_dev, int32_t* err_host, ChipAt chip_at, int n, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += LIST_CHIPS) {
    ChipList L{};
    L.count = std::min(LIST_CHIPS, n - k0);
    for (int k = 0; k < L.count; ++k) L.chip[k] = chip_at(k0 + k)->dd;
    hipLaunchKernelGGL(gather_errors, dim3(1), dim3(LIST_CHIPS < 64 ? 64 : 128), 0, s, err_dev, k0, L);
    HIPCHECK(hipGetLastError());
  }
  HIPCHECK(hipMemcpyAsync(err_host, err_dev, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  int worst = SIM_OK;
  for (int i = 0; i < n; ++i) {
    if (err_host[i] == 1) worst = SIM_EHANG;
    else if (err_host[i] == ERR_WATCHDOG && worst == SIM_OK) worst = SIM_ELIVELOCK;
    else if (err_host[i] && worst == SIM_OK) worst = SIM_EINVARIANT;
  }
  return worst;
}

void drop_graph(sim_group* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  g->graph_chunk = 0;
}

// Recomputes the members' table layout, launch groups and kernel after a membership change.
int rebuild(sim_group* g) {
  g->members.clear();
  g->first_entry.clear();
  g->groups.clear();
  for (size_t i = 0; i < g->slots.size(); ++i)
    if (g->slots[i]) g->members.push_back((int32_t)i);
  const int n = (int)g->members.size();
  auto chip_at = [g](int k) { return g->slots[g->members[k]]; };
  const BatchKind k = batch_kind(chip_at, n, g->block);
  g->fast = k.fast;
  g->opt = k.opt;
  g->var = k.var;
  const int limit = k.multi ? resident_limit(g->block, k.fast, k.opt, k.var, false) : 0;
  int64_t e = 0;
  for (int i = 0; i < n; ++i) {
    g->first_entry.push_back((int32_t)e);
    e += chip_at(i)->hd.n_patches;
  }
  g->n_entries = e;
  int rc = plan_groups(chip_at, n, limit, [g](const sim_launch_group& lg) { g->groups.push_back(lg); });
  if (rc) return rc;
  drop_graph(g);
  g->dirty = false;
  return SIM_OK;
}

// Builds the graph of one chunk: one kernel node per launch group, in order.
int build_graph(sim_group* g, int chunk) {
  drop_graph(g);
  HIPCHECK(hipGraphCreate(&g->graph, 0));
  hipGraphNode_t prev = nullptr;
  static unsigned long long* const no_digests = nullptr;
  static const int zero = 0;
  for (const sim_launch_group& lg : g->groups) {
    const LaunchEntry* table = g->table_dev + lg.first_entry;
    void* args[] = {(void*)&table, (void*)&chunk, (void*)&no_digests, (void*)&zero};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(batch_kernel(lg.multi, g->fast, g->opt, g->var));
    kp.gridDim = dim3((unsigned)lg.n_entries);
    kp.blockDim = dim3((unsigned)g->block);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    HIPCHECK(hipGraphAddKernelNode(&node, g->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
    if (lg.multi) {
      // the patches of a chip wait on each other: ask for co-residency as a cooperative launch does
      hipKernelNodeAttrValue v{};
      v.cooperative = 1;
      HIPCHECK(hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v));
    }
    prev = node;
  }
  HIPCHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  g->graph_chunk = chunk;
  return SIM_OK;
}

// ---- batched step without a workspace argument ---------------------------------------------------
// simb_step_noalloc keeps its launch table and error words in this array instead of a caller-owned
// workspace.  Host code never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): each device's copy is looked up once with hipGetSymbolAddress.
constexpr int NOALLOC_MAX_CHIPS = 1024;
constexpr int NOALLOC_MAX_ENTRIES = 32768;
constexpr size_t NOALLOC_TABLE_BYTES = (size_t)NOALLOC_MAX_ENTRIES * sizeof(LaunchEntry);
constexpr size_t NOALLOC_BYTES = NOALLOC_TABLE_BYTES + (size_t)NOALLOC_MAX_CHIPS * sizeof(int32_t);
static_assert(NOALLOC_TABLE_BYTES % 256 == 0, "error words start 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::atomic<void*> g_scratch_dev[NOALLOC_MAX_DEVICES];

// Device address of the current device's copy of `scratch` (looked up on first use).
int scratch_of_current_device(char** out) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SIM_EINVAL;
  void* p = g_scratch_dev[dev].load(std::memory_order_acquire);
  if (!p) {
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SIM_EHIP;
    g_scratch_dev[dev].store(p, std::memory_order_release);
  }
  *out = static_cast<char*>(p);
  return SIM_OK;
}

}  // namespace

extern "C" {

int simb_create(sim_t* const* chips, int32_t n, int32_t block, int32_t max_chips, int64_t max_patches, void* dev_mem,
                size_t bytes, void* stream, simb_t** out) {
  if (!out) return SIM_EINVAL;
  *out = nullptr;
  if (n < 0 || (n > 0 && !chips) || !dev_mem || block < 0 || block > 256 || block % 64) return SIM_EINVAL;
  if (reinterpret_cast<uintptr_t>(dev_mem) % 256) return SIM_EINVAL;
  int64_t entries = 0;
  int32_t bmax = 0;
  for (int i = 0; i < n; ++i) {
    if (!chips[i]) return SIM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (chips[j] == chips[i]) return SIM_EINVAL;
    entries += chips[i]->hd.n_patches;
    bmax = std::max(bmax, chips[i]->block);
  }
  if (!max_chips) max_chips = n;
  if (!max_patches) max_patches = entries;
  if (max_chips < n || max_patches < entries) return SIM_EINVAL;
  const size_t need = simb_state_bytes(max_chips, max_patches);
  if (!need) return SIM_EINVAL;
  if (bytes < need) return SIM_ENOMEM;
  const int32_t blk = block ? block : bmax;
  if (!blk) return SIM_EINVAL;
  sim_group* g = new (std::nothrow) sim_group();
  if (!g) return SIM_ENOMEM;
  g->slots.assign(chips, chips + n);
  g->block = blk;
  g->max_chips = max_chips;
  g->max_entries = max_patches;
  g->stream = static_cast<hipStream_t>(stream);
  g->table_dev = static_cast<LaunchEntry*>(dev_mem);
  g->err_dev = reinterpret_cast<int32_t*>(static_cast<char*>(dev_mem) +
                                          align_up((size_t)max_patches * sizeof(LaunchEntry), 256));
  g->use_graph = false;
  g->graph = nullptr;
  g->exec = nullptr;
  g->graph_chunk = 0;
  g->dirty = true;
  const int rc = rebuild(g);
  if (rc) {
    delete g;
    return rc;
  }
  *out = g;
  return SIM_OK;
}

int simb_add(simb_t* g, sim_t* chip, int32_t* slot) {
  if (!g || !chip || !slot) return SIM_EINVAL;
  int free_slot = -1, members = 0;
  int64_t entries = chip->hd.n_patches;
  for (size_t i = 0; i < g->slots.size(); ++i) {
    if (g->slots[i] == chip) return SIM_EINVAL;
    if (!g->slots[i]) {
      if (free_slot < 0) free_slot = (int)i;
    } else {
      members++;
      entries += g->slots[i]->hd.n_patches;
    }
  }
  if (members + 1 > g->max_chips || entries > g->max_entries) return SIM_EBUSY;
  // a chip of several patches must fit the device at once under the batch's kernel
  if (chip->hd.n_patches > 1) {
    std::vector<sim_chip*> all(1, chip);
    for (sim_chip* h : g->slots)
      if (h) all.push_back(h);
    const BatchKind k = batch_kind([&all](int i) { return all[i]; }, (int)all.size(), g->block);
    if (chip->hd.n_patches > resident_limit(g->block, k.fast, k.opt, k.var, false)) return SIM_EINVAL;
  }
  if (free_slot < 0) {
    free_slot = (int)g->slots.size();
    g->slots.push_back(chip);
  } else {
    g->slots[free_slot] = chip;
  }
  g->dirty = true;
  *slot = free_slot;
  return SIM_OK;
}

int simb_remove(simb_t* g, int32_t slot) {
  if (!g || slot < 0 || slot >= (int32_t)g->slots.size() || !g->slots[slot]) return SIM_EINVAL;
  g->slots[slot] = nullptr;
  g->dirty = true;
  return SIM_OK;
}

int32_t simb_slots(const simb_t* g) { return g ? (int32_t)g->slots.size() : -1; }

int simb_stats(simb_t* g, int32_t slot, sim_stats_t* out) {
  if (!g || slot < 0 || slot >= (int32_t)g->slots.size() || !g->slots[slot]) return SIM_EINVAL;
  return sim_stats(g->slots[slot], out);
}

int simb_set_graph(simb_t* g, int32_t on) {
  if (!g) return SIM_EINVAL;
  g->use_graph = on != 0;
  if (!g->use_graph) drop_graph(g);
  return SIM_OK;
}

int simb_step(simb_t* g, const int64_t* cycles) {
  if (!g || !cycles) return SIM_EINVAL;
  if (g->dirty) {
    const int rc = rebuild(g);
    if (rc) return rc;
  }
  const int n = (int)g->members.size();
  int64_t longest = 0;
  int chunk = 1 << 30;
  for (int k = 0; k < n; ++k) {
    const sim_chip* h = g->slots[g->members[k]];
    const int64_t c = cycles[g->members[k]];
    if (c < 0 || h->cycle + c > 0x7FFFFFFFll) return SIM_EINVAL;
    longest = std::max(longest, c);
    chunk = std::min(chunk, h->chunk);
  }
  if (!longest) return SIM_OK;
  auto chip_at = [g](int k) { return g->slots[g->members[k]]; };
  int rc = write_table(
      g->table_dev, chip_at, [g](int k) { return g->first_entry[k]; },
      [g, cycles](int k) { return (int)(g->slots[g->members[k]]->cycle + cycles[g->members[k]]); }, n, g->stream);
  if (rc) return rc;
  if (g->use_graph) {
    if (!g->exec || g->graph_chunk != chunk) {
      if ((rc = build_graph(g, chunk))) return rc;
    }
    const int64_t launches = (longest + chunk - 1) / chunk;
    for (int64_t k = 0; k < launches; ++k) HIPCHECK(hipGraphLaunch(g->exec, g->stream));
  } else {
    for (const sim_launch_group& lg : g->groups) {
      int64_t lg_longest = 0;
      for (int i = lg.first_chip; i < lg.first_chip + lg.n_chips; ++i)
        lg_longest = std::max(lg_longest, cycles[g->members[i]]);
      const int launches = (int)((lg_longest + chunk - 1) / chunk);
      for (int k = 0; k < launches; ++k) {
        rc = launch_entries(g->table_dev + lg.first_entry, lg.n_entries, lg.multi, g->fast, g->block, chunk, nullptr, 0,
                            g->stream, g->opt, g->var);
        if (rc) return rc;
      }
    }
  }
  for (int k = 0; k < n; ++k) g->slots[g->members[k]]->cycle += cycles[g->members[k]];
  std::vector<int32_t> errs((size_t)n);
  return gather_status(g->err_dev, errs.data(), chip_at, n, g->stream);
}

int simb_destroy(simb_t* g) {
  if (!g) return SIM_EINVAL;
  (void)hipStreamSynchronize(g->stream);
  drop_graph(g);
  delete g;
  return SIM_OK;
}

int simb_step_noalloc(sim_t* const* chips, int32_t n, int32_t block, const int64_t* cycles, void* stream) {
  if (n < 0 || (n > 0 && (!chips || !cycles)) || block < 0 || block > 256 || block % 64) return SIM_EINVAL;
  if (n > NOALLOC_MAX_CHIPS) return SIM_ENOMEM;
  int32_t first[NOALLOC_MAX_CHIPS];
  int64_t entries = 0, longest = 0;
  int32_t bmax = 0;
  int chunk = 1 << 30;
  for (int i = 0; i < n; ++i) {
    if (!chips[i]) return SIM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (chips[j] == chips[i]) return SIM_EINVAL;
    if (cycles[i] < 0 || chips[i]->cycle + cycles[i] > 0x7FFFFFFFll) return SIM_EINVAL;
    first[i] = (int32_t)std::min<int64_t>(entries, NOALLOC_MAX_ENTRIES);
    entries += chips[i]->hd.n_patches;
    bmax = std::max(bmax, chips[i]->block);
    longest = std::max(longest, cycles[i]);
    chunk = std::min(chunk, chips[i]->chunk);
  }
  if (entries > NOALLOC_MAX_ENTRIES) return SIM_ENOMEM;
  if (!longest) return SIM_OK;
  const int32_t blk = block ? block : bmax;
  char* ws = nullptr;
  int rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  LaunchEntry* table = reinterpret_cast<LaunchEntry*>(ws);
  int32_t* err_dev = reinterpret_cast<int32_t*>(ws + NOALLOC_TABLE_BYTES);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto chip_at = [chips](int k) { return chips[k]; };
  const BatchKind k = batch_kind(chip_at, n, blk);
  const int limit = k.multi ? resident_limit(blk, k.fast, k.opt, k.var, false) : 0;
  // a chip too large to be resident is refused before anything is launched
  rc = plan_groups(chip_at, n, limit, [](const sim_launch_group&) {});
  if (rc) return rc;
  // every entry the launches read is written here; nothing in the array needs clearing
  rc = write_table(
      table, chip_at, [&first](int i) { return first[i]; },
      [chips, cycles](int i) { return (int)(chips[i]->cycle + cycles[i]); }, n, s);
  if (rc) return rc;
  int launch_rc = SIM_OK;
  rc = plan_groups(chip_at, n, limit, [&](const sim_launch_group& lg) {
    if (launch_rc) return;
    int64_t lg_longest = 0;
    for (int i = lg.first_chip; i < lg.first_chip + lg.n_chips; ++i) lg_longest = std::max(lg_longest, cycles[i]);
    const int launches = (int)((lg_longest + chunk - 1) / chunk);
    for (int l = 0; l < launches && !launch_rc; ++l)
      launch_rc = launch_entries(table + lg.first_entry, lg.n_entries, lg.multi, k.fast, blk, chunk, nullptr, 0, s, k.opt,
                                 k.var);
  });
  if (rc) return rc;
  if (launch_rc) return launch_rc;
  for (int i = 0; i < n; ++i) chips[i]->cycle += cycles[i];
  int32_t errs[NOALLOC_MAX_CHIPS];
  return gather_status(err_dev, errs, chip_at, n, s);
}

}  // extern "C"
