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
// cycles.  A chip is cut into rectangular patches, one workgroup per patch; a workgroup
// steps its tiles, then publishes the number of cycles it has completed in a per-patch flag.
// Before cycle c it waits only for its (up to four) neighbouring patches to have completed c
// cycles, because the only state crossing a patch edge within a cycle is a link slot.  A chip
// that fits one workgroup needs no flags at all.  State is structure-of-arrays int32 in HBM:
// link slots double-buffered by cycle parity, core words, reply-queue nodes, L1/L2 tag sets
// stored most-recently-used first (a set is one or two 16-byte vectors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "nocsim.h"

namespace {

// ---- encodings ---------------------------------------------------------------------------
constexpr int KIND_REQ = 0, KIND_REPLY = 1, KIND_BG = 2;
constexpr int CORE_IDLE = 0, CORE_L1MISS = 1, CORE_SEND = 2, CORE_WAIT = 3, CORE_FILL = 4;
constexpr int32_t LINE_MASK = 0x3FFFFFFF;
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
  int32_t s1, w1, s2, w2;
  int32_t l1_lat, mem_lat, shared_lines, private_lines;
  int32_t pw, ph, pgx, pgy;  // patch shape and patch grid
  int32_t stop, max_patches; // cycle the chip stops at (single-chip launches); flag capacity
  int4* link;                // [2 parity][4 port][N]
  int4* core;                // [4][N]
  int4* node;                // [N]: next, ready, line, 0
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

// ---- coherent access for state that crosses workgroups -------------------------------------
// Link slots on a patch edge and reply-queue nodes of a multi-patch chip are read and written
// by different workgroups, possibly on different XCDs; they use device-scope relaxed atomics,
// and stores are ordered before the cycle flag with s_waitcnt.
__device__ __forceinline__ int ld_coh(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int4 ld_slot(const int4* p, bool coh) {
  if (!coh) return *p;
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  unsigned long long a = __hip_atomic_load(const_cast<unsigned long long*>(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long b = __hip_atomic_load(const_cast<unsigned long long*>(q + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_int4((int)(uint32_t)a, (int)(uint32_t)(a >> 32), (int)(uint32_t)b, (int)(uint32_t)(b >> 32));
}
__device__ __forceinline__ void st_slot(int4* p, int4 v, bool coh) {
  if (!coh) { *p = v; return; }
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)(uint32_t)v.x | ((unsigned long long)(uint32_t)v.y << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)(uint32_t)v.z | ((unsigned long long)(uint32_t)v.w << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool COH> __device__ __forceinline__ int ld_i(const int* p) { return COH ? ld_coh(p) : *p; }
template <bool COH> __device__ __forceinline__ void st_i(int* p, int v) { if (COH) st_coh(p, v); else *p = v; }

// ---- counter-based randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -----------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Zipf rank through a quantile table: bucket from the high half of u, linear position inside
// the bucket from the low half.
__device__ __forceinline__ int zipf_rank(const uint32_t* __restrict__ q, uint32_t u) {
  const uint32_t b = u >> 16, f = u & 0xFFFFu;
  const uint32_t lo = q[b], hi = q[b + 1];
  return (int)(lo + (uint32_t)(((unsigned long long)f * (hi - lo)) >> 16));
}

// ---- set-associative LRU sets: tags most recently used first -------------------------------
// touch: on a hit move the line to the front; on a miss insert it at the front if `insert`,
// dropping the last way (an invalid one if any, else the least recently used).
template <int WAYS> struct SetIO;
template <> struct SetIO<1> {
  __device__ static void ld(const int* p, int* v) { v[0] = p[0]; }
  __device__ static void st(int* p, const int* v) { p[0] = v[0]; }
};
template <> struct SetIO<2> {
  __device__ static void ld(const int* p, int* v) { int2 a = *reinterpret_cast<const int2*>(p); v[0] = a.x; v[1] = a.y; }
  __device__ static void st(int* p, const int* v) { *reinterpret_cast<int2*>(p) = make_int2(v[0], v[1]); }
};
template <> struct SetIO<4> {
  __device__ static void ld(const int* p, int* v) { int4 a = *reinterpret_cast<const int4*>(p); v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; }
  __device__ static void st(int* p, const int* v) { *reinterpret_cast<int4*>(p) = make_int4(v[0], v[1], v[2], v[3]); }
};
template <> struct SetIO<8> {
  __device__ static void ld(const int* p, int* v) {
    int4 a = reinterpret_cast<const int4*>(p)[0], b = reinterpret_cast<const int4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
  __device__ static void st(int* p, const int* v) {
    reinterpret_cast<int4*>(p)[0] = make_int4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<int4*>(p)[1] = make_int4(v[4], v[5], v[6], v[7]);
  }
};

template <int WAYS>
__device__ __forceinline__ bool touch_w(int* p, int line, bool insert) {
  int v[WAYS];
  SetIO<WAYS>::ld(p, v);
  int pos = WAYS;
#pragma unroll
  for (int i = WAYS - 1; i >= 0; --i)
    if (v[i] == line) pos = i;
  if (pos == 0) return true;
  if (pos == WAYS && !insert) return false;
  const int lim = pos == WAYS ? WAYS - 1 : pos;
#pragma unroll
  for (int i = WAYS - 1; i >= 1; --i)
    if (i <= lim) v[i] = v[i - 1];
  v[0] = line;
  SetIO<WAYS>::st(p, v);
  return pos != WAYS;
}

__device__ __forceinline__ bool touch(int* p, int ways, int line, bool insert) {
  switch (ways) {
    case 8: return touch_w<8>(p, line, insert);
    case 4: return touch_w<4>(p, line, insert);
    case 2: return touch_w<2>(p, line, insert);
    default: return touch_w<1>(p, line, insert);
  }
}

// Per-workgroup counters in LDS (rare events) and per-thread counters in registers (every
// cycle: link traversals, deflections, injections, ejections, latency sums).
struct LdsStats {
  unsigned long long v[NSTAT];
};
struct Acc {
  int trav, defl;
  int inj[3], ej[3];
  unsigned long long lat[3];
};
__device__ __forceinline__ void lds_add(LdsStats& L, int i, unsigned long long d) { atomicAdd(&L.v[i], d); }

// ---- one tile, one cycle ---------------------------------------------------------------------
// Phase one (Sec. 7.1, memory access), phase two (arbitration) and phase three (traversal,
// ejection, injection) of tile t in cycle c.  Reads the input slots of parity c, writes the
// neighbours' slots of parity c+1; every other word it writes is owned by t, except the
// queue nodes of requesters queued at t (t is their home while they wait).
template <bool MULTI>
__device__ __forceinline__ void tile_step(const ChipDev& C, int t, int x, int y, int c, const bool cross[4],
                                          Acc& acc, LdsStats& L) {
  const int N = C.N;
  const int cur = c & 1, nxt = cur ^ 1;
  const bool v0 = y > 0, v1 = y < C.H - 1, v2 = x < C.W - 1, v3 = x > 0;
  const int4 EMPTY = make_int4(-1, -1, -1, -1);

  int4 f0 = v0 ? ld_slot(&C.link[(cur * 4 + 0) * N + t], cross[0]) : EMPTY;
  int4 f1 = v1 ? ld_slot(&C.link[(cur * 4 + 1) * N + t], cross[1]) : EMPTY;
  int4 f2 = v2 ? ld_slot(&C.link[(cur * 4 + 2) * N + t], cross[2]) : EMPTY;
  int4 f3 = v3 ? ld_slot(&C.link[(cur * 4 + 3) * N + t], cross[3]) : EMPTY;
  int4 k0 = C.core[t];          // state, wake, line, issue
  int4 k1 = C.core[N + t];      // l2q, l2q_line, hit_head, hit_tail
  int4 k2 = C.core[2 * N + t];  // miss_head, miss_tail, bg_pending, force_line
  int fdst = C.core[3 * N + t].x;
  bool d0 = false, d1 = false, d2 = false, d3 = false;
  const uint4 r = philox((uint32_t)c, (uint32_t)t, 0u, 0u, C.key0, C.key1);

  // ---- phase one: home L2 service, then the core --------------------------------------------
  // Indices read from state are checked before they address memory: a corrupt index sets the
  // chip's error word (reported as SIM_EHANG's sibling, SIM_EINVARIANT) instead of faulting.
#define GUARD(i)                                                   \
  if ((unsigned)(i) >= (unsigned)N) {                              \
    st_coh(C.err, 2);                                              \
    return;                                                        \
  }
  if (k1.x >= 0) {  // a request ejected here last cycle: look up the home slice
    const int rq = k1.x, line = k1.y;
    GUARD(rq)
    if (k1.w >= 0) { GUARD(k1.w) }
    if (k2.y >= 0) { GUARD(k2.y) }
    int* set = C.l2 + ((size_t)t * C.s2 + ((uint32_t)line / (uint32_t)N & (uint32_t)(C.s2 - 1))) * C.w2;
    const bool hit = touch(set, C.w2, line, true);
    lds_add(L, hit ? SIM_ST_L2_HIT : SIM_ST_L2_MISS, 1);
    const int ready = hit ? c : c + C.mem_lat;
    int* nd = reinterpret_cast<int*>(&C.node[rq]);
    st_i<MULTI>(nd + 0, -1);
    st_i<MULTI>(nd + 1, ready);
    st_i<MULTI>(nd + 2, line);
    if (hit) {
      if (k1.w >= 0) st_i<MULTI>(reinterpret_cast<int*>(&C.node[k1.w]), rq);
      else k1.z = rq;
      k1.w = rq;
    } else {
      if (k2.y >= 0) st_i<MULTI>(reinterpret_cast<int*>(&C.node[k2.y]), rq);
      else k2.x = rq;
      k2.y = rq;
    }
    k1.x = -1;
    k1.y = -1;
    d1 = true;
    d2 = true;
  }
  if (k0.x == CORE_FILL) {
    if (k0.y == c) {  // the block arrived: fill L1, the op completes
      const int line = k0.z;
      touch(C.l1 + ((size_t)t * C.s1 + (line & (C.s1 - 1))) * C.w1, C.w1, line, true);
      const unsigned long long lat = (unsigned long long)(c - k0.w);
      lds_add(L, SIM_ST_OPS_DONE, 1);
      lds_add(L, SIM_ST_OP_LAT, lat);
      atomicMax(&L.v[SIM_ST_OP_LAT_MAX], lat);
      k0.x = CORE_IDLE;
      d0 = true;
    }
  } else if (k0.x == CORE_L1MISS) {
    if (k0.y == c) {  // L1 miss penalty over: local home slice, or a request flit
      const int line = k0.z;
      if ((uint32_t)line % (uint32_t)N == (uint32_t)t) {
        int* set = C.l2 + ((size_t)t * C.s2 + ((uint32_t)line / (uint32_t)N & (uint32_t)(C.s2 - 1))) * C.w2;
        const bool hit = touch(set, C.w2, line, true);
        lds_add(L, hit ? SIM_ST_L2_HIT : SIM_ST_L2_MISS, 1);
        k0.x = CORE_FILL;
        k0.y = hit ? c + 1 : c + C.mem_lat;
      } else {
        k0.x = CORE_SEND;
        lds_add(L, SIM_ST_REQ_MADE, 1);
      }
      d0 = true;
    }
  } else if (k0.x == CORE_IDLE) {
    bool issue = false;
    int line = 0;
    if (k2.w >= 0) {
      line = k2.w;
      k2.w = -1;
      d2 = true;
      issue = true;
    } else if (r.x < C.op_thr) {
      issue = true;
      if (C.private_lines > 0 && r.y >= C.shared_thr)
        line = C.shared_lines + t * C.private_lines + zipf_rank(C.zp, r.z);
      else
        line = zipf_rank(C.zs, r.z);
    }
    if (issue) {
      lds_add(L, SIM_ST_OPS_ISSUED, 1);
      k0.z = line;
      k0.w = c;
      d0 = true;
      if (touch(C.l1 + ((size_t)t * C.s1 + (line & (C.s1 - 1))) * C.w1, C.w1, line, false)) {
        lds_add(L, SIM_ST_L1_HIT, 1);
        lds_add(L, SIM_ST_OPS_DONE, 1);
      } else {
        lds_add(L, SIM_ST_L1_MISS, 1);
        k0.x = CORE_L1MISS;
        k0.y = c + C.l1_lat;
      }
    }
  }

  // ---- phase two: injection into a free input, then oldest-first arbitration ----------------
  const int arrivals = (f0.x >= 0) + (f1.x >= 0) + (f2.x >= 0) + (f3.x >= 0);
  const int deg = (int)v0 + (int)v1 + (int)v2 + (int)v3;
  int cls = -1;
  if (k2.x >= 0) { GUARD(k2.x) }
  if (k1.z >= 0) { GUARD(k1.z) }
  if (k2.x >= 0 && ld_i<MULTI>(reinterpret_cast<const int*>(&C.node[k2.x]) + 1) <= c) cls = 0;
  else if (k1.z >= 0) cls = 1;
  else if (k0.x == CORE_SEND) cls = 2;
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
    if (cls <= 1) {  // reply: pop the queue head
      const int rq = cls == 0 ? k2.x : k1.z;
      const int* nd = reinterpret_cast<const int*>(&C.node[rq]);
      const int next = ld_i<MULTI>(nd + 0);
      if (cls == 0) {
        k2.x = next;
        if (next < 0) k2.y = -1;
      } else {
        k1.z = next;
        if (next < 0) k1.w = -1;
      }
      fi.x = rq;
      fi.w = (KIND_REPLY << 30) | ld_i<MULTI>(nd + 2);
      lds_add(L, SIM_ST_REPLY_SENT, 1);
      acc.inj[KIND_REPLY]++;
      d1 = true;
      d2 = true;
    } else if (cls == 2) {
      fi.x = (int)((uint32_t)k0.z % (uint32_t)N);
      fi.w = (KIND_REQ << 30) | k0.z;
      k0.x = CORE_WAIT;
      d0 = true;
      acc.inj[KIND_REQ]++;
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
      acc.inj[KIND_BG]++;
    }
  }

  // Oldest first (key: inject cycle, then source tile; empty slots sort last).  Only
  // (key, dst, index) tuples are sorted; the port of flit i is packed at bits 3i..3i+2 of
  // `ports` (7 = none) and each flit is stored straight into its neighbour's slot.
  uint32_t qh0 = f0.x < 0 ? ~0u : (uint32_t)f0.y, ql0 = f0.x < 0 ? ~0u : (uint32_t)f0.z;
  uint32_t qh1 = f1.x < 0 ? ~0u : (uint32_t)f1.y, ql1 = f1.x < 0 ? ~0u : (uint32_t)f1.z;
  uint32_t qh2 = f2.x < 0 ? ~0u : (uint32_t)f2.y, ql2 = f2.x < 0 ? ~0u : (uint32_t)f2.z;
  uint32_t qh3 = f3.x < 0 ? ~0u : (uint32_t)f3.y, ql3 = f3.x < 0 ? ~0u : (uint32_t)f3.z;
  uint32_t qh4 = fi.x < 0 ? ~0u : (uint32_t)fi.y, ql4 = fi.x < 0 ? ~0u : (uint32_t)fi.z;
  int sd0 = f0.x, sd1 = f1.x, sd2 = f2.x, sd3 = f3.x, sd4 = fi.x;
  int si0 = 0, si1 = 1, si2 = 2, si3 = 3, si4 = 4;
#define CSWAP(a, b)                                                                              \
  if (qh##b < qh##a || (qh##b == qh##a && ql##b < ql##a)) {                                      \
    uint32_t th = qh##a; qh##a = qh##b; qh##b = th;                                              \
    uint32_t tl = ql##a; ql##a = ql##b; ql##b = tl;                                              \
    int td = sd##a; sd##a = sd##b; sd##b = td;                                                   \
    int ti = si##a; si##a = si##b; si##b = ti;                                                   \
  }
  CSWAP(0, 1) CSWAP(3, 4) CSWAP(2, 4) CSWAP(2, 3) CSWAP(1, 4) CSWAP(0, 3) CSWAP(0, 2) CSWAP(1, 3) CSWAP(1, 2)
#undef CSWAP

  const unsigned valid = (v0 ? 1u : 0u) | (v1 ? 2u : 0u) | (v2 ? 4u : 0u) | (v3 ? 8u : 0u);
  unsigned used = 0;
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

  // ---- phase three: traversal to the neighbours' next-cycle inputs, ejection, generation ---
  int4 oe = EMPTY;
  auto send = [&](const int4& f, unsigned port) {
    if (port == 4) { oe = f; return; }
    if (port > 3) return;
    const int nbr = port == 0 ? t - C.W : port == 1 ? t + C.W : port == 2 ? t + 1 : t - 1;
    const int slot = (int)(port ^ 1u);
    const bool cx = port == 0 ? cross[0] : port == 1 ? cross[1] : port == 2 ? cross[2] : cross[3];
    st_slot(&C.link[(nxt * 4 + slot) * N + nbr], f, cx);
  };
  send(f0, ports & 7u);
  send(f1, (ports >> 3) & 7u);
  send(f2, (ports >> 6) & 7u);
  send(f3, (ports >> 9) & 7u);
  send(fi, (ports >> 12) & 7u);
  const unsigned idle = valid & ~used;  // links that carry nothing next cycle
  if (idle & 1u) st_slot(&C.link[(nxt * 4 + 1) * N + t - C.W], EMPTY, cross[0]);
  if (idle & 2u) st_slot(&C.link[(nxt * 4 + 0) * N + t + C.W], EMPTY, cross[1]);
  if (idle & 4u) st_slot(&C.link[(nxt * 4 + 3) * N + t + 1], EMPTY, cross[2]);
  if (idle & 8u) st_slot(&C.link[(nxt * 4 + 2) * N + t - 1], EMPTY, cross[3]);

  if (oe.x >= 0) {
    const int kind = (int)((uint32_t)oe.w >> 30);
    const int lat = c - oe.y;
    acc.ej[kind]++;
    acc.lat[kind] += (unsigned long long)lat;
    atomicMax(&L.v[SIM_ST_LAT_MAX], (unsigned long long)lat);
    lds_add(L, SIM_ST_HIST + min(15, 31 - __builtin_clz((unsigned)max(lat, 1))), 1);
    if (kind == KIND_REQ) {
      lds_add(L, SIM_ST_REQ_RECV, 1);
      k1.x = oe.z;
      k1.y = oe.w & LINE_MASK;
      d1 = true;
    } else if (kind == KIND_REPLY) {
      lds_add(L, SIM_ST_REPLY_RECV, 1);
      k0.x = CORE_FILL;
      k0.y = c + 1;
      d0 = true;
    }
  }
  if (N > 1 && r.w < C.bg_thr) {
    k2.z += 1;
    d2 = true;
    lds_add(L, SIM_ST_BG_GEN, 1);
  }
  if (d0) C.core[t] = k0;
  if (d1) C.core[N + t] = k1;
  if (d2) C.core[2 * N + t] = k2;
  if (d3) C.core[3 * N + t] = make_int4(fdst, 0, 0, 0);
#undef GUARD
}

// ---- state digest of the words a tile owns after cycle c --------------------------------------
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {  // SplitMix64 finalizer
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ unsigned long long mix_pair(unsigned long long h, int a, int b) {
  return mix64(h ^ (((unsigned long long)(uint32_t)a << 32) | (uint32_t)b));
}
__device__ unsigned long long tile_digest(const ChipDev& C, int t, int x, int y, int c, const bool cross[4]) {
  const int N = C.N, par = (c + 1) & 1;
  const bool v[4] = {y > 0, y < C.H - 1, x < C.W - 1, x > 0};
  unsigned long long h = mix64(((unsigned long long)(uint32_t)c << 32) | (uint32_t)t);
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int4 f = v[p] ? ld_slot(&C.link[(par * 4 + p) * N + t], cross[p]) : make_int4(-1, -1, -1, -1);
    h = mix_pair(h, f.x, f.y);
    h = mix_pair(h, f.z, f.w);
  }
  const int4 k0 = C.core[t], k1 = C.core[N + t], k2 = C.core[2 * N + t], k3 = C.core[3 * N + t];
  h = mix_pair(h, k0.x, k0.y);
  h = mix_pair(h, k0.z, k0.w);
  h = mix_pair(h, k1.x, k1.y);
  h = mix_pair(h, k1.z, k1.w);
  h = mix_pair(h, k2.x, k2.y);
  h = mix_pair(h, k2.z, 0);      // bg_pending, (node words are written by the home, not hashed)
  h = mix_pair(h, 0, 0);
  h = mix_pair(h, k2.w, k3.x);   // force_line, force_dst
  return h;
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

// ---- the persistent step kernel ----------------------------------------------------------------
// Workgroup w runs patch table[w].patch of chip table[w].chip from the cycle its flag records
// up to min(flag + chunk, stop).  digests (optional, single chip): digests[c - digest_base] +=
// this patch's share of the digest of cycle c.
template <bool MULTI>
__global__ void __launch_bounds__(256) step_kernel(const LaunchEntry* __restrict__ table, int chunk,
                                                    unsigned long long* digests, int digest_base) {
  __shared__ LdsStats L;
  __shared__ int s_stop_flag;
  const LaunchEntry e = table[blockIdx.x];
  const ChipDev C = *e.chip;
  const int patch = e.patch;
  const int pxi = patch % C.pgx, pyi = patch / C.pgx;
  const int x0 = pxi * C.pw, y0 = pyi * C.ph;
  const int cols = min(C.pw, C.W - x0), rows = min(C.ph, C.H - y0);
  const int ntiles = cols * rows;
  // neighbouring patch watched by lane 0..3 of the first wave (N, S, E, W), -1 if none
  const int lane = (int)threadIdx.x;
  const int my_nb = lane == 0 ? (pyi > 0 ? patch - C.pgx : -1)
                  : lane == 1 ? (pyi < C.pgy - 1 ? patch + C.pgx : -1)
                  : lane == 2 ? (pxi < C.pgx - 1 ? patch + 1 : -1)
                  : lane == 3 ? (pxi > 0 ? patch - 1 : -1) : -1;
  for (int i = threadIdx.x; i < NSTAT; i += blockDim.x) L.v[i] = 0;
  Acc acc = {};
  const int c0 = ld_coh(&C.flags[patch * FLAG_STRIDE]);
  const int c_end = min(c0 + chunk, e.stop >= 0 ? e.stop : C.stop);
  __syncthreads();

  for (int c = c0; c <= c_end; ++c) {
    if (MULTI) {  // wait until every neighbouring patch has completed c cycles
      if (threadIdx.x == 0) s_stop_flag = 0;
      __syncthreads();
      if (my_nb >= 0) {
        const int* fl = &C.flags[my_nb * FLAG_STRIDE];
        int spins = 0;
        while (ld_coh(fl) < c) {
          if (++spins > SPIN_LIMIT || ld_coh(C.err)) {
            st_coh(C.err, 1);
            s_stop_flag = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (s_stop_flag) break;
    }
    if (digests && c > c0) {  // digest of cycle c-1 (all writes into this patch's slots are done)
      unsigned long long h = 0;
      for (int j = threadIdx.x; j < ntiles; j += blockDim.x) {
        const int lx = j % cols, ly = j / cols, x = x0 + lx, y = y0 + ly;
        const bool cross[4] = {MULTI && ly == 0 && y > 0, MULTI && ly == rows - 1 && y < C.H - 1,
                               MULTI && lx == cols - 1 && x < C.W - 1, MULTI && lx == 0 && x > 0};
        h += tile_digest(C, y * C.W + x, x, y, c - 1, cross);
      }
      h = wave_sum(h);
      if ((threadIdx.x & 63) == 0 && c - 1 - digest_base >= 0) atomicAdd(&digests[c - 1 - digest_base], h);
    }
    if (c == c_end) break;
    for (int j = threadIdx.x; j < ntiles; j += blockDim.x) {
      const int lx = j % cols, ly = j / cols, x = x0 + lx, y = y0 + ly;
      const bool cross[4] = {MULTI && ly == 0 && y > 0, MULTI && ly == rows - 1 && y < C.H - 1,
                             MULTI && lx == cols - 1 && x < C.W - 1, MULTI && lx == 0 && x > 0};
      tile_step<MULTI>(C, y * C.W + x, x, y, c, cross, acc, L);
    }
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores are complete before the flag moves
    __syncthreads();
    if (threadIdx.x == 0) st_coh(&C.flags[patch * FLAG_STRIDE], c + 1);
  }

  // ---- flush counters ----
  {
    int v[8] = {acc.trav, acc.defl, acc.inj[0], acc.inj[1], acc.inj[2], acc.ej[0], acc.ej[1], acc.ej[2]};
    const int idx[8] = {SIM_ST_TRAVERSALS, SIM_ST_DEFLECTIONS, SIM_ST_INJ_REQ, SIM_ST_INJ_REPLY, SIM_ST_INJ_BG,
                        SIM_ST_EJ_REQ, SIM_ST_EJ_REPLY, SIM_ST_EJ_BG};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int s = wave_sum_i(v[i]);
      if ((threadIdx.x & 63) == 0 && s) atomicAdd(&L.v[idx[i]], (unsigned long long)s);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const unsigned long long s = wave_sum(acc.lat[k]);
      if ((threadIdx.x & 63) == 0 && s) atomicAdd(&L.v[SIM_ST_LAT_REQ + k], s);
    }
  }
  __syncthreads();
  if (patch == 0 && threadIdx.x == 0 && c_end > c0) L.v[SIM_ST_CYCLES] += (unsigned long long)(c_end - c0);
  __syncthreads();
  for (int i = threadIdx.x; i < NSTAT; i += blockDim.x) {
    if (!L.v[i]) continue;
    if (i == SIM_ST_LAT_MAX || i == SIM_ST_OP_LAT_MAX) atomicMax(&C.stats[i], L.v[i]);
    else atomicAdd(&C.stats[i], L.v[i]);
  }
}

// ---- small utility kernels (no memsets: these also record safely into graphs) -----------------
__global__ void fill_i32(int32_t* p, int32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_u64(unsigned long long* p, unsigned long long v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void set_stop(ChipDev* d, int stop) { d->stop = stop; }
// core words of a fresh chip: state idle, bg 0, everything else -1
__global__ void init_core(int4* core, int N) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < N; t += gridDim.x * blockDim.x) {
    core[t] = make_int4(CORE_IDLE, -1, -1, -1);
    core[N + t] = make_int4(-1, -1, -1, -1);
    core[2 * N + t] = make_int4(-1, -1, 0, -1);
    core[3 * N + t] = make_int4(-1, 0, 0, 0);
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
  LaunchEntry* table_dev;  // MAX_PATCHES entries
  LaunchEntry* table_host; // pinned staging
};

struct sim_group {
  std::vector<sim_chip*> chips;
  std::vector<int32_t> first_entry;  // first table entry of chip i
  int32_t block;
  bool multi;
  hipStream_t stream;
  LaunchEntry* table_dev;
  LaunchEntry* table_host;
  int64_t n_entries;
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
  if (N > (1 << 20)) return false;
  if (!pow2(c->l1_sets) || !ways_ok(c->l1_ways) || !pow2(c->l2_sets) || !ways_ok(c->l2_ways)) return false;
  if (c->l1_lat < 1 || c->mem_lat < 1 || c->shared_lines < 1 || c->private_lines < 0) return false;
  if ((int64_t)c->shared_lines + N * c->private_lines > (int64_t)LINE_MASK + 1) return false;
  return true;
}

struct Layout {
  size_t desc, link, core, node, l1, l2, zs, zp, flags, table, stats, err, total;
};

int max_patches(const sim_config* c) { return (int)std::min<int64_t>(MAX_PATCHES, (int64_t)c->width * c->height); }

Layout layout(const sim_config* c) {
  Layout L{};
  const size_t N = (size_t)c->width * c->height;
  const size_t maxp = (size_t)max_patches(c);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  L.desc = take(sizeof(ChipDev));
  L.link = take(2 * 4 * N * sizeof(int4));
  L.core = take(4 * N * sizeof(int4));
  L.node = take(N * sizeof(int4));
  L.l1 = take(N * c->l1_sets * c->l1_ways * sizeof(int32_t));
  L.l2 = take(N * c->l2_sets * c->l2_ways * sizeof(int32_t));
  L.zs = take((ZIPF_K + 1) * sizeof(uint32_t));
  L.zp = take((ZIPF_K + 1) * sizeof(uint32_t));
  L.flags = take(maxp * FLAG_STRIDE * sizeof(int32_t));
  L.table = take(maxp * sizeof(LaunchEntry));
  L.stats = take(NSTAT * sizeof(unsigned long long));
  L.err = take(256);
  L.total = o;
  return L;
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

// how many workgroups of `block` threads of the multi-patch kernel can be resident at once
int resident_limit(int block) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(step_kernel<true>), block, 0) != hipSuccess)
    return 0;
  return per_cu * device_cus();
}

int upload_desc(sim_chip* h) {
  HIPCHECK(hipMemcpyAsync(h->dd, &h->hd, sizeof(ChipDev), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
}

// Default mapping: one workgroup for small chips; otherwise square-ish patches, about one per
// compute unit.
void default_mapping(const sim_config* c, int32_t* pw, int32_t* ph, int32_t* block) {
  const int N = c->width * c->height;
  if (N <= 1024) {
    *pw = c->width;
    *ph = c->height;
    *block = N <= 64 ? 64 : 256;
    return;
  }
  const int target = device_cus();
  int side = 1;
  while ((int64_t)((c->width + side - 1) / side) * ((c->height + side - 1) / side) > target) side++;
  *pw = std::min(side, c->width);
  *ph = std::min(side, c->height);
  const int tiles = (*pw) * (*ph);
  *block = tiles <= 64 ? 64 : tiles <= 128 ? 128 : tiles <= 192 ? 192 : 256;
}

int apply_mapping(sim_chip* h, int32_t pw, int32_t ph, int32_t block) {
  if (pw < 1 || ph < 1 || block < 64 || block > 256 || block % 64) return SIM_EINVAL;
  pw = std::min(pw, h->cfg.width);
  ph = std::min(ph, h->cfg.height);
  const int pgx = (h->cfg.width + pw - 1) / pw, pgy = (h->cfg.height + ph - 1) / ph;
  const int np = pgx * pgy;
  if (np > h->hd.max_patches) return SIM_EINVAL;
  if (np > 1 && np > resident_limit(block)) return SIM_EINVAL;
  h->hd.pw = pw;
  h->hd.ph = ph;
  h->hd.pgx = pgx;
  h->hd.pgy = pgy;
  h->hd.n_patches = np;
  h->block = block;
  // every patch's flag records the chip's cycle
  int rc = launch_grid_fill_i32(h->hd.flags, (int32_t)h->cycle, (size_t)h->hd.max_patches * FLAG_STRIDE, h->stream);
  if (rc) return rc;
  for (int p = 0; p < np; ++p) h->table_host[p] = LaunchEntry{h->dd, p, -1};
  HIPCHECK(hipMemcpyAsync(h->table_dev, h->table_host, np * sizeof(LaunchEntry), hipMemcpyHostToDevice, h->stream));
  return upload_desc(h);
}

int launch_entries(const LaunchEntry* table, int64_t n, bool multi, int block, int chunk, unsigned long long* digests,
                   int digest_base, hipStream_t s) {
  if (n <= 0) return SIM_OK;
  if (multi) {
    void* args[] = {(void*)&table, (void*)&chunk, (void*)&digests, (void*)&digest_base};
    HIPCHECK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(step_kernel<true>), dim3((unsigned)n), dim3(block),
                                        args, 0, s));
  } else {
    hipLaunchKernelGGL(step_kernel<false>, dim3((unsigned)n), dim3(block), 0, s, table, chunk, digests, digest_base);
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
    default: return "unknown error";
  }
}

int sim_last_hip_error(void) { return g_last_hip; }

size_t sim_state_bytes(const sim_config* cfg) {
  if (!config_ok(cfg)) return 0;
  return layout(cfg).total;
}

int sim_create(const sim_config* cfg, const uint32_t* zs, const uint32_t* zp, int32_t zk, void* dev_mem, size_t bytes,
               void* stream, sim_t** out) {
  if (!out) return SIM_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg) || !zs || zk != ZIPF_K || (cfg->private_lines > 0 && !zp) || !dev_mem) return SIM_EINVAL;
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
  d.w_magic = cfg->width > 1 ? (uint32_t)((0x100000000ull + cfg->width - 1) / cfg->width) : 0u;
  d.s1 = cfg->l1_sets;
  d.w1 = cfg->l1_ways;
  d.s2 = cfg->l2_sets;
  d.w2 = cfg->l2_ways;
  d.l1_lat = cfg->l1_lat;
  d.mem_lat = cfg->mem_lat;
  d.shared_lines = cfg->shared_lines;
  d.private_lines = cfg->private_lines;
  d.stop = 0;
  d.max_patches = max_patches(cfg);
  d.link = reinterpret_cast<int4*>(h->base + Lo.link);
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
  if (hipHostMalloc(reinterpret_cast<void**>(&h->table_host), d.max_patches * sizeof(LaunchEntry), hipHostMallocDefault) != hipSuccess) {
    delete h;
    return SIM_EHIP;
  }
  int rc = SIM_OK;
  auto fail = [&](int code) { (void)hipHostFree(h->table_host); delete h; return code; };
  if ((rc = launch_grid_fill_i32(reinterpret_cast<int32_t*>(d.link), -1, 2 * 4 * (size_t)N * 4, h->stream))) return fail(rc);
  hipLaunchKernelGGL(init_core, dim3(std::min((N + 255) / 256, 4096)), dim3(256), 0, h->stream, d.core, N);
  if (hipGetLastError() != hipSuccess) return fail(SIM_EHIP);
  if ((rc = launch_grid_fill_i32(reinterpret_cast<int32_t*>(d.node), -1, (size_t)N * 4, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_i32(d.l1, -1, (size_t)N * cfg->l1_sets * cfg->l1_ways, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_i32(d.l2, -1, (size_t)N * cfg->l2_sets * cfg->l2_ways, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_u64(d.stats, 0, NSTAT, h->stream))) return fail(rc);
  if ((rc = launch_grid_fill_i32(d.err, 0, 1, h->stream))) return fail(rc);
  if (hipMemcpyAsync(const_cast<uint32_t*>(d.zs), zs, (ZIPF_K + 1) * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(SIM_EHIP);
  if (hipMemcpyAsync(const_cast<uint32_t*>(d.zp), zp ? zp : zs, (ZIPF_K + 1) * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(SIM_EHIP);
  int32_t pw, ph, block;
  default_mapping(cfg, &pw, &ph, &block);
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
  return err == 0 ? SIM_OK : err == 1 ? SIM_EHANG : SIM_EINVARIANT;
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
    int rc = launch_entries(h->table_dev, np, np > 1, h->block, h->chunk, dig, (int)h->cycle, h->stream);
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
  return 16 + N * 16 + N * 16 + N * h->hd.s1 * h->hd.w1 + N * h->hd.s2 * h->hd.w2 + 2 * NSTAT;
}

int sim_dump(sim_t* h, int32_t* buf, size_t words) {
  if (!h || !buf || words < sim_dump_words(h)) return SIM_EINVAL;
  const size_t N = (size_t)h->hd.N;
  const int par = (int)(h->cycle & 1);
  std::vector<int4> link(4 * N), core(4 * N), node(N);
  HIPCHECK(hipMemcpyAsync(link.data(), h->hd.link + (size_t)par * 4 * N, 4 * N * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(core.data(), h->hd.core, 4 * N * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(node.data(), h->hd.node, N * sizeof(int4), hipMemcpyDeviceToHost, h->stream));
  size_t o = 16;
  const size_t n1 = N * h->hd.s1 * h->hd.w1, n2 = N * h->hd.s2 * h->hd.w2;
  int32_t* l1 = buf + 16 + N * 32;
  int32_t* l2 = l1 + n1;
  HIPCHECK(hipMemcpyAsync(l1, h->hd.l1, n1 * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(l2, h->hd.l2, n2 * 4, hipMemcpyDeviceToHost, h->stream));
  unsigned long long st[NSTAT];
  HIPCHECK(hipMemcpyAsync(st, h->hd.stats, sizeof st, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  const int32_t hdr[16] = {0x4E4F4353, 1, h->hd.W, h->hd.H, (int32_t)(uint32_t)h->cycle, (int32_t)(h->cycle >> 32),
                           h->hd.s1, h->hd.w1, h->hd.s2, h->hd.w2, 0, 0, 0, 0, 0, 0};
  std::memcpy(buf, hdr, sizeof hdr);
  for (size_t t = 0; t < N; ++t)
    for (int p = 0; p < 4; ++p) {
      const int4 f = link[p * N + t];
      int32_t* w = buf + o + t * 16 + p * 4;
      w[0] = f.x; w[1] = f.y; w[2] = f.z; w[3] = f.w;
    }
  o += N * 16;
  for (size_t t = 0; t < N; ++t) {
    const int4 k0 = core[t], k1 = core[N + t], k2 = core[2 * N + t], k3 = core[3 * N + t], nd = node[t];
    const int32_t rec[16] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w, k2.x, k2.y, k2.z, nd.x, nd.y, nd.z, k2.w, k3.x};
    std::memcpy(buf + o + t * 16, rec, sizeof rec);
  }
  o += N * 16 + n1 + n2;
  for (int i = 0; i < NSTAT; ++i) {
    buf[o++] = (int32_t)(uint32_t)st[i];
    buf[o++] = (int32_t)(st[i] >> 32);
  }
  return SIM_OK;
}

int sim_load(sim_t* h, const int32_t* buf, size_t words) {
  if (!h || !buf || words < sim_dump_words(h)) return SIM_EINVAL;
  if (buf[0] != 0x4E4F4353 || buf[2] != h->hd.W || buf[3] != h->hd.H || buf[6] != h->hd.s1 || buf[7] != h->hd.w1 ||
      buf[8] != h->hd.s2 || buf[9] != h->hd.w2)
    return SIM_EINVAL;
  const size_t N = (size_t)h->hd.N;
  const int64_t cyc = (int64_t)(((uint64_t)(uint32_t)buf[5] << 32) | (uint32_t)buf[4]);
  if (cyc < 0 || cyc > 0x7FFFFFFF) return SIM_EINVAL;
  std::vector<int4> link(4 * N), core(4 * N), node(N);
  size_t o = 16;
  for (size_t t = 0; t < N; ++t)
    for (int p = 0; p < 4; ++p) {
      const int32_t* w = buf + o + t * 16 + p * 4;
      link[p * N + t] = make_int4(w[0], w[1], w[2], w[3]);
    }
  o += N * 16;
  for (size_t t = 0; t < N; ++t) {
    const int32_t* r = buf + o + t * 16;
    core[t] = make_int4(r[0], r[1], r[2], r[3]);
    core[N + t] = make_int4(r[4], r[5], r[6], r[7]);
    core[2 * N + t] = make_int4(r[8], r[9], r[10], r[14]);
    core[3 * N + t] = make_int4(r[15], 0, 0, 0);
    node[t] = make_int4(r[11], r[12], r[13], 0);
  }
  o += N * 16;
  const size_t n1 = N * h->hd.s1 * h->hd.w1, n2 = N * h->hd.s2 * h->hd.w2;
  const int par = (int)(cyc & 1);
  HIPCHECK(hipMemcpyAsync(h->hd.link + (size_t)par * 4 * N, link.data(), 4 * N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  int rc = launch_grid_fill_i32(reinterpret_cast<int32_t*>(h->hd.link + (size_t)(par ^ 1) * 4 * N), -1, 4 * N * 4, h->stream);
  if (rc) return rc;
  HIPCHECK(hipMemcpyAsync(h->hd.core, core.data(), 4 * N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hd.node, node.data(), N * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hd.l1, buf + o, n1 * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hd.l2, buf + o + n1, n2 * 4, hipMemcpyHostToDevice, h->stream));
  o += n1 + n2;
  unsigned long long st[NSTAT];
  for (int i = 0; i < NSTAT; ++i) st[i] = (unsigned long long)(uint32_t)buf[o + 2 * i] | ((unsigned long long)(uint32_t)buf[o + 2 * i + 1] << 32);
  HIPCHECK(hipMemcpyAsync(h->hd.stats, st, sizeof st, hipMemcpyHostToDevice, h->stream));
  h->cycle = cyc;
  if ((rc = launch_grid_fill_i32(h->hd.flags, (int32_t)cyc, (size_t)h->hd.max_patches * FLAG_STRIDE, h->stream))) return rc;
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
  const int4 k3 = make_int4(dst, 0, 0, 0);
  HIPCHECK(hipMemcpyAsync(h->hd.core + 3 * (size_t)h->hd.N + tile, &k3, sizeof k3, hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return SIM_OK;
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
  (void)hipHostFree(h->table_host);
  delete h;
  return SIM_OK;
}

// ---- batches ------------------------------------------------------------------------------------
size_t simb_state_bytes(int32_t n_chips, int64_t n_patches) {
  if (n_chips < 1 || n_patches < n_chips) return 0;
  return align_up((size_t)n_patches * sizeof(LaunchEntry), 256);
}

int simb_create(sim_t* const* chips, int32_t n, int32_t block, void* dev_mem, size_t bytes, void* stream, simb_t** out) {
  if (!out || !chips || n < 1 || !dev_mem || block < 0 || block > 256 || block % 64) return SIM_EINVAL;
  *out = nullptr;
  int64_t entries = 0;
  int32_t bmax = 0;
  bool multi = false;
  for (int i = 0; i < n; ++i) {
    if (!chips[i]) return SIM_EINVAL;
    entries += chips[i]->hd.n_patches;
    bmax = std::max(bmax, chips[i]->block);
    multi = multi || chips[i]->hd.n_patches > 1;
  }
  if (bytes < simb_state_bytes(n, entries)) return SIM_ENOMEM;
  if (entries > 0x7FFFFFFF) return SIM_EINVAL;
  const int32_t blk = block ? block : bmax;
  if (multi && entries > resident_limit(blk)) return SIM_EINVAL;
  sim_group* g = new (std::nothrow) sim_group();
  if (!g) return SIM_ENOMEM;
  g->chips.assign(chips, chips + n);
  g->block = blk;
  g->multi = multi;
  g->stream = static_cast<hipStream_t>(stream);
  g->table_dev = static_cast<LaunchEntry*>(dev_mem);
  g->n_entries = entries;
  if (hipHostMalloc(reinterpret_cast<void**>(&g->table_host), (size_t)entries * sizeof(LaunchEntry), hipHostMallocDefault) != hipSuccess) {
    delete g;
    return SIM_EHIP;
  }
  int64_t e = 0;
  for (int i = 0; i < n; ++i) {
    g->first_entry.push_back((int32_t)e);
    for (int p = 0; p < chips[i]->hd.n_patches; ++p) g->table_host[e++] = LaunchEntry{chips[i]->dd, p, 0};
  }
  *out = g;
  return SIM_OK;
}

int simb_step(simb_t* g, const int64_t* cycles) {
  if (!g || !cycles) return SIM_EINVAL;
  int64_t longest = 0;
  int chunk = 1 << 30;
  for (size_t i = 0; i < g->chips.size(); ++i) {
    if (cycles[i] < 0 || g->chips[i]->cycle + cycles[i] > 0x7FFFFFFFll) return SIM_EINVAL;
    longest = std::max(longest, cycles[i]);
    chunk = std::min(chunk, g->chips[i]->chunk);
  }
  if (!longest) return SIM_OK;
  for (size_t i = 0; i < g->chips.size(); ++i) {
    sim_chip* h = g->chips[i];
    const int stop = (int)(h->cycle + cycles[i]);
    for (int p = 0; p < h->hd.n_patches; ++p) g->table_host[g->first_entry[i] + p].stop = stop;
  }
  HIPCHECK(hipMemcpyAsync(g->table_dev, g->table_host, (size_t)g->n_entries * sizeof(LaunchEntry), hipMemcpyHostToDevice, g->stream));
  const int launches = (int)((longest + chunk - 1) / chunk);
  for (int i = 0; i < launches; ++i) {
    int rc = launch_entries(g->table_dev, g->n_entries, g->multi, g->block, chunk, nullptr, 0, g->stream);
    if (rc) return rc;
  }
  for (size_t i = 0; i < g->chips.size(); ++i) g->chips[i]->cycle += cycles[i];
  HIPCHECK(hipStreamSynchronize(g->stream));
  for (size_t i = 0; i < g->chips.size(); ++i) {
    int32_t err = 0;
    HIPCHECK(hipMemcpy(&err, g->chips[i]->hd.err, sizeof err, hipMemcpyDeviceToHost));
    if (err) return SIM_EHANG;
  }
  return SIM_OK;
}

int simb_destroy(simb_t* g) {
  if (!g) return SIM_EINVAL;
  (void)hipStreamSynchronize(g->stream);
  (void)hipHostFree(g->table_host);
  delete g;
  return SIM_OK;
}

}  // extern "C"
