// sfmm_api.hip -- the C ABI of libsfmm.so (declared in include/sfmm.h):
// argument checks, the context's workspace and the order of the phases.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sfmm.h"
#include "sfmm_internal.h"

using namespace sfmm;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// every device buffer of a context, grown on demand and reused
enum BufId {
  B_BOXPART, B_BOX, B_STATUS, B_SMALL,
  B_KEY0, B_KEY1, B_VAL0, B_VAL1, B_HIST, B_SCANTMP,
  B_XS, B_YS, B_ZS, B_MS, B_HS, B_HIS, B_P4,
  B_KFIRST, B_KLAST, B_KLEFT, B_KRIGHT, B_KPAR, B_KSIDE, B_KEPT,
  B_LFLAG, B_LAT, B_INFO, B_REC, B_L2BITS, B_CHUNK,
  B_LEAFNODE, B_LEAFDEPTH, B_PLEAF,
  B_LDOFF, B_DEPTHCNT, B_M2LCNT, B_P2PCNT, B_PAIRCNT, B_M2L, B_P2P,
  B_FAR, B_MOMPART, B_MOM, B_L2LCNT,
  B_NDEPTH, B_LEVKEY0, B_LEVKEY1, B_LEVIDS, B_LEVOFF, B_LEVNODES, B_LEVINT, B_M2LORD,
  B_NM2LOFF, B_NM2LCNT, B_NOPENOFF, B_NOPENCNT, B_NP2POFF, B_NP2PCNT,
  B_M2LPOOL, B_NEXP, B_P2PPOOL, B_WALKTOT,
  B_REC32, B_PF32, B_PH32,
  B_SYSOFF, B_BOXES, B_SYS, B_SYSS, B_SYSSTART, B_SKEY0, B_SKEY1, B_SPOS0, B_SPOS1, B_NFLAG,
  B_LN, B_ITEMCNT, B_ITEMOFF, B_ITEMLEAF, B_ITEMK, B_PART, B_SRCTOT, B_SOFTCNT, B_ITEME0, B_ITEMC0, B_EXTMAP,
  B_LWM2LCNT, B_LWP2PCNT, B_LWM2LOFF, B_LWP2POFF, B_DIRPART, B_OVFLEAF, B_BIGPLAIN,
  B_COUNT
};

// small device scalars (B_SMALL, u64 slots)
enum SmallId { S_NKEPT = 0, S_NLEAVES, S_MAXDEPTH, S_NITEMS, S_M2LTOT, S_P2PTOT, S_PAIRTOT,
               S_DOFFTOT, S_SORTTOT, S_L2LTOT, S_COUNT };

}  // namespace

// The small device values each synchronisation of a solve reads back, in one
// pinned host block per context: the copies are then plain asynchronous
// transfers instead of staged copies into pageable memory.
struct Readback {
  uint64_t small[S_COUNT];
  int status[4];
  uint32_t level_off[kMaxDepthCap + 2];
  uint32_t level_int[kMaxDepthCap + 2];
  uint64_t walk_tot[11 + kXcds];
  uint32_t items;
};

struct sfmm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  sfmm_config cfg{};
  std::string err;
  DevBuf buf[B_COUNT];
  // tree state of the last build
  int64_t n = 0;
  int order = -1;
  int64_t nn = 0, nleaves = 0;
  int maxdepth = 0;
  uint64_t m2l_total = 0, p2p_total = 0, pair_total = 0, l2l_total = 0;
  uint64_t m2l_unique = 0;  // level walk: entries of all per-node M2L lists
  // phase timing: SFMM_NUM_PHASES event pairs per timed solve
  std::vector<hipEvent_t> events;
  int timing_cap = 0, timing_used = 0;
  bool timing = false;
  hipEvent_t order_ev = nullptr;  // orders work across a stream change
  // level walk: nodes per depth (host copy) and pool capacities
  std::vector<uint32_t> level_off;
  std::vector<uint32_t> level_int;  // end of each level's internal nodes
  uint64_t m2l_cap = 0, p2p_cap = 0;
  int64_t items_from_walk = 0;  // P2P work items counted by the level walk
  uint32_t stack_cap = 0;
  // per-leaf list slots of the level walk (entries; doubled, up to kSlotMax,
  // while more than 1/32 of the leaves outgrow them), and nbig large slots
  // for the leaves that do (the last walk's longest lists and an eighth more)
  uint32_t slot_m = 512, slot_p = 384;
  uint32_t nbig = 64, big_m = 4096, big_p = 4096;
  // slots of the internal nodes' regions (doubled, up to kIntSlotMax, while
  // more than 1/32 of the internal nodes need the arena) and the arena
  uint32_t int_slot = 256;
  uint64_t int_big = 1u << 16;
  // the last walk's slots, leaves that overflowed them, longest leaf lists
  uint32_t walk_slot_m = 0, walk_slot_p = 0;
  uint64_t leaf_overflow = 0, max_leaf_m = 0, max_leaf_p = 0;
  bool stats_pending = false;  // level walk: totals still on the device
  int nsys = 1;                // systems of the last build (a forest when > 1)
  int near_variant = 0;        // kernel shape of P2P (SFMM_NEAR_VARIANT)
  bool have_tree = false, have_lists = false, have_mom = false;
  // clear the list pools before each walk and check every list entry after
  // it (SFMM_CHECK_POOLS=1; for tests)
  bool check_pools = false;
  uint64_t pool_init = 0;  // first pool size in entries (SFMM_POOL_INIT; 0 = estimate)
  int walk_attempts = 0;   // walks made by the last solve (pools grown in between)
  sfmm_stats stats{};
  Readback* rb = nullptr;  // pinned host block for the read-backs
  // near field beside the far field (SFMM_OVERLAP): the P2P kernel runs on a
  // second stream of the context while the far field runs on `stream`; the
  // reduction waits for both (0 off, 1 P2P queued first, 2 far field first)
  int overlap = 0;
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};

namespace {

int fail(sfmm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

// Wait for the work queued on s.  The waits inside a solve are short (the
// read-backs of list and tree sizes), and a blocking wait's wake-up costs
// tens of microseconds, during which the queue is empty and the GPU idles:
// poll for up to 2 ms, then block.
hipError_t wait_stream(hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2))
      return hipStreamSynchronize(s);
  }
}

// the context's pinned read-back block (allocated on first use; null when
// the allocation fails)
Readback* readback(sfmm_ctx* ctx) {
  if (!ctx->rb) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(Readback), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ctx->rb = static_cast<Readback*>(p);
  }
  return ctx->rb;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, SFMM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// make buffer `id` hold at least `bytes`; contents are not preserved
int ensure(sfmm_ctx* ctx, int id, size_t bytes) {
  DevBuf& b = ctx->buf[id];
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return SFMM_OK;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    (void)e;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 4;  // grow with slack
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, SFMM_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  b.cap = want;
  return SFMM_OK;
}

template <typename T>
T* P(sfmm_ctx* ctx, int id) {
  return static_cast<T*>(ctx->buf[id].p);
}

void free_events(sfmm_ctx* ctx) {
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  ctx->events.clear();
  ctx->timing = false;
  ctx->timing_cap = ctx->timing_used = 0;
}

// the event of a phase's start (end = 0) or end of this solve, null when
// the solve is not timed
hipEvent_t phase_event(sfmm_ctx* ctx, int phase, int end) {
  if (!ctx->timing || ctx->timing_used >= ctx->timing_cap) return nullptr;
  return ctx->events[(size_t)ctx->timing_used * 2 * SFMM_NUM_PHASES + 2 * phase + end];
}

void phase_mark(sfmm_ctx* ctx, int phase, int end) {
  if (hipEvent_t e = phase_event(ctx, phase, end)) (void)hipEventRecord(e, ctx->stream);
}

int set_device(sfmm_ctx* ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  return SFMM_OK;
}

int do_build(sfmm_ctx* ctx, int64_t n64, const double* x, const double* m, const double* h,
             int order, int nsys = 1, const int64_t* offsets = nullptr) {
  if (n64 < 0 || n64 >= (int64_t(1) << 30)) return fail(ctx, SFMM_EINVAL, "n out of range");
  if (order < 0 || order > kMaxOrder) return fail(ctx, SFMM_EINVAL, "order must be 0..4");
  ctx->have_tree = ctx->have_lists = ctx->have_mom = ctx->stats_pending = false;
  ctx->n = n64;
  ctx->order = order;
  ctx->nsys = nsys;
  if (n64 == 0) {
    ctx->nn = ctx->nleaves = 0;
    ctx->maxdepth = 0;
    ctx->have_tree = true;
    return SFMM_OK;
  }
  if (!x || !m || !h) return fail(ctx, SFMM_EINVAL, "NULL particle array");
  int rc;
  if ((rc = set_device(ctx))) return rc;
  const int n = (int)n64;
  const hipStream_t s = ctx->stream;
  const int leaf_size = ctx->cfg.leaf_size;
  const int RS = rec_stride(order);
  const int nmax_nodes = 2 * n;  // 1 + 2 * (kept internal) <= 2n - 1
  // ---- workspace
  struct { int id; size_t bytes; } need[] = {
      {B_BOXPART, sizeof(double) * 6 * bbox_blocks(n)}, {B_BOX, sizeof(double) * 8},
      {B_STATUS, sizeof(int) * 4}, {B_SMALL, sizeof(uint64_t) * S_COUNT},
      {B_KEY0, sizeof(uint64_t) * n}, {B_KEY1, sizeof(uint64_t) * n},
      {B_VAL0, sizeof(uint32_t) * n}, {B_VAL1, sizeof(uint32_t) * n},
      {B_HIST, sizeof(uint32_t) * 256 * (size_t)radix_blocks(n)},
      {B_SCANTMP, sizeof(uint64_t) * scan_tmp_elems(std::max<int64_t>(256 * (int64_t)radix_blocks(n), 2 * (int64_t)n + 2))},
      {B_XS, sizeof(double) * n}, {B_YS, sizeof(double) * n}, {B_ZS, sizeof(double) * n},
      {B_MS, sizeof(double) * n}, {B_HS, sizeof(double) * n}, {B_HIS, sizeof(double) * n},
      {B_P4, sizeof(double) * 4 * n},
      {B_KFIRST, sizeof(int32_t) * n}, {B_KLAST, sizeof(int32_t) * n},
      {B_KLEFT, sizeof(int32_t) * n}, {B_KRIGHT, sizeof(int32_t) * n},
      {B_KPAR, sizeof(int32_t) * n}, {B_KSIDE, sizeof(int32_t) * n},
      {B_KEPT, sizeof(uint32_t) * (n + 1)},
      {B_LFLAG, sizeof(uint32_t) * (n + 1)}, {B_LAT, sizeof(int32_t) * n},
      {B_INFO, sizeof(NodeInfo) * nmax_nodes}, {B_REC, sizeof(double) * RS * (size_t)nmax_nodes},
      {B_L2BITS, sizeof(uint64_t) * nmax_nodes},
      {B_CHUNK, sizeof(uint32_t) * (nmax_nodes + 1)},
      {B_LEAFNODE, sizeof(int32_t) * n}, {B_LEAFDEPTH, sizeof(int32_t) * n},
      {B_PLEAF, sizeof(int32_t) * n},
  };
  for (auto& q : need)
    if ((rc = ensure(ctx, q.id, q.bytes))) return rc;
  int* status = P<int>(ctx, B_STATUS);
  uint64_t* small = P<uint64_t>(ctx, B_SMALL);
  phase_mark(ctx, 0, 0);
  HIPCHK(hipMemsetAsync(status, 0, sizeof(int) * 4, s));
  HIPCHK(hipMemsetAsync(small, 0, sizeof(uint64_t) * S_COUNT, s));
  // ---- keys, sort, gather
  const uint32_t* sys_sorted = nullptr;
  const int32_t* sys_start = nullptr;
  if (nsys <= 1) {
    launch_bbox(n, x, m, h, P<double>(ctx, B_BOXPART), P<double>(ctx, B_BOX), status,
                ctx->cfg.check_inputs, s);
    launch_keys(n, x, P<double>(ctx, B_BOX), P<uint64_t>(ctx, B_KEY0), P<uint32_t>(ctx, B_VAL0), s);
    radix_sort(n, P<uint64_t>(ctx, B_KEY0), P<uint32_t>(ctx, B_VAL0), P<uint64_t>(ctx, B_KEY1),
               P<uint32_t>(ctx, B_VAL1), P<uint32_t>(ctx, B_HIST), P<uint32_t>(ctx, B_SCANTMP),
               reinterpret_cast<uint32_t*>(small + S_SORTTOT), s);
  } else {
    // several systems: each keyed in its own box, sorted by (system, key, index)
    struct { int id; size_t bytes; } need1[] = {
        {B_SYSOFF, sizeof(int64_t) * (nsys + 1)}, {B_BOXES, sizeof(double) * 8 * nsys},
        {B_SYS, sizeof(uint32_t) * n}, {B_SYSS, sizeof(uint32_t) * n},
        {B_SYSSTART, sizeof(int32_t) * nsys}, {B_SKEY0, sizeof(uint64_t) * n},
        {B_SKEY1, sizeof(uint64_t) * n}, {B_SPOS0, sizeof(uint32_t) * n},
        {B_SPOS1, sizeof(uint32_t) * n}};
    for (auto& q : need1)
      if ((rc = ensure(ctx, q.id, q.bytes))) return rc;
    HIPCHK(hipMemcpyAsync(P<int64_t>(ctx, B_SYSOFF), offsets, sizeof(int64_t) * (nsys + 1),
                          hipMemcpyHostToDevice, s));
    launch_sys_keys(n, nsys, P<int64_t>(ctx, B_SYSOFF), x, m, h, P<double>(ctx, B_BOXES), status,
                    ctx->cfg.check_inputs, P<uint64_t>(ctx, B_KEY0), P<uint32_t>(ctx, B_VAL0),
                    P<uint32_t>(ctx, B_SYS), P<int32_t>(ctx, B_SYSSTART), s);
    radix_sort(n, P<uint64_t>(ctx, B_KEY0), P<uint32_t>(ctx, B_VAL0), P<uint64_t>(ctx, B_KEY1),
               P<uint32_t>(ctx, B_VAL1), P<uint32_t>(ctx, B_HIST), P<uint32_t>(ctx, B_SCANTMP),
               reinterpret_cast<uint32_t*>(small + S_SORTTOT), s);
    launch_sys_sortkey(n, P<uint32_t>(ctx, B_VAL0), P<uint32_t>(ctx, B_SYS), P<uint64_t>(ctx, B_SKEY0),
                       P<uint32_t>(ctx, B_SPOS0), s);
    uint64_t *ka = P<uint64_t>(ctx, B_SKEY0), *kb = P<uint64_t>(ctx, B_SKEY1);
    uint32_t *va = P<uint32_t>(ctx, B_SPOS0), *vb = P<uint32_t>(ctx, B_SPOS1);
    for (int shift = 0; shift < 32 && ((uint64_t)(nsys - 1) >> shift) != 0; shift += 8) {
      radix_pass(n, ka, va, kb, vb, shift, P<uint32_t>(ctx, B_HIST), P<uint32_t>(ctx, B_SCANTMP),
                 reinterpret_cast<uint32_t*>(small + S_SORTTOT), s);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
    // final permutation and keys into the spare buffers, then back in place
    launch_sys_final(n, va, P<uint32_t>(ctx, B_VAL0), P<uint64_t>(ctx, B_KEY0), P<uint32_t>(ctx, B_SYS),
                     vb, kb, P<uint32_t>(ctx, B_SYSS), s);
    HIPCHK(hipMemcpyAsync(P<uint32_t>(ctx, B_VAL0), vb, sizeof(uint32_t) * n,
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(P<uint64_t>(ctx, B_KEY0), kb, sizeof(uint64_t) * n,
                          hipMemcpyDeviceToDevice, s));
    sys_sorted = P<uint32_t>(ctx, B_SYSS);
    sys_start = P<int32_t>(ctx, B_SYSSTART);
  }
  const uint64_t* key = P<uint64_t>(ctx, B_KEY0);
  const uint32_t* perm = P<uint32_t>(ctx, B_VAL0);
  launch_gather(n, perm, x, m, h, P<double>(ctx, B_XS), P<double>(ctx, B_YS), P<double>(ctx, B_ZS),
                P<double>(ctx, B_MS), P<double>(ctx, B_HS), P<double>(ctx, B_HIS),
                P<double>(ctx, B_P4), s);
  NodeInfo* info = P<NodeInfo>(ctx, B_INFO);
  int32_t* leaf_node = P<int32_t>(ctx, B_LEAFNODE);
  // ---- topology
  if (n <= leaf_size && nsys <= 1) {
    launch_single_leaf(n, info, leaf_node, s);
  } else {
    launch_karras(n, key, sys_sorted, sys_start, leaf_size, P<int32_t>(ctx, B_KFIRST), P<int32_t>(ctx, B_KLAST),
                  P<int32_t>(ctx, B_KLEFT), P<int32_t>(ctx, B_KRIGHT), P<int32_t>(ctx, B_KPAR),
                  P<int32_t>(ctx, B_KSIDE), P<uint32_t>(ctx, B_KEPT), s);
    uint32_t* cidx = P<uint32_t>(ctx, B_KEPT);
    scan_u32(cidx, cidx, n - 1, reinterpret_cast<uint32_t*>(small + S_NKEPT),
             P<uint32_t>(ctx, B_SCANTMP), s);
    HIPCHK(hipMemsetAsync(P<uint32_t>(ctx, B_LFLAG), 0, sizeof(uint32_t) * (n + 1), s));
    launch_assign(n, leaf_size, sys_sorted, P<int32_t>(ctx, B_KFIRST), P<int32_t>(ctx, B_KLAST),
                  P<int32_t>(ctx, B_KLEFT), P<int32_t>(ctx, B_KRIGHT), P<int32_t>(ctx, B_KPAR),
                  P<int32_t>(ctx, B_KSIDE), cidx, info, P<uint32_t>(ctx, B_LFLAG),
                  P<int32_t>(ctx, B_LAT), s);
    // leaf_flag -> leaf index (scan into KFIRST's storage, no longer needed)
    uint32_t* lscan = reinterpret_cast<uint32_t*>(P<int32_t>(ctx, B_KFIRST));
    scan_u32(P<uint32_t>(ctx, B_LFLAG), lscan, n, reinterpret_cast<uint32_t*>(small + S_NLEAVES),
             P<uint32_t>(ctx, B_SCANTMP), s);
    launch_leaf_fill(n, P<uint32_t>(ctx, B_LFLAG), lscan, P<int32_t>(ctx, B_LAT), leaf_node, s);
  }
  // ---- sizes to the host (one synchronisation)
  Readback* hb = readback(ctx);
  if (!hb) return fail(ctx, SFMM_ENOMEM, "pinned host block for read-backs");
  const uint64_t* hsmall = hb->small;
  HIPCHK(hipMemcpyAsync(hb->small, small, sizeof(hb->small), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hb->status, status, sizeof(hb->status), hipMemcpyDeviceToHost, s));
  HIPCHK(wait_stream(s));
  if (hb->status[0] & ST_NONFINITE)
    return fail(ctx, SFMM_ENONFINITE, "non-finite position or non-positive m/h");
  if (n <= leaf_size && nsys <= 1) {
    ctx->nn = 1;
    ctx->nleaves = 1;
  } else {
    const uint32_t nkept = (uint32_t)(hsmall[S_NKEPT] & 0xffffffffu);
    ctx->nn = 1 + 2 * (int64_t)nkept;
    ctx->nleaves = (int64_t)(hsmall[S_NLEAVES] & 0xffffffffu);
  }
  // interaction-list entries carry a node index in kSrcBits bits
  if (ctx->nn > (int64_t)kSrcMask + 1)
    return fail(ctx, SFMM_EUNSUPPORTED, "tree has more than 2^25 nodes");
  const int nn = (int)ctx->nn, nl = (int)ctx->nleaves;
  // node depths and nodes grouped by depth (level walk): one stable radix
  // pass on the depth
  {
    struct { int id; size_t bytes; } need2[] = {
        {B_NDEPTH, sizeof(int32_t) * nn}, {B_LEVNODES, sizeof(uint32_t) * nn},
        {B_LEVKEY0, sizeof(uint64_t) * nn}, {B_LEVKEY1, sizeof(uint64_t) * nn},
        {B_LEVIDS, sizeof(uint32_t) * nn}, {B_LEVOFF, sizeof(uint32_t) * (kMaxDepthCap + 2)},
        {B_LEVINT, sizeof(uint32_t) * (kMaxDepthCap + 2)},
        {B_HIST, sizeof(uint32_t) * 256 * (size_t)radix_blocks(nn)},
        {B_SCANTMP, sizeof(uint64_t) * scan_tmp_elems(std::max<int64_t>(256 * (int64_t)radix_blocks(nn), 2 * (int64_t)n + 2))}};
    for (auto& q : need2)
      if ((rc = ensure(ctx, q.id, q.bytes))) return rc;
    launch_node_depth(nn, info, P<int32_t>(ctx, B_NDEPTH), P<uint64_t>(ctx, B_LEVKEY0),
                      P<uint32_t>(ctx, B_LEVIDS), s);
    radix_pass(nn, P<uint64_t>(ctx, B_LEVKEY0), P<uint32_t>(ctx, B_LEVIDS),
               P<uint64_t>(ctx, B_LEVKEY1), P<uint32_t>(ctx, B_LEVNODES), 0,
               P<uint32_t>(ctx, B_HIST), P<uint32_t>(ctx, B_SCANTMP),
               reinterpret_cast<uint32_t*>(small + S_SORTTOT), s);
    launch_level_offsets(kMaxDepthCap + 1, radix_blocks(nn), nn, P<uint32_t>(ctx, B_HIST),
                         P<uint32_t>(ctx, B_LEVOFF), P<uint32_t>(ctx, B_LEVINT), s);
  }
  if (nsys > 1) {
    if ((rc = ensure(ctx, B_NFLAG, sizeof(uint8_t) * nn))) return rc;
    launch_node_flags(nn, info, sys_sorted, P<uint8_t>(ctx, B_NFLAG), s);
  }
  int* maxd_dev = reinterpret_cast<int*>(small + S_MAXDEPTH);
  launch_leaf_depth(nl, leaf_node, info, P<int32_t>(ctx, B_NDEPTH), P<int32_t>(ctx, B_LEAFDEPTH),
                    P<int32_t>(ctx, B_PLEAF), maxd_dev, s);
  if (nn > 1) {
    uint32_t* chunk = P<uint32_t>(ctx, B_CHUNK);
    launch_extent_count(nn, info, chunk, s);
    scan_u32(chunk, chunk, nn, reinterpret_cast<uint32_t*>(small + S_NITEMS),
             P<uint32_t>(ctx, B_SCANTMP), s);
    HIPCHK(hipMemsetAsync(P<uint64_t>(ctx, B_L2BITS), 0, sizeof(uint64_t) * nn, s));
  }
  HIPCHK(hipMemcpyAsync(hb->small, small, sizeof(hb->small), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hb->level_off, P<uint32_t>(ctx, B_LEVOFF), sizeof(hb->level_off),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hb->level_int, P<uint32_t>(ctx, B_LEVINT), sizeof(hb->level_int),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(wait_stream(s));
  ctx->level_off.assign(hb->level_off, hb->level_off + kMaxDepthCap + 2);
  ctx->level_int.assign(hb->level_int, hb->level_int + kMaxDepthCap + 2);
  ctx->maxdepth = (int)(hsmall[S_MAXDEPTH] & 0x7fffffff);
  if (ctx->maxdepth > kMaxDepthCap) return fail(ctx, SFMM_EUNSUPPORTED, "tree deeper than 127");
  // ---- geometry and moments, level by level from the deepest
  launch_geometry(order, ctx->maxdepth, ctx->level_off.data(), P<uint32_t>(ctx, B_LEVOFF),
                  reinterpret_cast<const int32_t*>(P<uint32_t>(ctx, B_LEVNODES)), info,
                  P<double>(ctx, B_XS), P<double>(ctx, B_YS), P<double>(ctx, B_ZS),
                  P<double>(ctx, B_MS), P<double>(ctx, B_HS), P<double>(ctx, B_REC), s);
  if (nn > 1) {
    const int nitems = (int)(hsmall[S_NITEMS] & 0xffffffffu);
    if ((rc = ensure(ctx, B_EXTMAP, sizeof(uint32_t) * (size_t)std::max(nitems, 1)))) return rc;
    launch_extent(order, nn, nitems, info, P<uint32_t>(ctx, B_CHUNK), P<uint32_t>(ctx, B_EXTMAP),
                  P<double>(ctx, B_XS),
                  P<double>(ctx, B_YS), P<double>(ctx, B_ZS), P<double>(ctx, B_REC),
                  reinterpret_cast<unsigned long long*>(P<uint64_t>(ctx, B_L2BITS)), s);
    launch_extent_final(order, nn, info, reinterpret_cast<unsigned long long*>(P<uint64_t>(ctx, B_L2BITS)),
                        P<double>(ctx, B_REC), s);
  }
  phase_mark(ctx, 0, 1);
  HIPCHK(hipGetLastError());
  ctx->have_tree = true;
  return SFMM_OK;
}

// Algorithm 1 per leaf: count pass, list sizes to the host, fill pass
int walk_per_leaf(sfmm_ctx* ctx, double theta) {
  int rc;
  const hipStream_t s = ctx->stream;
  const int nl = (int)ctx->nleaves;
  uint64_t* small = P<uint64_t>(ctx, B_SMALL);
  int* status = P<int>(ctx, B_STATUS);
  uint64_t* ldoff = P<uint64_t>(ctx, B_LDOFF);
  launch_leaf_doff(nl, P<int32_t>(ctx, B_LEAFDEPTH), ldoff, s);
  scan_u64(ldoff, ldoff, nl, small + S_DOFFTOT, P<uint64_t>(ctx, B_SCANTMP), s);
  // depth counts need sum(d+1) <= nl * (maxdepth + 1)
  if ((rc = ensure(ctx, B_DEPTHCNT, sizeof(uint32_t) * (size_t)nl * (ctx->maxdepth + 1))))
    return rc;
  WalkArgs w{};
  w.nleaves = nl;
  w.leaf_node = P<int32_t>(ctx, B_LEAFNODE);
  w.leaf_depth = P<int32_t>(ctx, B_LEAFDEPTH);
  w.info = P<NodeInfo>(ctx, B_INFO);
  w.rec = P<double>(ctx, B_REC);
  w.stride = rec_stride(ctx->order);
  w.theta2 = theta * theta;
  w.r_kern = ctx->cfg.r_kern;
  w.leaf_doff = ldoff;
  w.depth_cnt = P<uint32_t>(ctx, B_DEPTHCNT);
  w.m2l_cnt = P<uint64_t>(ctx, B_M2LCNT);
  w.p2p_cnt = P<uint64_t>(ctx, B_P2PCNT);
  w.pair_cnt = P<uint64_t>(ctx, B_PAIRCNT);
  w.l2l_cnt = P<uint64_t>(ctx, B_L2LCNT);
  w.status = status;
  launch_walk(w, ctx->maxdepth, false, s);
  scan_u64(w.m2l_cnt, w.m2l_cnt, nl, small + S_M2LTOT, P<uint64_t>(ctx, B_SCANTMP), s);
  scan_u64(w.p2p_cnt, w.p2p_cnt, nl, small + S_P2PTOT, P<uint64_t>(ctx, B_SCANTMP), s);
  scan_u64(w.pair_cnt, w.pair_cnt, nl, small + S_PAIRTOT, P<uint64_t>(ctx, B_SCANTMP), s);
  scan_u64(w.l2l_cnt, w.l2l_cnt, nl, small + S_L2LTOT, P<uint64_t>(ctx, B_SCANTMP), s);
  // the totals also close the offset arrays: off[nl] = total
  HIPCHK(hipMemcpyAsync(w.m2l_cnt + nl, small + S_M2LTOT, sizeof(uint64_t),
                        hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(w.p2p_cnt + nl, small + S_P2PTOT, sizeof(uint64_t),
                        hipMemcpyDeviceToDevice, s));
  phase_mark(ctx, 1, 1);
  Readback* hb = readback(ctx);
  if (!hb) return fail(ctx, SFMM_ENOMEM, "pinned host block for read-backs");
  const uint64_t* hsmall = hb->small;
  HIPCHK(hipMemcpyAsync(hb->small, small, sizeof(hb->small), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hb->status, status, sizeof(hb->status), hipMemcpyDeviceToHost, s));
  HIPCHK(wait_stream(s));
  if (hb->status[0] & (ST_DEPTH | ST_OVERFLOW))
    return fail(ctx, SFMM_EDEVICE, "walk stack overflow (tree depth)");
  ctx->m2l_total = hsmall[S_M2LTOT];
  ctx->p2p_total = hsmall[S_P2PTOT];
  ctx->pair_total = hsmall[S_PAIRTOT];
  ctx->l2l_total = hsmall[S_L2LTOT];
  if ((rc = ensure(ctx, B_M2L, sizeof(uint32_t) * ctx->m2l_total))) return rc;
  if ((rc = ensure(ctx, B_P2P, sizeof(int32_t) * ctx->p2p_total))) return rc;
  w.m2l_list = P<uint32_t>(ctx, B_M2L);
  w.p2p_list = P<int32_t>(ctx, B_P2P);
  phase_mark(ctx, 2, 0);
  launch_walk(w, ctx->maxdepth, true, s);
  phase_mark(ctx, 2, 1);
  return SFMM_OK;
}

// per-leaf P2P item buffers (source totals, item counts, item offsets)
int ensure_item_buffers(sfmm_ctx* ctx) {
  int rc;
  const size_t nl = (size_t)std::max<int64_t>(ctx->nleaves, 1);
  if ((rc = ensure(ctx, B_SRCTOT, sizeof(uint32_t) * nl))) return rc;
  if ((rc = ensure(ctx, B_ITEMCNT, sizeof(uint32_t) * nl))) return rc;
  if ((rc = ensure(ctx, B_ITEMOFF, sizeof(uint32_t) * (nl + 1)))) return rc;
  return SFMM_OK;
}

// level-synchronous walk: one launch per depth; pools grow and the walk is
// repeated if a list pool or a lowering stack was too small
int walk_levels(sfmm_ctx* ctx, double theta) {
  int rc;
  const hipStream_t s = ctx->stream;
  const int nn = (int)ctx->nn, nl = (int)ctx->nleaves;
  uint64_t* small = P<uint64_t>(ctx, B_SMALL);
  int* status = P<int>(ctx, B_STATUS);
  const int node_arrays[] = {B_NM2LOFF, B_NM2LCNT, B_NOPENOFF, B_NOPENCNT, B_NP2POFF, B_NP2PCNT,
                             B_NEXP};
  for (int id : node_arrays)
    if ((rc = ensure(ctx, id, sizeof(uint32_t) * nn))) return rc;
  if ((rc = ensure(ctx, B_WALKTOT, sizeof(uint64_t) * (11 + kXcds)))) return rc;
  if ((rc = ensure_item_buffers(ctx))) return rc;
  for (int id : {B_LWM2LCNT, B_LWP2PCNT, B_OVFLEAF})
    if ((rc = ensure(ctx, id, sizeof(uint32_t) * std::max(nl, 1)))) return rc;
  for (int id : {B_LWM2LOFF, B_LWP2POFF})
    if ((rc = ensure(ctx, id, sizeof(uint64_t) * std::max(nl, 1)))) return rc;
  // pools keep the size of the largest walk so far, and never start below a
  // per-node estimate for this tree (a context may go from a small system to
  // a large one)
  // (the M2L pool also holds the opened lists of internal nodes)
  // (SFMM_POOL_INIT: start from that many entries instead, so that tests
  // meet pools too small for the walk)
  // (the leaves' slots come first in the estimates, then the internal
  // nodes' regions and the lists that overflow their slots)
  const uint32_t int_nodes = (uint32_t)(nn - nl);
  const uint64_t est_m = ctx->pool_init ? ctx->pool_init
                                         : (uint64_t)ctx->slot_m * nl +
                                               (uint64_t)ctx->nbig * ctx->big_m +
                                               (uint64_t)ctx->int_slot * int_nodes + ctx->int_big +
                                               8ull * nl + 2048;
  const uint64_t est_p = ctx->pool_init ? ctx->pool_init
                                         : (uint64_t)ctx->slot_p * nl +
                                               (uint64_t)ctx->nbig * ctx->big_p + 8ull * nl + 1024;
  ctx->m2l_cap = std::min(kPoolMax, std::max<uint64_t>(ctx->m2l_cap, est_m));
  ctx->p2p_cap = std::min(kPoolMax, std::max<uint64_t>(ctx->p2p_cap, est_p));
  const uint32_t stack_min = (uint32_t)std::min(16384, 64 * (ctx->maxdepth + 4) + 256);
  if (ctx->stack_cap < stack_min) ctx->stack_cap = stack_min;
  for (int attempt = 0;; ++attempt) {
    // the leaf kernel's LDS (stack and staged P2P entries) stays within 64 KB
    const uint32_t slot_m = ctx->slot_m;
    const uint32_t slot_p = std::min<uint32_t>(ctx->slot_p, 16384u - ctx->stack_cap);
    const uint32_t nbig = ctx->nbig, big_m = ctx->big_m, big_p = ctx->big_p;
    const uint32_t int_slot = ctx->int_slot;
    const uint64_t int_big = ctx->int_big;
    const uint64_t leaf_base = (uint64_t)int_slot * int_nodes + int_big;
    if ((rc = ensure(ctx, B_BIGPLAIN, sizeof(uint32_t) * (size_t)nbig * big_p))) return rc;
    ctx->walk_attempts = attempt + 1;
    if ((rc = ensure(ctx, B_M2LPOOL, sizeof(uint32_t) * ctx->m2l_cap))) return rc;
    if ((rc = ensure(ctx, B_P2PPOOL, sizeof(uint32_t) * ctx->p2p_cap))) return rc;
    uint64_t* tot = P<uint64_t>(ctx, B_WALKTOT);
    HIPCHK(hipMemsetAsync(tot, 0, sizeof(uint64_t) * (11 + kXcds), s));
    HIPCHK(hipMemsetAsync(status, 0, sizeof(int), s));
    if (ctx->check_pools) {
      // every entry a consumer reads must then come from this walk: clear
      // the pools to a value no node id takes (checked after the walk)
      HIPCHK(hipMemsetAsync(P<uint32_t>(ctx, B_M2LPOOL), 0xff, sizeof(uint32_t) * ctx->m2l_cap, s));
      HIPCHK(hipMemsetAsync(P<uint32_t>(ctx, B_P2PPOOL), 0xff, sizeof(uint32_t) * ctx->p2p_cap, s));
    }
    NodeWalkArgs a{};
    a.info = P<NodeInfo>(ctx, B_INFO);
    a.rec = P<double>(ctx, B_REC);
    a.stride = rec_stride(ctx->order);
    a.theta2 = theta * theta;
    a.r_kern = ctx->cfg.r_kern;
    a.level_nodes = P<int32_t>(ctx, B_LEVNODES);
    a.node_flag = ctx->nsys > 1 ? P<uint8_t>(ctx, B_NFLAG) : nullptr;
    a.level_off = P<uint32_t>(ctx, B_LEVOFF);
    a.level_int = P<uint32_t>(ctx, B_LEVINT);
    a.m2l_off = P<uint32_t>(ctx, B_NM2LOFF);
    a.m2l_cnt = P<uint32_t>(ctx, B_NM2LCNT);
    a.open_off = P<uint32_t>(ctx, B_NOPENOFF);
    a.open_cnt = P<uint32_t>(ctx, B_NOPENCNT);
    a.p2p_off = P<uint32_t>(ctx, B_NP2POFF);
    a.p2p_cnt = P<uint32_t>(ctx, B_NP2PCNT);
    a.m2l_pool = P<uint32_t>(ctx, B_M2LPOOL);
    a.open_pool = a.m2l_pool;
    a.exp = P<uint32_t>(ctx, B_NEXP);
    a.p2p_pool = P<uint32_t>(ctx, B_P2PPOOL);
    a.m2l_cap = ctx->m2l_cap;
    a.open_cap = a.m2l_cap;
    a.p2p_cap = ctx->p2p_cap;
    a.int_slot = int_slot;
    a.int_nodes = int_nodes;
    a.int_big = int_big;
    a.leaf_base = leaf_base;
    a.run = tot;
    a.stack_cap = ctx->stack_cap;
    a.status = status;
    a.nleaves = nl;
    a.leaf_node = P<int32_t>(ctx, B_LEAFNODE);
    a.slot_m = slot_m;
    a.slot_p = slot_p;
    a.nbig = nbig;
    a.big_m = big_m;
    a.big_p = big_p;
    a.big_plain = P<uint32_t>(ctx, B_BIGPLAIN);
    a.ovf_leaf = P<uint32_t>(ctx, B_OVFLEAF);
    a.leaf_m2l_cnt = P<uint32_t>(ctx, B_LWM2LCNT);
    a.leaf_p2p_cnt = P<uint32_t>(ctx, B_LWP2PCNT);
    a.leaf_m2l_off = P<uint64_t>(ctx, B_LWM2LOFF);
    a.leaf_p2p_off = P<uint64_t>(ctx, B_LWP2POFF);
    a.src_total = P<uint32_t>(ctx, B_SRCTOT);
    a.item_cnt = P<uint32_t>(ctx, B_ITEMCNT);
    a.item_off = P<uint32_t>(ctx, B_ITEMOFF);
    // internal nodes level by level, then every leaf
    uint32_t rank0 = 0;
    for (int k = 0; k <= ctx->maxdepth; ++k) {
      const uint32_t nk = ctx->level_int[k] - ctx->level_off[k];
      launch_nodewalk_level(a, k, (int)nk, rank0, s);
      rank0 += nk;
    }
    launch_nodewalk_leaves(a, P<uint32_t>(ctx, B_SCANTMP), s);
    // no consumer reads a list unless it lies in the part of its pool this
    // walk wrote (and, when checking, holds only node ids); with the totals
    // of M2L entries proper (the pool also holds the opened lists) and P2P
    // entries, and the longest lists of a leaf
    launch_check_lists(a, nn, ctx->check_pools, s);
    Readback* hb = readback(ctx);
    if (!hb) return fail(ctx, SFMM_ENOMEM, "pinned host block for read-backs");
    const uint64_t* htot = hb->walk_tot;
    const int* hstatus = hb->status;
    hb->items = 0;
    HIPCHK(hipMemcpyAsync(hb->walk_tot, tot, sizeof(hb->walk_tot), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hb->status, status, sizeof(hb->status), hipMemcpyDeviceToHost, s));
    if (nl > 0)
      HIPCHK(hipMemcpyAsync(&hb->items, a.item_off + nl, sizeof(uint32_t), hipMemcpyDeviceToHost,
                            s));
    HIPCHK(wait_stream(s));
    ctx->items_from_walk = hb->items;
    // 64-bit totals: internal regions, the leaves' slots, then the lists that
    // overflow their slots
    const uint64_t m2l_used = leaf_base + (uint64_t)slot_m * nl + (uint64_t)nbig * big_m + htot[3];
    const uint64_t p2p_used = (uint64_t)slot_p * nl + (uint64_t)nbig * big_p + htot[2];
    const bool arena_over = htot[0] > int_big;
    const bool pool_over = m2l_used > ctx->m2l_cap || p2p_used > ctx->p2p_cap || arena_over;
    const bool stack_over = (hstatus[0] & ST_OVERFLOW) != 0;
    uint64_t ovf_total = 0;  // leaves walked a second time
    for (unsigned q = 0; q < kXcds; ++q) ovf_total += htot[11 + q];
    if (!pool_over && !stack_over) {
      if (hstatus[0] & ST_BADLIST)
        return fail(ctx, SFMM_EDEVICE, "an interaction list lies outside what the walk wrote");
      ctx->p2p_total = htot[4];
      ctx->m2l_unique = htot[1];
      ctx->walk_slot_m = slot_m;
      ctx->walk_slot_p = slot_p;
      ctx->leaf_overflow = ovf_total;
      ctx->max_leaf_m = htot[6];
      ctx->max_leaf_p = htot[7];
      // slots for the next walk: the normal ones doubled while more than
      // 1/32 of the leaves outgrow them, large ones for this walk's longest
      // lists and an eighth more, twice as many as were asked for (within
      // 2^28 entries); pools that hold them, so that walk still fits at once
      const uint64_t asked = std::max(htot[8], htot[9]);
      auto big_for = [](uint64_t longest, uint32_t slot) {
        const uint64_t w = (longest + longest / 8 + 64) / 64 * 64;
        return (uint32_t)std::min<uint64_t>(kBigSlotMax, std::max<uint64_t>(2ull * slot, w));
      };
      const uint64_t ib = std::max<uint64_t>(1u << 16, htot[0] + htot[0] / 4 + 4096);
      uint32_t sm = slot_m, sp = ctx->slot_p, is = int_slot, bm = 0, bp = 0;
      uint64_t nb = 0, need_m = 0, need_p = 0;
      auto plan = [&]() {
        bm = big_for(htot[6], sm);
        bp = big_for(htot[7], sp);
        nb = std::min<uint64_t>(std::max<uint64_t>(64, 2 * asked), std::max(nl, 64));
        nb = std::min<uint64_t>(nb, (1ull << 28) / ((uint64_t)bm + 2ull * bp));
        need_m = (uint64_t)is * int_nodes + ib + (uint64_t)sm * nl + nb * bm + htot[3];
        need_p = (uint64_t)sp * nl + nb * bp + htot[2];
      };
      // normal slots double while more than 1/32 of the leaves (or internal
      // nodes) outgrow them, unless that would fill more than half of the
      // largest pool: then this walk's slots stay
      if ((asked + ovf_total) * 32 > (uint64_t)nl) {
        sm = std::min(kSlotMax, 2 * sm);
        sp = std::min(kSlotMax / 2, 2 * sp);
      }
      if (htot[10] * 32 > (uint64_t)int_nodes) is = std::min(kIntSlotMax, 2 * is);
      plan();
      if (need_m > kPoolMax / 2 || need_p > kPoolMax / 2) {
        sm = slot_m;
        sp = ctx->slot_p;
        is = int_slot;
        plan();
      }
      ctx->slot_m = sm;
      ctx->slot_p = sp;
      ctx->int_slot = is;
      ctx->nbig = (uint32_t)nb;
      ctx->big_m = bm;
      ctx->big_p = bp;
      ctx->int_big = ib;
      ctx->m2l_cap = std::min(kPoolMax, std::max(ctx->m2l_cap, need_m));
      ctx->p2p_cap = std::min(kPoolMax, std::max(ctx->p2p_cap, need_p));
      return SFMM_OK;
    }
    if (attempt >= 16) return fail(ctx, SFMM_EUNSUPPORTED, "interaction walk did not fit");
    if (pool_over) {
      // a truncated level under-reports the levels below it, so the totals
      // are lower bounds: grow at least twofold, up to the largest pool
      auto grow = [](uint64_t cap, uint64_t need) {
        return need > cap ? std::max<uint64_t>(2 * cap, need + need / 4 + 1024) : cap;
      };
      // (a larger arena moves the leaves' slots up by as much)
      if (arena_over) ctx->int_big = std::max<uint64_t>(2 * int_big, htot[0] + htot[0] / 4 + 4096);
      const uint64_t need_m = m2l_used + (ctx->int_big - int_big);
      if ((need_m > ctx->m2l_cap && ctx->m2l_cap >= kPoolMax) ||
          (p2p_used > ctx->p2p_cap && ctx->p2p_cap >= kPoolMax)) {
        // slots that leave no room: a quarter of their size, and walk again
        if (slot_m > 16 || ctx->slot_p > 16 || int_slot > 16 || ctx->nbig > 64) {
          ctx->slot_m = std::max(16u, slot_m / 4);
          ctx->slot_p = std::max(16u, ctx->slot_p / 4);
          ctx->int_slot = std::max(16u, int_slot / 4);
          ctx->nbig = 64;
          continue;
        }
        return fail(ctx, SFMM_EUNSUPPORTED, "interaction lists exceed the largest list pool (" +
                                                std::to_string(kPoolMax) + " entries)");
      }
      ctx->m2l_cap = std::min(kPoolMax, grow(ctx->m2l_cap, need_m));
      ctx->p2p_cap = std::min(kPoolMax, grow(ctx->p2p_cap, p2p_used));
    }
    if (stack_over) {
      if (ctx->stack_cap >= 16384) return fail(ctx, SFMM_EUNSUPPORTED, "lowering stack > 64 KB");
      ctx->stack_cap = std::min<uint32_t>(16384, ctx->stack_cap * 4);
    }
  }
}

int do_walk_and_eval(sfmm_ctx* ctx, double theta, int precision, const double* m, double* acc,
                     double* pot) {
  int rc;
  const hipStream_t s = ctx->stream;
  const int n = (int)ctx->n, nl = (int)ctx->nleaves;
  uint64_t* small = P<uint64_t>(ctx, B_SMALL);
  struct { int id; size_t bytes; } need[] = {
      {B_LDOFF, sizeof(uint64_t) * (nl + 1)}, {B_M2LCNT, sizeof(uint64_t) * (nl + 1)},
      {B_P2PCNT, sizeof(uint64_t) * (nl + 1)}, {B_PAIRCNT, sizeof(uint64_t) * (nl + 1)},
      {B_L2LCNT, sizeof(uint64_t) * (nl + 1)},
      {B_FAR, sizeof(double) * 4 * (size_t)n},
      {B_MOMPART, sizeof(double) * 4 * momentum_blocks(n)}, {B_MOM, sizeof(double) * 4},
      {B_SCANTMP, sizeof(uint64_t) * scan_tmp_elems(nl + 1)},
  };
  for (auto& q : need)
    if ((rc = ensure(ctx, q.id, q.bytes))) return rc;
  const bool level = ctx->cfg.walk_mode == SFMM_WALK_LEVEL;
  if (!level && ctx->nsys > 1)
    return fail(ctx, SFMM_EUNSUPPORTED, "several systems need SFMM_WALK_LEVEL");
  // per-node lists exist only with the level walk; the per-leaf walk keeps
  // the per-leaf far field
  const bool mutual = ctx->cfg.far_mode == SFMM_FAR_MUTUAL && level;
  const bool shared = (ctx->cfg.far_mode == SFMM_FAR_SHARED || mutual) && level;
  if (mutual && precision == SFMM_FP32C)
    return fail(ctx, SFMM_EUNSUPPORTED, "SFMM_FAR_MUTUAL is FP64 only");
  if (shared && (rc = ensure(ctx, B_LN, sizeof(double) * local_count(ctx->order) * (size_t)ctx->nn)))
    return rc;
  if (shared && !mutual && (rc = ensure(ctx, B_M2LORD, sizeof(uint32_t) * (size_t)ctx->nn)))
    return rc;
  if (!level) ctx->m2l_unique = 0;
  phase_mark(ctx, 1, 0);
  if (level) {
    if ((rc = walk_levels(ctx, theta))) return rc;
    phase_mark(ctx, 1, 1);
    phase_mark(ctx, 2, 0);
    phase_mark(ctx, 2, 1);
  } else {
    if ((rc = walk_per_leaf(ctx, theta))) return rc;
  }
  ctx->have_lists = true;
  // ---- far field, near field, output
  FarArgs f{};
  f.nleaves = nl;
  f.leaf_node = P<int32_t>(ctx, B_LEAFNODE);
  f.leaf_depth = P<int32_t>(ctx, B_LEAFDEPTH);
  f.info = P<NodeInfo>(ctx, B_INFO);
  f.rec = P<double>(ctx, B_REC);
  f.m2l_off = P<uint64_t>(ctx, B_M2LCNT);
  f.m2l_list = P<uint32_t>(ctx, B_M2L);
  f.depth_cnt = P<uint32_t>(ctx, B_DEPTHCNT);
  f.leaf_doff = P<uint64_t>(ctx, B_LDOFF);
  f.node_m2l_off = P<uint32_t>(ctx, B_NM2LOFF);
  f.node_m2l_cnt = P<uint32_t>(ctx, B_NM2LCNT);
  f.node_m2l_pool = P<uint32_t>(ctx, B_M2LPOOL);
  f.xs = P<double>(ctx, B_XS);
  f.ys = P<double>(ctx, B_YS);
  f.zs = P<double>(ctx, B_ZS);
  f.far = P<double>(ctx, B_FAR);
  const bool f32 = precision == SFMM_FP32C;
  if (f32) {
    if (ctx->cfg.leaf_size > 16)
      return fail(ctx, SFMM_EUNSUPPORTED, "SFMM_FP32C needs leaf_size <= 16");
    struct { int id; size_t bytes; } need3[] = {
        {B_REC32, sizeof(float) * rec32_stride(ctx->order) * (size_t)ctx->nn},
        {B_PF32, sizeof(float4) * (size_t)n}, {B_PH32, sizeof(float2) * (size_t)n}};
    for (auto& q : need3)
      if ((rc = ensure(ctx, q.id, q.bytes))) return rc;
  }
  NearArgs a{};
  a.n = n;
  a.nleaves = nl;
  a.p_leaf = P<int32_t>(ctx, B_PLEAF);
  a.info = f.info;
  a.p2p_off = P<uint64_t>(ctx, B_P2PCNT);
  a.p2p_list = P<int32_t>(ctx, B_P2P);
  a.leaf_node = f.leaf_node;
  a.node_p2p_off = P<uint32_t>(ctx, B_NP2POFF);
  a.node_p2p_cnt = P<uint32_t>(ctx, B_NP2PCNT);
  a.node_p2p_pool = P<uint32_t>(ctx, B_P2PPOOL);
  a.xs = f.xs; a.ys = f.ys; a.zs = f.zs;
  a.ms = P<double>(ctx, B_MS);
  a.hs = P<double>(ctx, B_HS);
  a.his = P<double>(ctx, B_HIS);
  a.p4 = P<double>(ctx, B_P4);
  a.far = f.far;
  a.rec = f.rec;
  a.rec_stride = rec_stride(ctx->order);
  a.perm = P<uint32_t>(ctx, B_VAL0);
  a.G = ctx->cfg.G;
  a.include_self = ctx->cfg.include_self_potential;
  a.acc = acc;
  a.pot = pot;
  if ((rc = ensure(ctx, B_SOFTCNT, sizeof(unsigned long long)))) return rc;
  a.soft_pairs = P<unsigned long long>(ctx, B_SOFTCNT);
  // P2P work items: runs of at most kP2PItem flattened source particles of
  // one leaf; their number is read back to size the partial sums
  int64_t items = 0;
  if (ctx->cfg.leaf_size <= 32) {
    // P2P work items: the level walk has counted them (and read their total
    // back with its own totals); the per-leaf walk's lists are counted here
    if ((rc = ensure_item_buffers(ctx))) return rc;
    uint32_t* item_off = P<uint32_t>(ctx, B_ITEMOFF);
    a.src_total = P<uint32_t>(ctx, B_SRCTOT);
    a.item_off = item_off;
    if (level) {
      items = ctx->items_from_walk;
    } else {
      launch_p2p_items_count(level, a, P<uint32_t>(ctx, B_SRCTOT), P<uint32_t>(ctx, B_ITEMCNT), s);
      scan_u32(P<uint32_t>(ctx, B_ITEMCNT), item_off, nl, item_off + nl, P<uint32_t>(ctx, B_SCANTMP),
               s);
      Readback* hb = readback(ctx);
      if (!hb) return fail(ctx, SFMM_ENOMEM, "pinned host block for read-backs");
      HIPCHK(hipMemcpyAsync(&hb->items, item_off + nl, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(wait_stream(s));
      items = hb->items;
    }
    const int ls = p2p_leaf_slots(ctx->cfg.leaf_size);
    struct { int id; size_t bytes; } need5[] = {
        {B_ITEMLEAF, sizeof(int32_t) * (size_t)items}, {B_ITEMK, sizeof(uint32_t) * (size_t)items},
        {B_ITEME0, sizeof(uint32_t) * (size_t)items}, {B_ITEMC0, sizeof(uint32_t) * (size_t)items},
        {B_PART, sizeof(double) * 4 * (size_t)ls * (size_t)items}};
    for (auto& q : need5)
      if ((rc = ensure(ctx, q.id, q.bytes))) return rc;
    a.item_leaf = P<int32_t>(ctx, B_ITEMLEAF);
    a.item_k = P<uint32_t>(ctx, B_ITEMK);
    a.part = P<double>(ctx, B_PART);
    a.item_e0 = P<uint32_t>(ctx, B_ITEME0);
    a.item_c0 = P<uint32_t>(ctx, B_ITEMC0);
  }
  // the P2P kernel runs beside the far field when it writes only item partial
  // sums: the reduction, which adds the far field, then waits for both
  const bool overlap = ctx->overlap != 0 && ctx->cfg.leaf_size <= 32 && ctx->near_variant != 1;
  if (overlap && !ctx->aux) {
    HIPCHK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
  }
  KernelMarks km;
  km.begin = phase_event(ctx, 6, 0);
  km.end = phase_event(ctx, 6, 1);
  km.skip_reduce = overlap;
  auto near_field = [&](hipStream_t ns) -> int {
    HIPCHK(hipMemsetAsync(a.soft_pairs, 0, sizeof(unsigned long long), ns));
    if (ctx->cfg.leaf_size <= 32)
      launch_p2p_items_fill(level, a, P<int32_t>(ctx, B_ITEMLEAF), P<uint32_t>(ctx, B_ITEMK),
                            P<uint32_t>(ctx, B_ITEME0), P<uint32_t>(ctx, B_ITEMC0), ns);
    if (f32) launch_near32(ctx->order, level, ctx->cfg.leaf_size, ctx->near_variant, a,
                          P<float4>(ctx, B_PF32), P<float2>(ctx, B_PH32), items, ns, km);
    else launch_near(level, ctx->cfg.leaf_size, ctx->near_variant, a, items, ns, km);
    return SFMM_OK;
  };
  auto far_field = [&]() {
    if (shared) {
      SharedFarArgs sa{};
      sa.nn = (int)ctx->nn;
      sa.level_nodes = reinterpret_cast<const int32_t*>(P<uint32_t>(ctx, B_LEVNODES));
      sa.depth = P<int32_t>(ctx, B_NDEPTH);
      sa.m2l_off = f.node_m2l_off;
      sa.m2l_cnt = f.node_m2l_cnt;
      sa.pool = f.node_m2l_pool;
      sa.rec = f.rec;
      sa.rec32 = f32 ? P<float>(ctx, B_REC32) : nullptr;
      sa.top = ctx->cfg.fp64_top_depth;
      sa.ln = P<double>(ctx, B_LN);
      if (mutual) {
        launch_far_mutual(ctx->order, f, sa, s);
      } else {
        // nodes grouped by list length for the M2L kernel (the level sort's
        // key and id buffers are free once the tree is built)
        M2LOrderBufs ob{};
        ob.key0 = P<uint64_t>(ctx, B_LEVKEY0);
        ob.key1 = P<uint64_t>(ctx, B_LEVKEY1);
        ob.ids0 = P<uint32_t>(ctx, B_LEVIDS);
        ob.ids1 = P<uint32_t>(ctx, B_M2LORD);
        ob.hist = P<uint32_t>(ctx, B_HIST);
        ob.hist_tmp = P<uint32_t>(ctx, B_SCANTMP);
        ob.total = reinterpret_cast<uint32_t*>(small + S_SORTTOT);
        launch_m2l_order(sa, f32, ob, s);
        sa.level_nodes = reinterpret_cast<const int32_t*>(ob.ids1);
        launch_far_shared(ctx->order, f, sa, f32, s);
      }
    } else if (f32) {
      launch_far32(ctx->order, level, f, P<float>(ctx, B_REC32), ctx->cfg.fp64_top_depth, s);
    } else {
      launch_far(ctx->order, level, f, s);
    }
  };
  phase_mark(ctx, 3, 0);
  if (f32) {
    launch_prep32(ctx->order, (int)ctx->nn, nl, f.leaf_node, f.info, f.rec, P<int32_t>(ctx, B_NDEPTH),
                  f.xs, f.ys, f.zs, P<double>(ctx, B_MS), P<double>(ctx, B_HS),
                  P<float>(ctx, B_REC32), P<float4>(ctx, B_PF32), P<float2>(ctx, B_PH32), s);
  }
  if (overlap) {
    // phase 3 is then the far field with the P2P kernel beside it, phase 4
    // what is left of the near field after it, with the reduction
    HIPCHK(hipEventRecord(ctx->fork_ev, s));
    if (ctx->overlap == 2) far_field();
    HIPCHK(hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
    if ((rc = near_field(ctx->aux))) return rc;
    HIPCHK(hipEventRecord(ctx->join_ev, ctx->aux));
    if (ctx->overlap == 1) far_field();
    phase_mark(ctx, 3, 1);
    phase_mark(ctx, 4, 0);
    HIPCHK(hipStreamWaitEvent(s, ctx->join_ev, 0));
    launch_p2p_reduce(a, p2p_leaf_slots(ctx->cfg.leaf_size), s);
    phase_mark(ctx, 4, 1);
  } else {
    far_field();
    phase_mark(ctx, 3, 1);
    phase_mark(ctx, 4, 0);
    if ((rc = near_field(s))) return rc;
    phase_mark(ctx, 4, 1);
  }
  phase_mark(ctx, 5, 0);
  launch_momentum(n, m, acc, P<double>(ctx, B_MOMPART), P<double>(ctx, B_MOM), s);
  phase_mark(ctx, 5, 1);
  if (ctx->timing && ctx->timing_used < ctx->timing_cap) ctx->timing_used++;
  HIPCHK(hipGetLastError());
  // statistics totals of the level walk are read lazily (sfmm_get_stats)
  if (level) ctx->stats_pending = true;
  ctx->have_mom = true;
  (void)small;
  return SFMM_OK;
}

// common checks of the two direct-sum entry points (0 = go on, 1 = nothing
// to do, < 0 = error)
int direct_args(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
                int64_t nt, const int64_t* targets, double* acc, double* pot) {
  if (n < 0 || nt < 0 || n >= (int64_t(1) << 30))
    return fail(ctx, SFMM_EINVAL, "n or target count out of range");
  if (nt == 0) return 1;
  if (n == 0) return fail(ctx, SFMM_EINVAL, "targets given for an empty system");
  if (!x || !m || !h || !acc || !pot) return fail(ctx, SFMM_EINVAL, "NULL array");
  if (!targets && nt > n) return fail(ctx, SFMM_EINVAL, "more targets than particles");
  return 0;
}

// runs the direct sum with the status word and partial sums at the given
// device addresses, then reads the status back (one synchronisation)
int direct_run(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
               int64_t nt, const int64_t* targets, double* acc, double* pot, int* status,
               double* part, int nchunk) {
  const hipStream_t s = ctx->stream;
  launch_direct(n, x, m, h, nt, targets, ctx->cfg.G, ctx->cfg.include_self_potential, acc, pot,
                status, part, nchunk, s);
  HIPCHK(hipGetLastError());
  int hs = 0;
  HIPCHK(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(wait_stream(s));
  if (hs & ST_OVERFLOW) return fail(ctx, SFMM_EINVAL, "target index out of range");
  return SFMM_OK;
}

// ---- the direct sum in a fixed device array (no allocation) ----------------
// Each GPU holds one copy of `scratch` until the process ends: the status
// word, then the partial sums ([chunk][target][4] doubles).  Host code never
// uses the array's name as an address: hipGetSymbolAddress gives each
// device's own copy, once per device, with that device current.
constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB
constexpr size_t kScratchStatus = 256;               // bytes before the partial sums
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// the device address of this device's scratch (device already current)
int scratch_address(sfmm_ctx* ctx, unsigned char** out) {
  if (ctx->device < 0 || ctx->device >= kMaxScratchDevices)
    return fail(ctx, SFMM_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ctx, SFMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
    g_scratch_ptr[ctx->device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[ctx->device]);
  return SFMM_OK;
}

const char* kStatusText[] = {"ok", "invalid argument", "out of device memory", "HIP error",
                             "unsupported", "non-finite or non-positive input"};

}  // namespace

extern "C" {

int sfmm_config_default(sfmm_config* cfg) {
  if (!cfg) return SFMM_EINVAL;
  cfg->G = 1.0;
  cfg->leaf_size = 10;
  cfg->r_kern = 2.0;
  cfg->include_self_potential = 1;
  cfg->check_inputs = 1;
  cfg->walk_mode = SFMM_WALK_LEVEL;
  cfg->fp64_top_depth = 8;
  cfg->far_mode = SFMM_FAR_SHARED;
  cfg->far_kernel = 0;
  cfg->near_kernel = 0;
  return SFMM_OK;
}

// the P2P kernel shapes (sfmm_config.near_kernel)
static bool near_shape_ok(int v) { return v == 0 || v == 1 || v == 6 || v == 7 || v == 13; }

int sfmm_create(sfmm_ctx** out, int device, void* hip_stream, const sfmm_config* cfg) {
  if (!out) return SFMM_EINVAL;
  *out = nullptr;
  sfmm_config c;
  sfmm_config_default(&c);
  if (cfg) c = *cfg;
  if (!(c.leaf_size >= 1 && c.leaf_size <= 64) || !(c.r_kern >= 0.0) || !std::isfinite(c.G) ||
      !std::isfinite(c.r_kern) || (c.walk_mode != SFMM_WALK_LEVEL && c.walk_mode != SFMM_WALK_LEAF) ||
      c.fp64_top_depth < 0 || c.fp64_top_depth > 128 ||
      (c.far_mode != SFMM_FAR_LEAF && c.far_mode != SFMM_FAR_SHARED &&
       c.far_mode != SFMM_FAR_MUTUAL) || c.far_kernel != 0 || !near_shape_ok(c.near_kernel))
    return SFMM_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SFMM_EDEVICE;
  }
  sfmm_ctx* ctx = new (std::nothrow) sfmm_ctx();
  if (!ctx) return SFMM_ENOMEM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->cfg = c;
  ctx->near_variant = c.near_kernel;
  // measurement override (an unknown shape is refused)
  if (const char* nv = std::getenv("SFMM_NEAR_VARIANT")) {
    const int v = std::atoi(nv);
    if (!near_shape_ok(v)) {
      delete ctx;
      return SFMM_EINVAL;
    }
    ctx->near_variant = v;
  }
  if (const char* cp = std::getenv("SFMM_CHECK_POOLS")) ctx->check_pools = std::atoi(cp) != 0;
  if (const char* pi = std::getenv("SFMM_POOL_INIT"))
    ctx->pool_init = (uint64_t)std::max(0ll, std::atoll(pi));
  // first per-leaf list slots "m,p", optionally ",i" for the internal nodes'
  // slots (tests meet lists that overflow them)
  if (const char* ls = std::getenv("SFMM_LEAF_SLOTS")) {
    unsigned sm = 0, sp = 0, si = ctx->int_slot;
    const int got = std::sscanf(ls, "%u,%u,%u", &sm, &sp, &si);
    if (got < 2 || sm < 1 || sm > kSlotMax || sp < 1 || sp > kSlotMax / 2 || si < 1 ||
        si > kIntSlotMax) {
      delete ctx;
      return SFMM_EINVAL;
    }
    ctx->slot_m = sm;
    ctx->slot_p = sp;
    ctx->int_slot = si;
  }
  if (const char* ov = std::getenv("SFMM_OVERLAP")) {
    const int v = std::atoi(ov);
    if (v < 0 || v > 2) {
      delete ctx;
      return SFMM_EINVAL;
    }
    ctx->overlap = v;
  }
  *out = ctx;
  return SFMM_OK;
}

int sfmm_destroy(sfmm_ctx* ctx) {
  if (!ctx) return SFMM_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  free_events(ctx);
  if (ctx->order_ev) (void)hipEventDestroy(ctx->order_ev);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  for (auto& b : ctx->buf)
    if (b.p) (void)hipFree(b.p);
  if (ctx->rb) (void)hipHostFree(ctx->rb);
  delete ctx;
  return SFMM_OK;
}

int sfmm_set_stream(sfmm_ctx* ctx, void* hip_stream) {
  if (!ctx) return SFMM_EINVAL;
  hipStream_t ns = static_cast<hipStream_t>(hip_stream);
  if (ns == ctx->stream) return SFMM_OK;
  // the workspace is shared: work enqueued on the new stream must not start
  // before what is still queued on the old one
  HIPCHK(hipSetDevice(ctx->device));
  if (!ctx->order_ev) HIPCHK(hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ctx->order_ev, ctx->stream));
  HIPCHK(hipStreamWaitEvent(ns, ctx->order_ev, 0));
  ctx->stream = ns;
  return SFMM_OK;
}

int sfmm_build(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
               int order) {
  if (!ctx) return SFMM_EINVAL;
  ctx->err.clear();
  return do_build(ctx, n, x, m, h, order);
}

int sfmm_solve(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
               double theta, int order, int precision, double* acc, double* pot) {
  if (!ctx) return SFMM_EINVAL;
  ctx->err.clear();
  if (!(theta > 0.0 && theta < 1.0)) return fail(ctx, SFMM_EINVAL, "theta must be in (0, 1)");
  if (precision != SFMM_FP64 && precision != SFMM_FP32C)
    return fail(ctx, SFMM_EUNSUPPORTED, "unknown precision");
  if (n > 0 && (!acc || !pot)) return fail(ctx, SFMM_EINVAL, "NULL output array");
  int rc = do_build(ctx, n, x, m, h, order);
  if (rc) return rc;
  if (n == 0) return SFMM_OK;
  return do_walk_and_eval(ctx, theta, precision, m, acc, pot);
}

int sfmm_solve_batch(sfmm_ctx* ctx, int k, const int64_t* offsets, const double* x,
                     const double* m, const double* h, double theta, int order, int precision,
                     double* acc, double* pot) {
  if (!ctx) return SFMM_EINVAL;
  ctx->err.clear();
  if (k < 1 || k > (1 << 24) || !offsets) return fail(ctx, SFMM_EINVAL, "bad system count");
  if (offsets[0] != 0) return fail(ctx, SFMM_EINVAL, "offsets[0] must be 0");
  int nonempty = 0, only = 0;
  for (int s = 0; s < k; ++s) {
    if (offsets[s + 1] < offsets[s]) return fail(ctx, SFMM_EINVAL, "offsets must not decrease");
    if (offsets[s + 1] > offsets[s]) { ++nonempty; only = s; }
  }
  (void)only;
  const int64_t n = offsets[k];
  if (!(theta > 0.0 && theta < 1.0)) return fail(ctx, SFMM_EINVAL, "theta must be in (0, 1)");
  if (precision != SFMM_FP64 && precision != SFMM_FP32C)
    return fail(ctx, SFMM_EUNSUPPORTED, "unknown precision");
  if (n > 0 && (!acc || !pot)) return fail(ctx, SFMM_EINVAL, "NULL output array");
  // one non-empty system is an ordinary solve of the concatenated arrays
  int rc = nonempty <= 1 ? do_build(ctx, n, x, m, h, order)
                         : do_build(ctx, n, x, m, h, order, k, offsets);
  if (rc) return rc;
  if (n == 0) return SFMM_OK;
  return do_walk_and_eval(ctx, theta, precision, m, acc, pot);
}

int sfmm_get_stats(sfmm_ctx* ctx, sfmm_stats* out) {
  if (!ctx || !out) return SFMM_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->n = ctx->n;
  out->num_nodes = ctx->nn;
  out->num_leaves = ctx->nleaves;
  out->max_depth = ctx->maxdepth;
  out->walk_attempts = ctx->walk_attempts;
  out->leaf_slot_m2l = (int32_t)ctx->walk_slot_m;
  out->leaf_slot_p2p = (int32_t)ctx->walk_slot_p;
  out->n_leaf_overflow = (int64_t)ctx->leaf_overflow;
  out->max_leaf_m2l = (int64_t)ctx->max_leaf_m;
  out->max_leaf_p2p = (int64_t)ctx->max_leaf_p;
  if (ctx->have_lists && ctx->stats_pending) {
    // the level walk's per-leaf totals are only computed when asked for
    const int nl = (int)ctx->nleaves;
    const hipStream_t s = ctx->stream;
    uint64_t* small = P<uint64_t>(ctx, B_SMALL);
    LeafStatArgs ls{};
    ls.nleaves = nl;
    ls.leaf_node = P<int32_t>(ctx, B_LEAFNODE);
    ls.leaf_depth = P<int32_t>(ctx, B_LEAFDEPTH);
    ls.info = P<NodeInfo>(ctx, B_INFO);
    ls.m2l_cnt = P<uint32_t>(ctx, B_NM2LCNT);
    ls.p2p_off = P<uint32_t>(ctx, B_NP2POFF);
    ls.p2p_cnt = P<uint32_t>(ctx, B_NP2PCNT);
    ls.p2p_pool = P<uint32_t>(ctx, B_P2PPOOL);
    ls.m2l = P<uint64_t>(ctx, B_M2LCNT);
    ls.l2l = P<uint64_t>(ctx, B_L2LCNT);
    ls.pairs = P<uint64_t>(ctx, B_PAIRCNT);
    launch_leaf_stats(ls, s);
    scan_u64(ls.m2l, ls.m2l, nl, small + S_M2LTOT, P<uint64_t>(ctx, B_SCANTMP), s);
    scan_u64(ls.l2l, ls.l2l, nl, small + S_L2LTOT, P<uint64_t>(ctx, B_SCANTMP), s);
    scan_u64(ls.pairs, ls.pairs, nl, small + S_PAIRTOT, P<uint64_t>(ctx, B_SCANTMP), s);
    uint64_t hsmall[S_COUNT];
    if (hipMemcpyAsync(hsmall, ctx->buf[B_SMALL].p, sizeof(hsmall), hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail(ctx, SFMM_EDEVICE, "statistics copy failed");
    ctx->m2l_total = hsmall[S_M2LTOT];
    ctx->l2l_total = hsmall[S_L2LTOT];
    ctx->pair_total = hsmall[S_PAIRTOT];
    ctx->stats_pending = false;
  }
  if (ctx->have_lists) {
    out->n_m2l = (int64_t)ctx->m2l_total;
    out->n_l2l = (int64_t)ctx->l2l_total;
    out->n_p2p_leaf_pairs = (int64_t)ctx->p2p_total;
    out->n_p2p_pairs = (int64_t)ctx->pair_total;
    out->n_m2l_unique = (int64_t)ctx->m2l_unique;
    unsigned long long soft = 0;
    if (ctx->buf[B_SOFTCNT].p &&
        (hipMemcpyAsync(&soft, ctx->buf[B_SOFTCNT].p, sizeof(soft), hipMemcpyDeviceToHost,
                        ctx->stream) != hipSuccess ||
         hipStreamSynchronize(ctx->stream) != hipSuccess))
      return fail(ctx, SFMM_EDEVICE, "statistics copy failed");
    out->n_p2p_soft_pairs = (int64_t)soft;
  }
  if (ctx->have_mom && ctx->n > 0) {
    double mom[4];
    if (hipMemcpyAsync(mom, ctx->buf[B_MOM].p, sizeof(mom), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail(ctx, SFMM_EDEVICE, "momentum copy failed");
    out->momentum[0] = mom[0];
    out->momentum[1] = mom[1];
    out->momentum[2] = mom[2];
    out->momentum_abs = mom[3];
  }
  return SFMM_OK;
}

int sfmm_get_tree(sfmm_ctx* ctx, int64_t* num_nodes, int64_t* num_leaves, int32_t* perm,
                  uint64_t* keys, int32_t* lo, int32_t* cnt, int32_t* child, int32_t* parent,
                  double* s, double* mass, double* l, double* hmax, double* Q) {
  if (!ctx) return SFMM_EINVAL;
  if (!ctx->have_tree) return fail(ctx, SFMM_EINVAL, "no tree built");
  if (num_nodes) *num_nodes = ctx->nn;
  if (num_leaves) *num_leaves = ctx->nleaves;
  const int64_t n = ctx->n, nn = ctx->nn;
  if (n == 0) return SFMM_OK;
  const hipStream_t st = ctx->stream;
  HIPCHK(hipStreamSynchronize(st));
  if (perm) HIPCHK(hipMemcpy(perm, ctx->buf[B_VAL0].p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  if (keys) HIPCHK(hipMemcpy(keys, ctx->buf[B_KEY0].p, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
  if (lo || cnt || child || parent) {
    NodeInfo* tmp = static_cast<NodeInfo*>(std::malloc(sizeof(NodeInfo) * nn));
    if (!tmp) return SFMM_ENOMEM;
    hipError_t e = hipMemcpy(tmp, ctx->buf[B_INFO].p, sizeof(NodeInfo) * nn, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { std::free(tmp); return fail(ctx, SFMM_EDEVICE, "copy failed"); }
    for (int64_t v = 0; v < nn; ++v) {
      if (lo) lo[v] = tmp[v].lo;
      if (cnt) cnt[v] = tmp[v].cnt;
      if (child) child[v] = tmp[v].child;
      if (parent) parent[v] = tmp[v].parent;
    }
    std::free(tmp);
  }
  if (s || mass || l || hmax || Q) {
    const int RS = rec_stride(ctx->order), NQ = ncoef(ctx->order);
    double* tmp = static_cast<double*>(std::malloc(sizeof(double) * RS * nn));
    if (!tmp) return SFMM_ENOMEM;
    hipError_t e = hipMemcpy(tmp, ctx->buf[B_REC].p, sizeof(double) * RS * nn, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { std::free(tmp); return fail(ctx, SFMM_EDEVICE, "copy failed"); }
    for (int64_t v = 0; v < nn; ++v) {
      const double* r = tmp + v * RS;
      if (s) { s[3 * v] = r[0]; s[3 * v + 1] = r[1]; s[3 * v + 2] = r[2]; }
      if (l) l[v] = r[3];
      if (hmax) hmax[v] = r[4];
      if (mass) mass[v] = r[5];
      if (Q) for (int k = 0; k < NQ; ++k) Q[v * NQ + k] = r[8 + k];
    }
    std::free(tmp);
  }
  return SFMM_OK;
}

int sfmm_get_leaves(sfmm_ctx* ctx, int32_t* leaf_node, int32_t* leaf_depth) {
  if (!ctx) return SFMM_EINVAL;
  if (!ctx->have_tree) return fail(ctx, SFMM_EINVAL, "no tree built");
  if (ctx->nleaves == 0) return SFMM_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (leaf_node)
    HIPCHK(hipMemcpy(leaf_node, ctx->buf[B_LEAFNODE].p, sizeof(int32_t) * ctx->nleaves,
                     hipMemcpyDeviceToHost));
  if (leaf_depth)
    HIPCHK(hipMemcpy(leaf_depth, ctx->buf[B_LEAFDEPTH].p, sizeof(int32_t) * ctx->nleaves,
                     hipMemcpyDeviceToHost));
  return SFMM_OK;
}

int sfmm_get_leaf_lists(sfmm_ctx* ctx, int64_t leaf, int32_t* m2l_depth, int32_t* m2l_src,
                        int64_t cap_m2l, int64_t* n_m2l, int32_t* p2p_src, int64_t cap_p2p,
                        int64_t* n_p2p) {
  if (!ctx) return SFMM_EINVAL;
  if (!ctx->have_lists) return fail(ctx, SFMM_EINVAL, "no lists (run sfmm_solve first)");
  if (leaf < 0 || leaf >= ctx->nleaves) return fail(ctx, SFMM_EINVAL, "leaf out of range");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->cfg.walk_mode == SFMM_WALK_LEVEL) {
    // the leaf's list is its ancestors' node lists, root first, then its P2P list
    const int64_t nn = ctx->nn;
    std::vector<NodeInfo> info(nn);
    std::vector<uint32_t> moff(nn), mcnt(nn);
    int32_t node = 0;
    HIPCHK(hipMemcpy(info.data(), ctx->buf[B_INFO].p, sizeof(NodeInfo) * nn, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(moff.data(), ctx->buf[B_NM2LOFF].p, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(mcnt.data(), ctx->buf[B_NM2LCNT].p, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&node, P<int32_t>(ctx, B_LEAFNODE) + leaf, sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> dep, src;
    int v = 0, k = 0;
    for (;;) {
      std::vector<uint32_t> seg(mcnt[v]);
      if (mcnt[v])
        HIPCHK(hipMemcpy(seg.data(), P<uint32_t>(ctx, B_M2LPOOL) + moff[v], sizeof(uint32_t) * mcnt[v],
                         hipMemcpyDeviceToHost));
      for (uint32_t e : seg) { dep.push_back(k); src.push_back((int32_t)e); }
      if (v == node) break;
      const int c = info[v].child;
      if (c < 0) return fail(ctx, SFMM_EDEVICE, "inconsistent tree");
      v = (info[node].lo < info[c + 1].lo) ? c : c + 1;
      ++k;
    }
    uint32_t po2[2];
    HIPCHK(hipMemcpy(&po2[0], P<uint32_t>(ctx, B_NP2POFF) + node, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&po2[1], P<uint32_t>(ctx, B_NP2PCNT) + node, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (n_m2l) *n_m2l = (int64_t)dep.size();
    if (n_p2p) *n_p2p = po2[1];
    for (int64_t q = 0; q < (int64_t)dep.size() && q < cap_m2l; ++q) {
      if (m2l_depth) m2l_depth[q] = dep[q];
      if (m2l_src) m2l_src[q] = src[q];
    }
    const int64_t cp = std::min<int64_t>(po2[1], cap_p2p < 0 ? 0 : cap_p2p);
    if (cp > 0 && p2p_src)
      HIPCHK(hipMemcpy(p2p_src, P<uint32_t>(ctx, B_P2PPOOL) + po2[0], sizeof(int32_t) * cp,
                       hipMemcpyDeviceToHost));
    return SFMM_OK;
  }
  uint64_t mo[2], po[2];
  HIPCHK(hipMemcpy(mo, P<uint64_t>(ctx, B_M2LCNT) + leaf, sizeof(mo), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(po, P<uint64_t>(ctx, B_P2PCNT) + leaf, sizeof(po), hipMemcpyDeviceToHost));
  const int64_t nm = (int64_t)(mo[1] - mo[0]), np = (int64_t)(po[1] - po[0]);
  if (n_m2l) *n_m2l = nm;
  if (n_p2p) *n_p2p = np;
  const int64_t cm = std::min<int64_t>(nm, cap_m2l < 0 ? 0 : cap_m2l);
  if (cm > 0 && (m2l_depth || m2l_src)) {
    uint32_t* tmp = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * cm));
    if (!tmp) return SFMM_ENOMEM;
    hipError_t e = hipMemcpy(tmp, P<uint32_t>(ctx, B_M2L) + mo[0], sizeof(uint32_t) * cm,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) { std::free(tmp); return fail(ctx, SFMM_EDEVICE, "copy failed"); }
    for (int64_t k = 0; k < cm; ++k) {
      if (m2l_depth) m2l_depth[k] = (int32_t)(tmp[k] >> kSrcBits);
      if (m2l_src) m2l_src[k] = (int32_t)(tmp[k] & kSrcMask);
    }
    std::free(tmp);
  }
  const int64_t cp = std::min<int64_t>(np, cap_p2p < 0 ? 0 : cap_p2p);
  if (cp > 0 && p2p_src)
    HIPCHK(hipMemcpy(p2p_src, P<int32_t>(ctx, B_P2P) + po[0], sizeof(int32_t) * cp,
                     hipMemcpyDeviceToHost));
  return SFMM_OK;
}

int sfmm_timing_start(sfmm_ctx* ctx, int max_solves) {
  if (!ctx || max_solves < 1 || max_solves > 100000) return SFMM_EINVAL;
  free_events(ctx);
  HIPCHK(hipSetDevice(ctx->device));
  const size_t ne = (size_t)max_solves * 2 * SFMM_NUM_PHASES;
  ctx->events.resize(ne, nullptr);
  for (size_t k = 0; k < ne; ++k) {
    hipError_t e = hipEventCreate(&ctx->events[k]);
    if (e != hipSuccess) {
      ctx->events.resize(k);
      free_events(ctx);
      return fail(ctx, SFMM_EDEVICE, "hipEventCreate failed");
    }
  }
  ctx->timing_cap = max_solves;
  ctx->timing_used = 0;
  ctx->timing = true;
  return SFMM_OK;
}

int sfmm_timing_stop(sfmm_ctx* ctx, double* ms, int cap, int* nsolves) {
  if (!ctx) return SFMM_EINVAL;
  if (nsolves) *nsolves = ctx->timing_used;
  int rc = SFMM_OK;
  if (ctx->timing_used > 0 && ms && cap > 0) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) rc = SFMM_EDEVICE;
    const int k_max = std::min(cap, ctx->timing_used);
    for (int k = 0; k < k_max && rc == SFMM_OK; ++k)
      for (int p = 0; p < SFMM_NUM_PHASES; ++p) {
        float t = 0.f;
        const size_t b = (size_t)k * 2 * SFMM_NUM_PHASES + 2 * p;
        if (hipEventElapsedTime(&t, ctx->events[b], ctx->events[b + 1]) != hipSuccess) {
          (void)hipGetLastError();
          t = -1.f;
        }
        ms[(size_t)k * SFMM_NUM_PHASES + p] = t;
      }
  }
  free_events(ctx);
  return rc;
}

const char* sfmm_phase_name(int phase) {
  static const char* names[SFMM_NUM_PHASES] = {"tree",     "walk_count", "walk_fill",  "far",
                                               "near",     "momentum",   "near_kernel"};
  return (phase >= 0 && phase < SFMM_NUM_PHASES) ? names[phase] : "unknown";
}

int sfmm_workspace_bytes(const sfmm_ctx* ctx, uint64_t* out) {
  if (!ctx || !out) return SFMM_EINVAL;
  uint64_t b = 0;
  for (const auto& q : ctx->buf) b += q.cap;
  *out = b;
  return SFMM_OK;
}

int sfmm_direct(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
                int64_t nt, const int64_t* targets, double* acc, double* pot) {
  if (!ctx) return SFMM_EINVAL;
  ctx->err.clear();
  int rc = direct_args(ctx, n, x, m, h, nt, targets, acc, pot);
  if (rc) return rc > 0 ? SFMM_OK : rc;
  if ((rc = set_device(ctx))) return rc;
  const int nchunk = direct_chunks(n, nt, uint64_t(1) << 30);
  if (nchunk < 1) return fail(ctx, SFMM_EINVAL, "too many targets");
  if ((rc = ensure(ctx, B_STATUS, sizeof(int) * 4))) return rc;
  if ((rc = ensure(ctx, B_DIRPART, sizeof(double) * 4 * (size_t)nt * nchunk))) return rc;
  return direct_run(ctx, n, x, m, h, nt, targets, acc, pot, P<int>(ctx, B_STATUS),
                    P<double>(ctx, B_DIRPART), nchunk);
}

int sfmm_direct_noalloc(sfmm_ctx* ctx, int64_t n, const double* x, const double* m,
                        const double* h, int64_t nt, const int64_t* targets, double* acc,
                        double* pot) {
  if (!ctx) return SFMM_EINVAL;
  ctx->err.clear();
  int rc = direct_args(ctx, n, x, m, h, nt, targets, acc, pot);
  if (rc) return rc > 0 ? SFMM_OK : rc;
  if ((rc = set_device(ctx))) return rc;
  const int nchunk = direct_chunks(n, nt, kScratchBytes - kScratchStatus);
  if (nchunk < 1)
    return fail(ctx, SFMM_EINVAL,
                "too many targets for the fixed scratch: at most " +
                    std::to_string((kScratchBytes - kScratchStatus) / (4 * sizeof(double))) +
                    " targets per call");
  unsigned char* base = nullptr;
  if ((rc = scratch_address(ctx, &base))) return rc;
  return direct_run(ctx, n, x, m, h, nt, targets, acc, pot, reinterpret_cast<int*>(base),
                    reinterpret_cast<double*>(base + kScratchStatus), nchunk);
}

int sfmm_leapfrog(void* hip_stream, int64_t n, double* x, double* v, const double* acc,
                  double kick, double drift) {
  if (n < 0 || (n > 0 && (!x || !v || !acc))) return SFMM_EINVAL;
  launch_leapfrog(n, x, v, acc, kick, drift, static_cast<hipStream_t>(hip_stream));
  return hipGetLastError() == hipSuccess ? SFMM_OK : SFMM_EDEVICE;
}

const char* sfmm_strerror(int status) {
  if (status > 0 || status < -5) return "unknown status";
  return kStatusText[-status];
}

const char* sfmm_last_error(const sfmm_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"
