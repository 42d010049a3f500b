// sfmm_internal.h -- device data layout and launch wrappers of libsfmm.so.
//
// Layout in HBM (all arrays owned by the context workspace):
//   particles, sorted by Morton key: xs, ys, zs, ms, hs   FP64 SoA, n each
//   perm       u32[n]   sorted position -> caller index
//   NodeInfo   {lo, cnt, child, parent} per node (16 B); the two children of
//              an internal node are adjacent (child, child + 1)
//   rec        FP64 node records, REC_STRIDE(P) doubles per node:
//                [0..2] centre of mass, [3] size l, [4] h_max, [5] mass,
//                [8 .. 8+NQ) mass moments Q~ (graded multi-index order)
//   leaf_node / leaf_depth   i32 per leaf, Morton order
//   M2L lists  u32 per entry: depth of the target ancestor (7 bits) | source
//              node (25 bits), grouped by depth inside each leaf's segment
//   P2P lists  i32 source leaf node per entry
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "expansions_gen.h"

namespace sfmm {

struct NodeInfo {
  int32_t lo, cnt, child, parent;
};

constexpr int kDepthBits = 7;
constexpr int kSrcBits = 25;
constexpr uint32_t kSrcMask = (1u << kSrcBits) - 1u;
constexpr int kMaxDepthCap = (1 << kDepthBits) - 1;  // 127; radix trees stay below 96
constexpr int kMaxOrder = 4;

__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int rec_stride(int p) { return ((8 + ncoef(p) + 7) / 8) * 8; }
inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// f(std::integral_constant<int, 0>{}), ..., f(std::integral_constant<int, N - 1>{})
template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// Workgroups of a launch are dealt to the chip's 8 XCDs (each with its own
// L2) in turn.  Work whose neighbours share data (leaves in Morton order,
// nodes of one level) is better kept together in one L2: this maps block b
// of nb so that each XCD's blocks cover one contiguous range.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned per = nb / kXcds, rem = nb % kXcds;
  const unsigned x = b % kXcds, k = b / kXcds;
  return x * per + (x < rem ? x : rem) + k;
}

// local (field) coefficients: H_g for 1 <= |g| <= p+1, then P_b for |b| <= p
__host__ __device__ constexpr int local_count(int p) { return ncoef(p + 1) - 1 + ncoef(p); }
// FP32 copy of the moments (SFMM_FP32C): ncoef floats, then the node depth
__host__ __device__ constexpr int rec32_stride(int p) { return ((ncoef(p) + 1 + 7) / 8) * 8; }

// ---- status bits written by kernels --------------------------------------
// ST_BADLIST: after a walk, a list a consumer would read lies outside the
// pool part written by that walk, or (pool check mode) holds an entry that is
// not a node of the tree; the solve stops with an error before any consumer
// kernel runs
enum : int { ST_NONFINITE = 1, ST_DEPTH = 2, ST_OVERFLOW = 4, ST_BADLIST = 8 };
// per-node list offset of a list that did not fit in its pool: any read of
// it is clamped away ((uint64_t)kNoList + count > every pool capacity)
constexpr uint32_t kNoList = 0xFFFFFFFFu;
// list pools hold at most this many entries, so every offset of a list that
// fits is below kNoList
constexpr uint64_t kPoolMax = 0xF0000000ull;
// the largest per-leaf M2L list slot of the level walk (P2P: half of it)
constexpr uint32_t kSlotMax = 1024;
// the largest of the level walk's large per-leaf list slots
constexpr uint32_t kBigSlotMax = 1u << 18;
// the largest slot of an internal node's region in the level walk
constexpr uint32_t kIntSlotMax = 4096;

// ---- scan ------------------------------------------------------------------
// Exclusive prefix sum of `in` (n entries) into `out` (may alias in); the
// grand total is written to *total.  tmp must hold scan_tmp_elems(n) T's.
size_t scan_tmp_elems(int64_t n);
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
              hipStream_t s);
void scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total, uint64_t* tmp,
              hipStream_t s);
// u32 counts, u64 offsets and total
void scan_u32_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total, uint64_t* tmp,
                  hipStream_t s);

// ---- tree ------------------------------------------------------------------
int bbox_blocks(int64_t n);
void launch_bbox(int n, const double* x, const double* m, const double* h, double* part,
                 double* box, int* status, int check, hipStream_t s);
void launch_keys(int n, const double* x, const double* box, uint64_t* key, uint32_t* idx,
                 hipStream_t s);
int radix_blocks(int64_t n);
// sorts (key, idx) by key, stable; returns in key0/val0 (ping-pong via key1/val1)
void radix_sort(int n, uint64_t* key0, uint32_t* val0, uint64_t* key1, uint32_t* val1,
                uint32_t* hist, uint32_t* hist_tmp, uint32_t* scratch_total, hipStream_t s);
// one stable pass on the 8-bit digit at `shift`; hist holds 256 * radix_blocks(n)
// counters and, after the pass, their exclusive scan (digit-major)
void radix_pass(int n, const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                int shift, uint32_t* hist, uint32_t* hist_tmp, uint32_t* scratch_total,
                hipStream_t s);
// sorted particle data: separate arrays and one 32-byte record per particle
// (p4: x, y, z, m)
void launch_gather(int n, const uint32_t* perm, const double* x, const double* m,
                   const double* h, double* xs, double* ys, double* zs, double* ms,
                   double* hs, double* his, double* p4, hipStream_t s);
// sys / sys_start: system of each sorted position and first position of each
// system (nullptr for a single system)
void launch_karras(int n, const uint64_t* key, const uint32_t* sys, const int32_t* sys_start,
                   int leaf_size, int32_t* kfirst, int32_t* klast, int32_t* kleft,
                   int32_t* kright, int32_t* kpar, int32_t* kside, uint32_t* kept, hipStream_t s);
void launch_assign(int n, int leaf_size, const uint32_t* sys, const int32_t* kfirst,
                   const int32_t* klast, const int32_t* kleft, const int32_t* kright,
                   const int32_t* kpar, const int32_t* kside, const uint32_t* cidx, NodeInfo* info,
                   uint32_t* leaf_flag, int32_t* leaf_at, hipStream_t s);
// several systems: per-system boxes and keys, then (system, key) order
void launch_sys_keys(int n, int nsys, const int64_t* off, const double* x, const double* m,
                     const double* h, double* boxes, int* status, int check, uint64_t* key,
                     uint32_t* idx, uint32_t* sys, int32_t* sys_start, hipStream_t s);
void launch_sys_sortkey(int n, const uint32_t* perm1, const uint32_t* sys, uint64_t* skey,
                        uint32_t* pos, hipStream_t s);
void launch_sys_final(int n, const uint32_t* q, const uint32_t* perm1, const uint64_t* key1,
                      const uint32_t* sys, uint32_t* perm, uint64_t* key, uint32_t* sys_sorted,
                      hipStream_t s);
// per node: 0 spans two systems, 1 root of a system, 2 other
void launch_node_flags(int nn, const NodeInfo* info, const uint32_t* sys, uint8_t* flag,
                       hipStream_t s);
void launch_leaf_fill(int n, const uint32_t* leaf_flag, const uint32_t* leaf_scan,
                      const int32_t* leaf_at, int32_t* leaf_node, hipStream_t s);
void launch_single_leaf(int n, NodeInfo* info, int32_t* leaf_node, hipStream_t s);
void launch_leaf_depth(int nleaves, const int32_t* leaf_node, const NodeInfo* info,
                       const int32_t* node_depth, int32_t* leaf_depth, int32_t* p_leaf,
                       int* maxdepth, hipStream_t s);
// geometry and moments, deepest level first (level offsets: a host copy for
// the launch sizes and the device array for runs of small levels)
void launch_geometry(int order, int maxdepth, const uint32_t* level_off_host,
                     const uint32_t* level_off_dev, const int32_t* level_nodes,
                     const NodeInfo* info, const double* xs, const double* ys, const double* zs,
                     const double* ms, const double* hs, double* rec, hipStream_t s);
void launch_extent_count(int nn, const NodeInfo* info, uint32_t* chunks, hipStream_t s);
void launch_extent(int order, int nn, int nitems, const NodeInfo* info,
                   const uint32_t* chunk_off, uint32_t* item_node, const double* xs,
                   const double* ys, const double* zs, double* rec, unsigned long long* l2bits,
                   hipStream_t s);
void launch_extent_final(int order, int nn, const NodeInfo* info,
                         const unsigned long long* l2bits, double* rec, hipStream_t s);
constexpr int kExtentChunk = 2048;

// ---- walk (Algorithms 1 and 2) ---------------------------------------------
struct WalkArgs {
  int nleaves;
  const int32_t* leaf_node;
  const int32_t* leaf_depth;
  const NodeInfo* info;
  const double* rec;
  int stride;
  double theta2, r_kern;
  const uint64_t* leaf_doff;   // per-leaf offset into the per-depth count array
  uint32_t* depth_cnt;         // [sum (d+1)] M2L counts per (leaf, depth)
  uint64_t* m2l_cnt;           // [nleaves] (count pass) -> offsets after the scan
  uint64_t* p2p_cnt;           // [nleaves] idem
  uint64_t* pair_cnt;          // [nleaves] particle pairs (statistics)
  uint64_t* l2l_cnt;           // [nleaves] L2L translations (statistics)
  uint32_t* m2l_list;
  int32_t* p2p_list;
  int* status;
};
void launch_walk(const WalkArgs& a, int maxdepth, bool fill, hipStream_t s);
void launch_leaf_doff(int nleaves, const int32_t* leaf_depth, uint64_t* out, hipStream_t s);

// ---- level-synchronous node walk -------------------------------------------------
struct NodeWalkArgs {
  const NodeInfo* info;
  const double* rec;
  int stride;
  double theta2, r_kern;
  const int32_t* level_nodes;  // nodes grouped by depth
  const uint8_t* node_flag;    // 0 spans systems (skipped), 1 walk root, 2 other
  const uint32_t* level_off;   // [levels + 1]
  const uint32_t* level_int;   // [levels] end of each level's internal nodes
  // per node (node-indexed): M2L list, opened list (internal), P2P list (leaf).
  // An internal node's M2L and opened lists share one region of the M2L pool
  // (M2L from the front, opened from the back); its size, the node's tested
  // list, is known before the node is walked: exp[parent], the parent's
  // opened sources with internal ones counted twice (their two children).
  uint32_t *m2l_off, *m2l_cnt, *open_off, *open_cnt, *p2p_off, *p2p_cnt;
  uint32_t *m2l_pool, *open_pool, *p2p_pool;  // open_pool: the M2L pool
  // pool capacities (entries, <= kPoolMax).  Every running offset and total
  // below is 64-bit, so a demand beyond 2^32 entries is counted, not wrapped;
  // a list that does not fit gets the per-node offset kNoList and the host
  // grows the pools and walks again
  uint64_t m2l_cap, open_cap, p2p_cap;
  uint32_t* exp;  // per internal node: tested-list size of each of its children
  // the regions of the internal nodes: int_nodes slots of int_slot entries,
  // then an arena of int_big entries for larger ones; the leaves' slots
  // start at leaf_base = int_nodes * int_slot + int_big
  uint32_t int_slot, int_nodes;
  uint64_t int_big, leaf_base;
  uint64_t* run;      // [11 + kXcds] arena entries taken by internal nodes, M2L
                      // entries proper (the walk's sum), P2P pool used after the
                      // leaf slots, M2L pool used after the leaf slots, P2P entries
                      // proper, (unused), the longest M2L and P2P lists of a leaf,
                      // large M2L and P2P slots asked for, internal nodes in the
                      // arena, then the leaves of each of kXcds leaf ranges whose
                      // lists did not fit their slots
  // leaves (walked after all levels, in leaf order): fixed slots of slot_m M2L
  // and slot_p P2P entries per leaf, then nbig large slots of big_m and big_p
  // entries for leaves that outgrow theirs (big_plain: [nbig * big_p] staging
  // of the large P2P slots); the lists of a leaf that fit neither go after
  // all slots (leaf_*_cnt: their sizes, 0 for a leaf that fits; ovf_leaf:
  // such leaves, [nleaves])
  int nleaves;
  const int32_t* leaf_node;
  uint32_t slot_m, slot_p;
  uint32_t nbig, big_m, big_p;
  uint32_t* big_plain;
  uint32_t* ovf_leaf;
  uint32_t *leaf_m2l_cnt, *leaf_p2p_cnt;
  uint64_t *leaf_m2l_off, *leaf_p2p_off;
  // per leaf: particles over its P2P entries, P2P work items and their offsets
  // ([nleaves + 1], the last entry the total)
  uint32_t *src_total, *item_cnt, *item_off;
  uint32_t stack_cap;  // LDS lowering stack, entries
  int* status;
};
// node depth as a sort key (u64) and node ids (u32) for the bucketing by depth
void launch_node_depth(int nn, const NodeInfo* info, int32_t* depth, uint64_t* key,
                       uint32_t* ids, hipStream_t s);
// level_off[k] = first position of depth k in the depth-sorted node list
// (sort key 2 depth + leaf: a level's internal nodes first), level_int[k] =
// the end of its internal nodes; read from the scanned radix histogram
// (digit-major, nb blocks)
void launch_level_offsets(int nlev, int nb, int nn, const uint32_t* hist_scanned,
                          uint32_t* level_off, uint32_t* level_int, hipStream_t s);
// every leaf's lists (the slot pass, scans over the leaves, the second pass
// over leaves whose lists overflow their slots); scan_tmp holds
// scan_tmp_elems(nleaves) words; LDS of (stack_cap + slot_p) words per wave
void launch_nodewalk_leaves(const NodeWalkArgs& a, uint32_t* scan_tmp, hipStream_t s);
// after a walk: every node's M2L list and every leaf's P2P list must lie in
// the part of its pool the walk wrote (the internal regions, the leaf slots,
// then run[3] M2L and run[2] P2P entries); with check_entries, each entry
// must also be a node of the tree (below nn).  Sets ST_BADLIST in *status
// otherwise.  Adds the walk's M2L and P2P entries to run[1] and run[4], and
// takes the longest M2L and P2P lists of a leaf into run[6] and run[7].
void launch_check_lists(const NodeWalkArgs& a, int nn, bool check_entries, hipStream_t s);
void launch_nodewalk_level(const NodeWalkArgs& a, int level, int nodes_in_level, uint32_t rank0,
                           hipStream_t s);

// per-leaf statistics of node lists: replicated M2L count, L2L count, pairs
struct LeafStatArgs {
  int nleaves;
  const int32_t* leaf_node;
  const int32_t* leaf_depth;
  const NodeInfo* info;
  const uint32_t *m2l_cnt, *p2p_off, *p2p_cnt, *p2p_pool;
  uint64_t *m2l, *l2l, *pairs;  // per leaf
};
void launch_leaf_stats(const LeafStatArgs& a, hipStream_t s);

// ---- far field: M2L + L2L chain + L2P ----------------------------------------
struct FarArgs {
  int nleaves;
  const int32_t* leaf_node;
  const int32_t* leaf_depth;
  const NodeInfo* info;
  const double* rec;
  const uint64_t* m2l_off;  // [nleaves + 1]  (per-leaf lists)
  const uint32_t* m2l_list;
  const uint32_t* depth_cnt;  // per-leaf lists: entries per (leaf, depth)
  const uint64_t* leaf_doff;  //   at depth_cnt + leaf_doff[leaf]
  const uint32_t *node_m2l_off, *node_m2l_cnt, *node_m2l_pool;  // (node lists)
  const double *xs, *ys, *zs;
  double* far;  // [n][4]: field x, y, z, potential (before the -G factor)
};
// replicated per-leaf far field, 4 lanes per leaf
void launch_far(int order, bool node_lists, const FarArgs& a, hipStream_t s);

// shared far field: per-node M2L sums, then the per-leaf L2L chain and L2P
struct SharedFarArgs {
  int nn;
  const int32_t* level_nodes;  // nodes in the order the M2L kernel takes them
  const int32_t* depth;        // node depth
  const uint32_t *m2l_off, *m2l_cnt, *pool;  // per-node M2L lists
  const double* rec;
  const float* rec32;  // FP32 moments (FP32C)
  int top;             // FP32C: targets at depth < top in FP64
  double* ln;          // [nn][NL] per-node local expansions (written where cnt > 0)
};
void launch_far_shared(int order, const FarArgs& f, const SharedFarArgs& a, bool f32,
                       hipStream_t s);
// node order for the shared M2L (k_m2l_nodes): nodes grouped by the number of
// steps their lists take, longest first, stable over level order; result in
// ids1 (key0/ids0 and key1 are scratch of nn entries, hist/hist_tmp/total as
// for radix_pass)
struct M2LOrderBufs {
  uint64_t *key0, *key1;
  uint32_t *ids0, *ids1;
  uint32_t *hist, *hist_tmp, *total;
};
void launch_m2l_order(const SharedFarArgs& a, bool f32, const M2LOrderBufs& b, hipStream_t s);
// the one-sided symmetric form of the shared far field: each unordered node
// pair once (one D(r) for both nodes, the partner's side added atomically),
// then the per-leaf L2L chain and L2P (FP64 only)
void launch_far_mutual(int order, const FarArgs& f, const SharedFarArgs& a, hipStream_t s);

// ---- near field (P2P) + output in the caller's order ----------------------
struct NearArgs {
  int n;
  int nleaves;
  const int32_t* p_leaf;
  const NodeInfo* info;
  const uint64_t* p2p_off;  // [nleaves + 1]  (per-leaf lists)
  const int32_t* p2p_list;
  const int32_t* leaf_node;  // (node lists)
  const uint32_t *node_p2p_off, *node_p2p_cnt, *node_p2p_pool;
  const double *xs, *ys, *zs, *ms, *hs, *his;  // his = 1/h
  const double* p4;  // [n][4] x, y, z, m (one record per particle)
  const double* far;
  const double* rec;  // node records (leaf centres, FP32C; leaf spheres)
  int rec_stride;     // doubles per node record
  const uint32_t* perm;
  double G;
  int include_self;
  double* acc;  // caller order [n][3]
  double* pot;  // caller order [n]
  // work items (leaf_size <= 32): a leaf's P2P sources, flattened over its
  // list entries (leaves, or whole subtrees), are cut into runs of at most
  // kP2PItem source particles, one wave per run; each item writes partial
  // sums for the leaf's targets, which a second kernel adds in item order
  const uint32_t* src_total;  // per leaf: particles over its P2P list entries
  const uint32_t* item_off;  // [nleaves + 1] first item of each leaf; [nleaves] = total
  const int32_t* item_leaf;  // [items] leaf of each item
  const uint32_t* item_k;    // [items] index of the item within its leaf
  const uint32_t* item_e0;   // [items] (k > 0) list entry holding the item's first source
  const uint32_t* item_c0;   // [items] (k > 0) that entry's start in the flattened order
  double* part;              // [items][LS][4] partial field (x, y, z) and potential
  unsigned long long* soft_pairs;  // count of pairs inside a kernel (queueing shape)
};
constexpr uint32_t kP2PItem = 2048;
// particles over each leaf's P2P entries (src_total) and the number of
// items of each leaf (item_cnt), nleaves entries each; one wave per leaf
void launch_p2p_items_count(bool node_lists, const NearArgs& a, uint32_t* src_total,
                            uint32_t* item_cnt, hipStream_t s);
// item_leaf / item_k from the scanned item offsets
// item_leaf / item_k of every item; item_e0 / item_c0 of the items after a
// leaf's first (one wave per leaf)
void launch_p2p_items_fill(bool node_lists, const NearArgs& a, int32_t* item_leaf,
                           uint32_t* item_k, uint32_t* item_e0, uint32_t* item_c0, hipStream_t s);
// target slots per P2P work item: the kernels are built for leaves of at most
// 10, 16 and 32 particles
inline int p2p_leaf_slots(int leaf_size) { return leaf_size <= 10 ? 10 : leaf_size <= 16 ? 16 : 32; }
// wave-per-item kernel for leaf_size <= 32 (then the reduction in item
// order), particle-per-thread otherwise; items: the bound on the item count
// HIP events recorded on the stream around the main P2P kernel alone (null:
// none), for the timing of that kernel
struct KernelMarks {
  hipEvent_t begin = nullptr, end = nullptr;
  // the caller launches the reduction itself (after the far field, when the
  // P2P kernel runs on a stream of its own)
  bool skip_reduce = false;
};
inline void record_mark(hipEvent_t e, hipStream_t s) {
  if (e) (void)hipEventRecord(e, s);
}
void launch_near(bool node_lists, int leaf_size, int variant, const NearArgs& a, int64_t items,
                 hipStream_t s, KernelMarks km = {});
// the default P2P kernel: targets of the leaf in lanes (NS stripes of nt
// lanes), sources staged through LDS and split into far and near sources by
// the target leaf's sphere (ls = 10 or 16: the partial-sum layout)
void launch_p2p_tile(bool node_lists, int ls, const NearArgs& a, int64_t items, hipStream_t s);
// sum of the item partials per target, plus the far field and the self term,
// written in the caller's order (LS = the P2P kernel's target count)
void launch_p2p_reduce(const NearArgs& a, int ls, hipStream_t s);

// ---- FP32-compensated form ------------------------------------------------------
// FP32 moments per node and FP32 leaf-relative particle offsets (+ mass, h, 1/h)
void launch_prep32(int order, int nn, int nleaves, const int32_t* leaf_node, const NodeInfo* info,
                   const double* rec, const int32_t* node_depth, const double* xs, const double* ys,
                   const double* zs, const double* ms, const double* hs, float* rec32, float4* pf,
                   float2* ph, hipStream_t s);
void launch_far32(int order, bool node_lists, const FarArgs& a, const float* rec32, int top,
                  hipStream_t s);
// false when leaf_size > 16 (not built)
// variant: the P2P shape (0 the wave kernel with scalar-register targets,
// 6 the earlier one with targets in LDS; others as 0)
bool launch_near32(int order, bool node_lists, int leaf_size, int variant, const NearArgs& a,
                   const float4* pf, const float2* ph, int64_t items, hipStream_t s,
                   KernelMarks km = {});

void launch_leapfrog(int64_t n, double* x, double* v, const double* acc, double kick, double drift,
                     hipStream_t s);

// softened direct sum over all n sources for nt targets (targets == nullptr:
// 0..nt-1), the sources in nchunk chunks whose partial sums go to part
// ([nchunk][nt][4] doubles) and are added per target in chunk order; *status
// is cleared first (by a kernel) and an out-of-range target index sets
// ST_OVERFLOW in it
void launch_direct(int64_t n, const double* x, const double* m, const double* h, int64_t nt,
                   const int64_t* targets, double G, int include_self, double* acc, double* pot,
                   int* status, double* part, int nchunk, hipStream_t s);
// source chunks for nt targets: enough blocks to fill the chip, at most one
// per tile of 256 sources and at most what max_part_bytes of partial sums
// hold (0 when not even one chunk fits)
int direct_chunks(int64_t n, int64_t nt, uint64_t max_part_bytes);

// ---- momentum diagnostics ----------------------------------------------------
int momentum_blocks(int64_t n);
void launch_momentum(int n, const double* m, const double* acc, double* part, double* out,
                     hipStream_t s);

}  // namespace sfmm
