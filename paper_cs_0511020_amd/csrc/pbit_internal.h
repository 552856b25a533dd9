// Internal types shared by the host planner and the kernels of libpbit.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace pbit {

constexpr uint32_t kNil = 0xFFFFFFFFu;

// Level 0 walks the node list; every node index that is a multiple of
// 2^kLog0 (and the head) starts a chain.
#ifndef PBIT_LOG0
#define PBIT_LOG0 4
#endif
#ifndef PBIT_LOGUP
#define PBIT_LOGUP 2
#endif
#ifndef PBIT_BASEMAX
#define PBIT_BASEMAX 8192
#endif
// Level-0 entries a walker keeps in registers between stores (half for
// 64-bit keys); the chain slots hold a multiple of it.
#ifndef PBIT_SEGLEN
#define PBIT_SEGLEN 32
#endif
constexpr uint32_t kLog0 = PBIT_LOG0;
// Levels >= 1 walk the list of chains of the level below.
constexpr uint32_t kLogUp = PBIT_LOGUP;
// Relink by node ranges: lists of 2^18 .. 2^25 nodes; ranges of 2^14 nodes
// (2^15 above 2^24 nodes), at most kRelinkRangesMax of them; tiles of
// kRelinkTile list positions in the bucketing kernel.
constexpr uint64_t kRelinkMinNodes = 1ull << 18;
constexpr uint64_t kRelinkMaxNodes = 1ull << 25;
constexpr uint32_t kRelinkRangesMax = 1024;
constexpr uint32_t kRelinkTile = 16384;
// The last level is ranked inside one workgroup's LDS.
constexpr uint32_t kBaseMax = PBIT_BASEMAX;
constexpr int kMaxLevels = 12;
// Chains longer than their level-0 slot that the unchain launch's first
// blocks take (each further one is walked by its own chain's group).
constexpr uint32_t kLongListMax = 16 * 256;
constexpr int kMaxPasses = 64;
// Many-list sorts.  Lists of more than a cutoff of nodes (at least
// kMinSegLen) take the digit passes as segments of one position array; the
// others are sorted in LDS, one workgroup each, with cutoffs of 1024, 2048 or
// 4096 nodes.
constexpr uint32_t kMinSegLen = 1024;
constexpr uint32_t kMaxCutoff = 4096;
// Lists per group of the per-list digit base scan.
constexpr uint32_t kSegChunk = 64;
// Segments whose digit counts one pack block keeps in LDS.
constexpr uint32_t kPackSlots = 8;
// Position -> segment table granularity (log2).
constexpr uint32_t kSegLog = 8;
// Sleeps a digit pass's look-back waits on one predecessor tile before it
// counts that tile's digit itself (default; pbit_set_lookback_spin_limit
// changes it, 0 makes every tile whose predecessor has not published yet
// take that fallback at once).
constexpr uint32_t kSpinLimit = 4096;

// Lookback words: 2 flag bits + 30-bit count.
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagPrefix = 2u << 30;
constexpr uint32_t kCountMask = (1u << 30) - 1u;

// List-order buffers: (key, node) pairs while passes remain, node indices
// alone after the last pass.  Packed: one 32-bit word per element, the last
// pass's digit in the top K bits over the node index (in the memory of pairs
// A or B), written by the last pass but one when the index fits 32 - K bits.
// Half: for 64-bit keys of one list, once the patterns of the low 32 bits are
// done, (high 32 key bits, node) pairs of 8 bytes in the memory of pairs A or
// B; the passes over the high half then run as 32-bit-key passes.
enum BufKind : uint32_t {
    kBufPairsA = 0, kBufPairsB = 1, kBufIdxA = 2, kBufIdxB = 3, kBufPackA = 4, kBufPackB = 5,
    kBufHalfA = 6, kBufHalfB = 7
};
constexpr bool buf_in_b(uint32_t k)
{
    return k == kBufPairsB || k == kBufPackB || k == kBufHalfB;
}
constexpr bool buf_packed(uint32_t k) { return k == kBufPackA || k == kBufPackB; }
constexpr bool buf_half(uint32_t k) { return k == kBufHalfA || k == kBufHalfB; }
constexpr bool buf_pairs(uint32_t k) { return k == kBufPairsA || k == kBufPairsB; }

struct PassSched {
    uint32_t skip;      // every element has the same digit: the pass is the identity
    uint32_t in_kind;   // BufKind read
    uint32_t out_kind;  // BufKind written
    uint32_t ballot;    // rank by ballots (one digit holds over 1/16 of the elements)
    uint32_t pk_shift;  // out_kind packed: bit position of the digit the word carries
};

// Device-side header at the start of the workspace (zeroed per sort).
struct Header {
    int32_t status;
    uint32_t final_kind;      // BufKind holding the sorted order
    uint32_t nil_count;       // next[] entries equal to NIL
    uint32_t expect_nil;      // many-list sorts: non-empty lists (one NIL each)
    uint32_t n_long;          // level-0 chains longer than their slot
    uint32_t n_segs;          // many-list sorts: lists that take the digit passes
    uint64_t hsum[2];         // sum of h(next) over non-NIL next[] minus sum of h(i)
    uint32_t seg_nodes;       // many-list sorts: their nodes
    uint32_t pad1;
    uint32_t seg_trivial[kMaxPasses];  // lists whose pattern p is one value for all nodes
    uint32_t pass_ticket[kMaxPasses];  // next tile of each digit pass, in block start order
    PassSched sched[kMaxPasses];
};

struct LevelPlan {
    uint32_t log_l;       // chain start spacing 2^log_l
    uint64_t m;           // elements at this level
    uint64_t n_static;    // chains (= elements of the next level)
    size_t o_chain_rec;   // uint2 {successor chain, weight} per chain
    size_t o_ent;         // level 0: stored head entries of every chain
    size_t o_resume;      // level 0: node where the unstored rest of a chain starts
    size_t o_long;        // level 0: {chain, resume node} of the first long chains
    uint32_t cap;         // level 0: entries stored per chain
    size_t o_offn;        // u32 offset (in nodes) of every chain
};

// Stages of one sort, in launch order (measurement hooks name them).
enum Stage : int32_t {
    kStageZero = 0, kStagePack, kStageWalk0, kStageWalkUp, kStageBase, kStageDown,
    kStageUnchain, kStageSchedule, kStagePass, kStageRelink,
    kStagePlan,   // many-list sorts: slab checks, segments, tables
    kStageSmall,  // short lists sorted in LDS (one list, or the short ones of many)
    kStageBases,  // many-list sorts: per-list digit bases
    kStageCommit, // many-list sorts: short lists' results copied out
    kStageCount
};

// Optional event recording between stages: events[i] is recorded before the
// i-th launched stage, and one more after the last stage.
struct Prof {
    void** events;   // hipEvent_t handles owned by the caller
    int32_t* ids;    // stage id of each recorded interval
    int n_events;
    int count;
};

struct Plan {
    uint64_t n;
    uint32_t M, K, RB, radix, passes, flags, key_bytes;
    uint32_t tile, tiles;
    uint32_t hi_from;     // one list of 64-bit keys: first pass over the high half (else passes)
    uint32_t tiles_hi;    // tiles of those passes (32-bit-key shape)
    uint32_t look_tiles;  // look-back words per pass and digit: max(tiles, tiles_hi)
    uint32_t spin_limit;  // look-back sleeps on one predecessor before the fallback
    uint32_t look64;      // 64-bit look-back words (counts of 2^30 and more)
    uint32_t num_lists;   // many-list sorts
    uint32_t log_block;   // many-list sorts: node block size of the list table
    uint32_t cutoff;      // many-list sorts: lists of at most this many nodes sort in LDS
    uint32_t seg_max;     // many-list sorts: most lists that can exceed the cutoff
    uint32_t seg_chunks;  // many-list sorts: groups of kSegChunk lists in the base scan
    uint32_t pack_chunk;  // many-list sorts: nodes per pack block
    int levels;           // walk levels; the base ranks level `levels`
    LevelPlan lv[kMaxLevels];
    size_t o_header, o_hist, o_dbase, o_look, zero_end;
    size_t o_nodes, o_pairsA, o_pairsB, o_idxA, o_idxB;
    // relink by node ranges (one list, 2^18 <= n <= 2^25): 2^relink_r nodes
    // per range; per tile of the bucketing kernel, the first slot of each
    // range's pairs ([range][tile]); relink_r = 0: the direct scatter
    uint32_t relink_r, relink_ranges, relink_tiles;
    size_t o_rstart;
    // many-list sorts
    size_t o_table, o_headbits;     // node -> list, head marks
    size_t o_lseg, o_segl, o_coff;  // list -> segment, segment -> list, segment offsets
    size_t o_ctable;                // position -> segment
    size_t o_lcnt, o_lbase, o_csum; // per-segment digit counts, bases, chunk sums
    size_t o_snext, o_shead;        // results of the lists sorted in LDS
    size_t total;
};

}  // namespace pbit
