// Host-side launch helpers shared by the single-list and many-list paths.
#pragma once
#include <hip/hip_runtime.h>

#include "pbit_device.h"

namespace pbit {

static inline void mark(Prof* prof, hipStream_t s, int32_t stage)
{
    if (!prof || prof->count >= prof->n_events)
        return;
    (void)hipEventRecord((hipEvent_t)prof->events[prof->count], s);
    if (prof->ids)
        prof->ids[prof->count] = stage;
    prof->count++;
}

// The key transform of the flags: the mask every key is XORed with after the
// floating-point transform (signed: the sign bit; descending: all bits), and
// the all-ones selector of that transform.
template <typename KeyT> static inline KeyT key_xor_mask(uint32_t flags)
{
    KeyT mask = 0;
    if (flags & PBIT_SIGNED)
        mask ^= (KeyT)((KeyT)1 << (sizeof(KeyT) * 8 - 1));
    if (flags & PBIT_DESCENDING)
        mask ^= (KeyT)~(KeyT)0;
    return mask;
}
template <typename KeyT> static inline KeyT key_float_sel(uint32_t flags)
{
    return (flags & PBIT_FLOAT) ? (KeyT)~(KeyT)0 : (KeyT)0;
}

static inline hipError_t launch_zero(const Plan& P, char* ws, hipStream_t s)
{
    const size_t words = (P.zero_end - P.o_header) / 4;
    const size_t want = (words + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (uint32_t*)(ws + P.o_header), words);
    return hipGetLastError();
}

template <typename KeyT, int RB, class Src>
static hipError_t launch_pack_rb(const Plan& P, const Src& src, char* ws, hipStream_t s)
{
    const KeyT mask = key_xor_mask<KeyT>(P.flags);
    const KeyT float_sel = key_float_sel<KeyT>(P.flags);
    const uint64_t want = (P.n + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 1024 ? want : 1024);
    const size_t shm = (size_t)P.passes * P.radix * sizeof(uint32_t);
    hipLaunchKernelGGL((k_pack<KeyT, RB, Src>), dim3(blocks), dim3(256), shm, s, src,
                       (uint32_t)P.n, float_sel, mask, P.passes, (NodeRec<KeyT>*)(ws + P.o_nodes),
                       (uint32_t*)(ws + P.o_hist), (Header*)(ws + P.o_header));
    return hipGetLastError();
}

template <typename KeyT, class Src>
static hipError_t launch_pack_src(const Plan& P, const Src& src, char* ws, hipStream_t s)
{
    switch (P.RB) {
    case 1: return launch_pack_rb<KeyT, 1>(P, src, ws, s);
    case 2: return launch_pack_rb<KeyT, 2>(P, src, ws, s);
    case 4: return launch_pack_rb<KeyT, 4>(P, src, ws, s);
    default: return launch_pack_rb<KeyT, 8>(P, src, ws, s);
    }
}

template <typename KeyT>
static hipError_t launch_pack(const Plan& P, const uint32_t* next, const void* keys, char* ws,
                              hipStream_t s)
{
    return launch_pack_src<KeyT>(P, DirectSrc<KeyT>{next, (const KeyT*)keys}, ws, s);
}

// The digit passes, least-significant pattern first.  One list: the
// schedule has run (as one extra block of the level-0 walk) unless
// `scheduled` is false.  SEG: many lists in segments, each pass with its
// per-segment base table (the schedule ran with the base scan).  One list of
// 64-bit keys: the passes from P.hi_from on (the high 32 key bits) run as
// 32-bit-key passes with the 32-bit tile shape.
template <typename KeyT, int RB, typename LW, bool SEG>
static hipError_t launch_passes_rb(const Plan& P, char* ws, hipStream_t s, Prof* prof,
                                   bool scheduled)
{
    constexpr int BLOCK = PassShape<KeyT, RB>::block;
    constexpr int ITEMS = PassShape<KeyT, RB>::items;
    constexpr int BLOCK_HI = PassShape<uint32_t, RB>::block;
    constexpr int ITEMS_HI = PassShape<uint32_t, RB>::items;
    constexpr uint32_t RADIX = 1u << RB;
    hipError_t e;
    if (!SEG && !scheduled) {
        mark(prof, s, kStageSchedule);
        hipLaunchKernelGGL((k_schedule<RB>), dim3(1), dim3(256), 0, s,
                           (const uint32_t*)(ws + P.o_hist), (uint32_t*)(ws + P.o_dbase),
                           P.passes, (uint32_t)P.n, (Header*)(ws + P.o_header), P.hi_from);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const uint32_t ticket = (P.flags & PBIT_SHARED) ? 1u : 0u;
    const uint32_t group = 8u * kPassChunk;
    auto grid_of = [&](uint32_t tiles) {
        return ticket ? tiles : (uint32_t)((tiles + group - 1) / group * group);
    };
    // the buffer each pass reads when no pattern is skipped (one list): the
    // pass loads its tile from there before it reads the schedule
    uint32_t exp_in[kMaxPasses];
    for (uint32_t p = 0; p < P.passes; p++)
        exp_in[p] = kNil;
    if (!SEG) {
        const uint32_t none[kMaxPasses] = {};
        pass_kinds(none, P.passes, P.n <= (1ull << (32 - RB)), RB, P.hi_from,
                   [&](uint32_t p, uint32_t in, uint32_t, uint32_t) { exp_in[p] = in; });
    }
    for (uint32_t p = 0; p < P.passes; p++) {
        LW* look = (LW*)(ws + P.o_look) + (size_t)p * P.look_tiles * RADIX;
        const uint32_t* dbase = SEG ? nullptr : (const uint32_t*)(ws + P.o_dbase) + (size_t)p * RADIX;
        SegMap sm{};
        if (SEG)
            sm = SegMap{(const uint32_t*)(ws + P.o_ctable), (const uint32_t*)(ws + P.o_coff),
                        (const uint32_t*)(ws + P.o_lbase) + (size_t)p * P.seg_max * RADIX};
        mark(prof, s, kStagePass);
        if constexpr (!SEG && sizeof(KeyT) == 8) {
            if (p >= P.hi_from) {
                hipLaunchKernelGGL(
                    (k_digit_pass<uint32_t, RB, BLOCK_HI, ITEMS_HI, LW, false, true>),
                    dim3(grid_of(P.tiles_hi)), dim3(BLOCK_HI), 0, s, p, p * RB - 32u,
                    (uint32_t)P.n, (Pair<uint32_t>*)(ws + P.o_pairsA),
                    (Pair<uint32_t>*)(ws + P.o_pairsB), (uint32_t*)(ws + P.o_idxA),
                    (uint32_t*)(ws + P.o_idxB), dbase, look, (Header*)(ws + P.o_header), sm,
                    P.spin_limit, ticket, exp_in[p]);
                if ((e = hipGetLastError()) != hipSuccess)
                    return e;
                continue;
            }
        }
        hipLaunchKernelGGL((k_digit_pass<KeyT, RB, BLOCK, ITEMS, LW, SEG>), dim3(grid_of(P.tiles)),
                           dim3(BLOCK), 0, s, p, p * RB, (uint32_t)P.n,
                           (Pair<KeyT>*)(ws + P.o_pairsA), (Pair<KeyT>*)(ws + P.o_pairsB),
                           (uint32_t*)(ws + P.o_idxA), (uint32_t*)(ws + P.o_idxB), dbase, look,
                           (Header*)(ws + P.o_header), sm, P.spin_limit, ticket, exp_in[p]);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename KeyT, typename LW, bool SEG>
static hipError_t launch_passes(const Plan& P, char* ws, hipStream_t s, Prof* prof,
                                bool scheduled = false)
{
    switch (P.RB) {
    case 1: return launch_passes_rb<KeyT, 1, LW, SEG>(P, ws, s, prof, scheduled);
    case 2: return launch_passes_rb<KeyT, 2, LW, SEG>(P, ws, s, prof, scheduled);
    case 4: return launch_passes_rb<KeyT, 4, LW, SEG>(P, ws, s, prof, scheduled);
    default: return launch_passes_rb<KeyT, 8, LW, SEG>(P, ws, s, prof, scheduled);
    }
}

// The buffers the relink may find the sorted order in.
template <typename KeyT> static OrderSrc order_src(const Plan& P, char* ws)
{
    constexpr uint32_t words = sizeof(Pair<KeyT>) / 4;
    static_assert(sizeof(Pair<KeyT>) == (sizeof(KeyT) == 8 ? 12 : 8), "pair layout");
    return OrderSrc{(const uint32_t*)(ws + P.o_pairsA) + (sizeof(KeyT) == 8 ? 2 : 1), words,
                    (const uint32_t*)(ws + P.o_idxA), (const uint32_t*)(ws + P.o_idxB)};
}

// Level-0 chains (lv[0]) to list order: stored entries and re-walked rests.
template <typename KeyT>
static hipError_t launch_unchain(const Plan& P, char* ws, hipStream_t s, Prof* prof)
{
    const LevelPlan& L = P.lv[0];
    const uint64_t threads = L.n_static * (kUnchainThreads / UnchainPer<KeyT>::value);
    mark(prof, s, kStageUnchain);
    hipLaunchKernelGGL((k_unchain<KeyT>), dim3(kLongBlocks + (uint32_t)((threads + 255) / 256)),
                       dim3(256), 0, s, (const uint2*)(ws + L.o_chain_rec),
                       (const Entry<KeyT>*)(ws + L.o_ent), (uint32_t)L.n_static, L.cap,
                       (const uint32_t*)(ws + L.o_offn), (uint32_t)P.n,
                       (const NodeRec<KeyT>*)(ws + P.o_nodes), (const uint32_t*)(ws + L.o_resume),
                       (const uint32_t*)(ws + L.o_long), (Pair<KeyT>*)(ws + P.o_pairsA),
                       (Header*)(ws + P.o_header));
    return hipGetLastError();
}

}  // namespace pbit
