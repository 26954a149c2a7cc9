// Device helpers shared by the step kernels (kernels.hip) and the adjoint
// kernels (adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "common.hpp"

namespace ugk {

// The launches of step n carry K.gate = n and may be enqueued behind steps
// that have not run yet.  A launch from before the step's commit runs only
// when n steps have committed (after = 0), one from after it only when n + 1
// have (after = 1).  Behind a step that did not commit, every later step's
// launches therefore return at once and leave that step's state as its
// failure left it.  The value read is uniform, so whole grids return together.
// s = c sigma dt / eps^2 of a slot from its opacity, in one evaluation order:
// the coefficient tables store it and the sweeps re-form it from sigma alone
// (the same bits), so that they need not read both.
__device__ inline double s_of_sigma(const Consts& K, double sg) { return K.c * sg * K.dt / (K.eps * K.eps); }

__device__ inline bool gate_open(const Dev& D, const Consts& K, uint32_t after)
{
    return K.gate == GATE_OFF || *D.step == K.gate + after;
}

struct Slot {
    int inst, lcell, g;
    bool cell_ok, active;
};

// Slot j of a thread whose wavefront covers the 64 slots j & ~63 .. (j & ~63) + 63.
// Instance blocks start on multiples of 64, so those slots belong to one
// instance: it is looked up once per wavefront and its record is read with
// scalar loads.
__device__ inline Slot decode_slot(const Dev& D, const Consts& K, int64_t j)
{
    Slot s;
    const bool in = j < K.n_cg;
    const int w = __builtin_amdgcn_readfirstlane((int)(j >> 6));
    s.inst = ((int64_t)w << 6) < K.n_cg ? D.wave_inst[w] : K.n_inst - 1;
    const Inst& I = D.inst[s.inst];
    const int64_t local = j - I.cg_off;
    s.lcell = (int)(local >> I.lgGp);
    s.g = (int)(local & (I.Gp - 1));
    s.cell_ok = in && local >= 0 && s.lcell < I.ncell;
    s.active = s.cell_ok && s.g < I.G;
    return s;
}

// decode_slot, also handing out the slot's instance record: SINGLE (a context
// of one instance) takes it from the kernel arguments, with no memory read on
// the critical path; otherwise it comes from the instance table.
template <bool SINGLE>
__device__ inline Slot decode_slot_rec(const Dev& D, const Consts& K, int64_t j, Inst& I)
{
    Slot s;
    const bool in = j < K.n_cg;
    if (SINGLE) {
        s.inst = 0;
        I = K.inst0;
    } else {
        const int w = __builtin_amdgcn_readfirstlane((int)(j >> 6));
        s.inst = ((int64_t)w << 6) < K.n_cg ? D.wave_inst[w] : K.n_inst - 1;
        I = D.inst[s.inst];
    }
    const int64_t local = j - I.cg_off;
    s.lcell = (int)(local >> I.lgGp);
    s.g = (int)(local & (I.Gp - 1));
    s.cell_ok = in && local >= 0 && s.lcell < I.ncell;
    s.active = s.cell_ok && s.g < I.G;
    return s;
}

__device__ inline unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ inline double bitsd(unsigned long long v) { return __longlong_as_double((long long)v); }


// Largest value over the wavefront by DPP row steps: within quads, half rows,
// rows, then across rows (row broadcasts 15 and 31); lane 63 ends with the
// maximum, which is returned to every lane.
__device__ inline uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// A double moved across lanes by one DPP step; lanes of rows outside ROW_MASK,
// and lanes whose source is outside the row, read 0.0.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    int lo, hi;
    if (ROW_MASK == 0xF) {
        // every lane is written: no old value to set up
        lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    }
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over aligned groups of n lanes (n a power of two up to 64, the same in
// every lane).  Each step adds two partial sums that every lane of a group
// holds with the same bits, so all lanes of a group end with the same bits:
// pairs and quads (quad permutes), 8 and 16 lanes (half-row and row mirrors),
// then 32 and 64 lanes by shuffles.
__device__ inline double group_sum(double v, int n)
{
    if (n > 1) v += dpp_f64<0xB1, 0xF>(v);     // quad_perm 1,0,3,2
    if (n > 2) v += dpp_f64<0x4E, 0xF>(v);     // quad_perm 2,3,0,1
    if (n > 4) v += dpp_f64<0x141, 0xF>(v);    // row_half_mirror
    if (n > 8) v += dpp_f64<0x140, 0xF>(v);    // row_mirror
    if (n > 16) v += __shfl_xor(v, 16, WAVE);
    if (n > 32) v += __shfl_xor(v, 32, WAVE);
    return v;
}

// Sum over the wavefront, returned to every lane: the group steps up to rows,
// then the row broadcasts 15 and 31 gather the four row sums into lane 63.
__device__ inline double wave_sum(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);
    v += dpp_f64<0x4E, 0xF>(v);
    v += dpp_f64<0x141, 0xF>(v);
    v += dpp_f64<0x140, 0xF>(v);
    v += dpp_f64<0x142, 0xA>(v);               // row_bcast15 into rows 1, 3
    v += dpp_f64<0x143, 0xC>(v);               // row_bcast31 into rows 2, 3
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Largest of non-negative doubles (NaN allowed) over the wavefront, as IEEE bit
// patterns: for these the unsigned order of the bits is the numeric order, and
// every NaN lies above +inf, so a NaN anywhere wins.  The high words are
// reduced first, then the low words of the lanes that hold the largest high word.
__device__ inline unsigned long long wave_max_bits(double x)
{
    const unsigned long long b = dbits(x);
    const uint32_t hi = wave_max_u32((uint32_t)(b >> 32));
    const uint32_t lo = wave_max_u32((uint32_t)(b >> 32) == hi ? (uint32_t)b : 0u);
    return ((unsigned long long)hi << 32) | lo;
}

}  // namespace ugk
