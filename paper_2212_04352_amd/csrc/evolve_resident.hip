// evolve_resident.hip -- "resident" path of the fTWA time integration: every
// trajectory stays on chip for the whole horizon.
//
// Equation of motion: Eq. (6) of arXiv:2212.04352 with j_ij = t on bonds and
// u_ij = U delta_ij (Sec. II):
//   f_ij = i [ t (sum_{k in nb(j)} rho_ik - sum_{k in nb(i)} rho_kj) + U (d_i - d_j) rho_ij ],
// d = diagonal of the other spin, integrated with classical RK4.
//
// Layout on chip.  A workgroup holds UNITS "units"; a unit is one trajectory
// (S = 2: both spin blocks) or one spin block of one trajectory (S = 1, the
// partner workgroup holds the other spin).  The current Runge-Kutta stage
// input Y of a unit lives in LDS, one block of complex slots per spin: the
// P packed elements in "class order" (the even class -- diagonal first,
// element (i,i) at slot i -- then the odd class, see below), then slots that
// always hold zero (they stand in for missing neighbours: one, or for the
// spin split 32, one per LDS bank pair, so that the zero reads of a 32-lane
// group can avoid the banks its other lanes read), then a scratch slot owned
// by padding elements.  The base point y and the accumulator acc of every
// element live in the registers of the thread that owns it.  The U term reads the other
// spin's diagonal from slots 0..N-1 of its block (S = 2) or from a copy of
// the partner's diagonal placed before the block (S = 1; N reals ordered by
// sublattice, so the diagonal values read by a wave's consecutive
// same-sublattice sites sit in consecutive banks; two copies at a fixed
// distance, alternating by stage).  The kernel declares no static LDS, so
// block offsets are LDS addresses.
//
// Descriptors.  Each element has a descriptor with the LDS locations of its
// six neighbour elements and of itself, and of the two diagonal values: 32
// bytes of byte offsets, or, for the spin split, 16 bytes of 16-bit slot
// numbers and 8-bit diagonal positions (the descriptor stream is a large part
// of the kernel's memory traffic; each field becomes a byte offset with one
// sub-dword-select shift).  The LDS stores one orientation of every pair
// (chosen by a bandwidth-reducing site ranking); a neighbour stored as its
// transpose carries a flag, and its imaginary part enters the sums with the
// factor -1 (fma(+-1, v, s) rounds exactly like s +- v), so the arithmetic is
// that of the equation of motion in a fixed order.  The few elements with
// such neighbours come first in their class and fill the leading GE even and
// GO odd slots; all other slots are compiled without the flag handling.
// Consecutive threads own consecutive slots, so own reads and writes of a
// wave are contiguous; neighbours of consecutive same-class elements of a row
// are mostly consecutive slots of the other class.
//
// Two-phase stages.  The honeycomb is bipartite: an element (i, j) with i and
// j on the same sublattice ("even") reads only elements joining different
// sublattices ("odd") and vice versa.  Phase 1 updates the even elements and
// keeps their next-stage values in registers; after a barrier phase 2 updates
// the odd elements and writes their next values straight into LDS (nothing
// reads an odd element during phase 2 except its owner); after a second
// barrier the held even values are written.  Only half of the next-stage
// values is ever held, which is what lets the 198-site FP32 spin block live in
// one CU (157.6 KB of LDS, y/acc in VGPRs).  Each element's descriptor is
// loaded one or two elements ahead; every stage is compiled separately (no
// per-element tests of the stage number).
//
// Element slots.  Thread t of a unit owns element t + NTU*u of the even class
// for u < UE and of the odd class for UE <= u < UE + UO.  Both classes are
// padded to whole slots with dummy elements, so the stage loop carries no
// per-lane validity tests.
//
// Spin split (S = 1).  The two workgroups of a trajectory run on the same XCD
// and exchange only the N diagonal values per stage through a two-slot
// mailbox in global memory: the diagonal is even, so it is known after phase
// 1 and is published then, half a stage before the partner needs it.  Every
// mailbox word holds a value together with the number of the stage it belongs
// to, written and read with single 64-bit relaxed agent-scope atomics, so no
// fence (and no cache write-back or invalidation) is needed.  Waits are
// bounded; a timeout aborts both workgroups and is reported.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

struct ResidentArgs {
    const ResidentInst* table;  // entries (instance windows), item0 ascending
    int n_entries;
    int64_t n_items;            // total items over the table
    double dt;
    int64_t n_steps;
    int record_every;
    uint64_t* mailbox;          // S = 1: [pairs][2 spins][2 slots][Nmax] stage-stamped words
    int Nmax;
    uint32_t tail_off;          // LDS byte offset of the record sums and the abort flag
    int* error;                 // set to 1 when a wait times out
    unsigned spin_limit;        // polls before a bounded wait gives up
};

constexpr unsigned kSpinLimit = 1u << 26;  // default: ~2 s of polling

// Descriptor table as a global-address-space pointer.  It is passed through
// an SGPR every phase ("laundered") so that the compiler re-reads descriptors
// instead of keeping one address or index register per slot alive across the
// time loop; keeping the address space lets the loads use a scalar base plus
// the one per-thread offset shared by all slots.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(1))) ResDesc* gdesc_t;
#else
typedef const ResDesc* gdesc_t;  // host pass of the kernel source only
#endif

// A value the compiler cannot prove wave-uniform (read from the launch
// table) moved into scalar registers: every lane holds the same value.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <typename T> __device__ __forceinline__ T uniform_real(T v);
template <> __device__ __forceinline__ float uniform_real<float>(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
template <> __device__ __forceinline__ double uniform_real<double>(double v) {
    return __longlong_as_double((long long)uniform64((uint64_t)__double_as_longlong(v)));
}

__device__ __forceinline__ gdesc_t launder(gdesc_t p) {
    uint64_t v = (uint64_t)p;
    __asm__ volatile("" : "+s"(v)::"memory");
    return (gdesc_t)v;
}

__device__ __forceinline__ ResDesc load_desc(gdesc_t p) {
    ResDesc d;
    d.a = p->a;
    d.b = p->b;
    return d;
}

// Descriptor of slot `slot` of this thread: a wave-uniform slot base (scalar
// registers, opaque so that it stays one) plus the thread's 32-bit byte
// offset, the same for every slot.
__device__ __forceinline__ ResDesc slot_desc(gdesc_t desc, int slot, uint32_t toff) {
    uint64_t b = (uint64_t)(desc + slot);
    __asm__("" : "+s"(b));
    const __attribute__((address_space(1))) char* base =
        (const __attribute__((address_space(1))) char*)b;
    return load_desc((gdesc_t)(base + toff));
}

// The stage loop's descriptor reads: buffer loads with the slot base in a
// scalar offset and the thread's byte offset in a vector register (no
// per-thread address arithmetic).  DT = ResDesc (wide) or uint4 (compact).
template <typename DT>
__device__ __forceinline__ DT slot_desc_buf(__amdgpu_buffer_rsrc_t r, int slot, uint32_t toff) {
    constexpr int B = (int)sizeof(DT);
    if constexpr (B == 16) {
        return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, toff, slot * B, 0));
    } else {
        ResDesc d;
        d.a = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, toff, slot * B, 0));
        d.b = __builtin_bit_cast(uint4,
                                 __builtin_amdgcn_raw_buffer_load_b128(r, toff, slot * B + 16, 0));
        return d;
    }
}

// Byte offset = 16-bit field (low or high half of w) x 8, and diagonal word
// offset = byte field 2 or 3 of w x 4: one VALU instruction each (a
// sub-dword operand select).
__device__ __forceinline__ uint32_t lo16x8(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:WORD_0" : "=v"(r) : "v"(w));
    return r;
}
__device__ __forceinline__ uint32_t hi16x8(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:WORD_1" : "=v"(r) : "v"(w));
    return r;
}
__device__ __forceinline__ uint32_t b2x4(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:BYTE_2" : "=v"(r) : "v"(w));
    return r;
}
__device__ __forceinline__ uint32_t b3x4(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:BYTE_3" : "=v"(r) : "v"(w));
    return r;
}

// One element's stencil in LDS byte offsets: n[0..2] the column neighbours,
// n[3..5] the row neighbours (with GEN: bit 31 = read the conjugate), own the
// element's slot (within its spin block), di, dj the diagonal values of the
// U term (within the diagonal array).
struct Stencil {
    uint32_t n[6];
    uint32_t own, di, dj;
};

template <bool GEN> __device__ __forceinline__ Stencil decode(const ResDesc& d) {
    Stencil e;
    e.n[0] = d.a.x;
    e.n[1] = d.a.y;
    e.n[2] = d.a.z;
    e.n[3] = d.b.x;
    e.n[4] = d.b.y;
    e.n[5] = d.b.z;
    e.own = d.a.w;
    e.di = d.b.w & 0xffffu;
    e.dj = d.b.w >> 16;
    return e;
}
template <bool GEN> __device__ __forceinline__ Stencil decode(const uint4& w) {
    Stencil e;
    const uint32_t f[3] = {w.x, w.y, w.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if constexpr (GEN) {
            e.n[2 * k] = ((f[k] & 0x7fffu) << 3) | ((f[k] & 0x8000u) << 16);
            e.n[2 * k + 1] = ((f[k] >> 13) & 0x3fff8u) | (f[k] & 0x80000000u);
        } else {
            e.n[2 * k] = lo16x8(f[k]);
            e.n[2 * k + 1] = hi16x8(f[k]);
        }
    }
    e.own = lo16x8(w.w);
    e.di = b2x4(w.w);
    e.dj = b3x4(w.w);
    return e;
}

// Conjugation by bit 31 of a neighbour offset: the imaginary part enters the
// neighbour sums with the factor -1 (+1 otherwise).  The factor is formed
// from the descriptor alone, so all LDS reads of an element can be issued
// before any of their values is needed; fma(+-1, v, s) rounds exactly like
// s +- v.
template <typename T> __device__ __forceinline__ T conj_sign(uint32_t f);
template <> __device__ __forceinline__ float conj_sign<float>(uint32_t f) {
    return __uint_as_float((f & 0x80000000u) | 0x3f800000u);
}
template <> __device__ __forceinline__ double conj_sign<double>(uint32_t f) {
    return __hiloint2double((int)((f & 0x80000000u) | 0x3ff00000u), 0);
}

template <typename T>
__device__ __forceinline__ cplx_t<T> lds_at(const unsigned char* base, uint32_t f) {
    return *reinterpret_cast<const cplx_t<T>*>(base + (f & 0x7fffffffu));
}

// Right-hand side of one element from its stencil: Yb is the LDS block of its
// spin, Yd the diagonal array of the U term.  Sums as in the equation of
// motion: col = (v0 + v1) + v2 over the column neighbours, row likewise.
// GEN: a neighbour may be stored as its transpose (its imaginary part enters
// with the factor -1); otherwise no offset carries a flag and the sums are
// plain (fma(1, v, s) and s + v round alike, so both forms give the same
// bits).  The element's own value is read from LDS, or taken from `own`
// (OWN_REG).
// POT: an external on-site potential adds A (v_i - v_j) to the U factor (Vd:
// the profile v in the layout of the diagonal array, Aw: the envelope at the
// stage time; only when `pot_on`).
// HOP: complex hopping j_ik = t w_ik: col = sum_n w_jn x_n over
// the column neighbours x_n = rho_ik, row = sum_n conj(w_in) rho_kj, each
// product as (fma(wr, xr, -(wi xi)), fma(wr, xi, wi xr)), slots summed in
// order; Wt: this stage's ratio table, three complex ratios per site at the
// site's position in the diagonal array that the descriptors index (spin
// split: its place; shared blocks: the site), zero for a missing neighbour.
// The ratio table of one stage: base and size in bytes in global memory (read
// through a buffer resource: 32-bit offsets, its own wait counter), and its
// copy in LDS (`lds`): the triples whose diagonal offset is below lds_end
// (spin split: the first kHopLds places; otherwise the whole table) are read
// there.
struct HopTab {
    const unsigned char* p = nullptr;
    int bytes = 0;
    const unsigned char* lds = nullptr;
    uint32_t lds_end = 0;
    uint32_t mul = 6;  // diagonal offset -> triple offset (6: place x sizeof(T); 3: site x sizeof(C))
};

// A site's three ratios (24 bytes in FP32, 48 in FP64, at byte offset `off`).
__device__ __forceinline__ void ratio_triple(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                             cplx_t<double>* w) {
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const double2 a =
            __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * n, 0, 0));
        w[n].x = a.x;
        w[n].y = a.y;
    }
}
__device__ __forceinline__ void ratio_triple(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                             cplx_t<float>* w) {
    const float4 a = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const float2 b =
        __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off + 16, 0, 0));
    w[0].x = a.x;
    w[0].y = a.y;
    w[1].x = a.z;
    w[1].y = a.w;
    w[2].x = b.x;
    w[2].y = b.y;
}

template <typename T>
__device__ __forceinline__ cplx_t<T> hop_mul(cplx_t<T> w, cplx_t<T> x) {
    cplx_t<T> r;
    r.x = fma_rn<T>(w.x, x.x, -(w.y * x.y));
    r.y = fma_rn<T>(w.x, x.y, w.y * x.x);
    return r;
}

// Four consecutive values of T from LDS (16-byte aligned): one 16-byte read
// in FP32, two in FP64.
template <typename T>
__device__ __forceinline__ void quad_lds(const unsigned char* p, T* out) {
    if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        out[0] = v.x;
        out[1] = v.y;
        out[2] = v.z;
        out[3] = v.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 16);
        out[0] = a.x;
        out[1] = a.y;
        out[2] = b.x;
        out[3] = b.y;
    }
}

// The six ratios of an element from a ratio table held whole in LDS (the
// shared-block tiles): j's triple, then i's, unconjugated.
template <typename T>
__device__ __forceinline__ void ratios_lds(const HopTab& Wt, uint32_t di, uint32_t dj,
                                           cplx_t<T>* w) {
    const cplx_t<T>* a = reinterpret_cast<const cplx_t<T>*>(Wt.lds + __umul24(dj, Wt.mul));
    const cplx_t<T>* b = reinterpret_cast<const cplx_t<T>*>(Wt.lds + __umul24(di, Wt.mul));
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        w[n] = a[n];
        w[n + 3] = b[n];
    }
}

// WPRE (with HOP): the element's six ratios come in `wpre` (ratios_lds), read
// once for both spin blocks of a shared-block tile, which share them.
template <typename T, bool OWN_REG, bool GEN, bool T1, bool POT = false, bool HOP = false,
          bool WPRE = false>
__device__ __forceinline__ cplx_t<T> element_rhs(const unsigned char* Yb, const unsigned char* Yd,
                                                 const Stencil& e, T t, T U, cplx_t<T> own,
                                                 const unsigned char* Vd = nullptr, T Aw = 0,
                                                 bool pot_on = false,
                                                 HopTab Wt = {}, const cplx_t<T>* wpre = nullptr) {
    using C = cplx_t<T>;
    C col, row;
    if constexpr (HOP && WPRE) {
        C x[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            x[n] = GEN ? lds_at<T>(Yb, e.n[n]) : *reinterpret_cast<const C*>(Yb + e.n[n]);
            if constexpr (GEN) x[n].y = conj_sign<T>(e.n[n]) * x[n].y;
        }
        C p[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            C w = wpre[n];
            if (n >= 3) w.y = -w.y;
            p[n] = hop_mul<T>(w, x[n]);
        }
        col = cadd(cadd(p[0], p[1]), p[2]);
        row = cadd(cadd(p[3], p[4]), p[5]);
    } else if constexpr (HOP) {
        // Ratios of the element's sites: j's for the column sums, i's
        // (conjugated) for the row sums.  A ratio triple is 3 sizeof(C) =
        // 6 sizeof(T); the diagonal offsets are site places x sizeof(T) (spin
        // split: Wt.mul = 6) or sites x sizeof(C) (shared blocks: Wt.mul = 3),
        // < 4096, so the product fits 24 bits.  Offsets below Wt.lds_end
        // come from the stage's copy in LDS, the others from global memory:
        // every lane reads LDS (at place 0 when its site is not there) and
        // only the other lanes then issue the global loads, which overwrite
        // those values, so the texture unit sees the global reads alone.
        const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
            (void*)Wt.p, (short)0, Wt.bytes, 0x00020000);
        auto triple = [&](uint32_t d, C* w) {
            const uint32_t o = __umul24(d, Wt.mul);
            const bool in_lds = d < Wt.lds_end;
            const C* l = reinterpret_cast<const C*>(Wt.lds + (in_lds ? o : 0u));
            w[0] = l[0];
            w[1] = l[1];
            w[2] = l[2];
            if (!in_lds) ratio_triple(wr, o, w);
        };
        C x[6], w[6];
        triple(e.dj, w);
        triple(e.di, w + 3);
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            x[n] = GEN ? lds_at<T>(Yb, e.n[n]) : *reinterpret_cast<const C*>(Yb + e.n[n]);
            if constexpr (GEN) x[n].y = conj_sign<T>(e.n[n]) * x[n].y;
        }
        C p[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            if (n >= 3) w[n].y = -w[n].y;
            p[n] = hop_mul<T>(w[n], x[n]);
        }
        col = cadd(cadd(p[0], p[1]), p[2]);
        row = cadd(cadd(p[3], p[4]), p[5]);
    } else if constexpr (GEN) {
        const C c0 = lds_at<T>(Yb, e.n[0]), c1 = lds_at<T>(Yb, e.n[1]), c2 = lds_at<T>(Yb, e.n[2]);
        const C r0 = lds_at<T>(Yb, e.n[3]), r1 = lds_at<T>(Yb, e.n[4]), r2 = lds_at<T>(Yb, e.n[5]);
        col.x = (c0.x + c1.x) + c2.x;
        col.y = fma_rn<T>(conj_sign<T>(e.n[2]), c2.y,
                          fma_rn<T>(conj_sign<T>(e.n[1]), c1.y, conj_sign<T>(e.n[0]) * c0.y));
        row.x = (r0.x + r1.x) + r2.x;
        row.y = fma_rn<T>(conj_sign<T>(e.n[5]), r2.y,
                          fma_rn<T>(conj_sign<T>(e.n[4]), r1.y, conj_sign<T>(e.n[3]) * r0.y));
    } else {
        const C c0 = *reinterpret_cast<const C*>(Yb + e.n[0]);
        const C c1 = *reinterpret_cast<const C*>(Yb + e.n[1]);
        const C c2 = *reinterpret_cast<const C*>(Yb + e.n[2]);
        const C r0 = *reinterpret_cast<const C*>(Yb + e.n[3]);
        const C r1 = *reinterpret_cast<const C*>(Yb + e.n[4]);
        const C r2 = *reinterpret_cast<const C*>(Yb + e.n[5]);
        col.x = (c0.x + c1.x) + c2.x;
        col.y = (c0.y + c1.y) + c2.y;
        row.x = (r0.x + r1.x) + r2.x;
        row.y = (r0.y + r1.y) + r2.y;
    }
    const C rho = OWN_REG ? own : *reinterpret_cast<const C*>(Yb + e.own);
    const T di = *reinterpret_cast<const T*>(Yd + e.di);
    const T dj = *reinterpret_cast<const T*>(Yd + e.dj);
    T a = U * (di - dj);
    if constexpr (POT) {
        if (pot_on)
            a = a + Aw * (*reinterpret_cast<const T*>(Vd + e.di) -
                          *reinterpret_cast<const T*>(Vd + e.dj));
    }
    if constexpr (T1) {
        // t = 1: t * x is x exactly, the hopping sums enter unscaled
        cplx_t<T> f;
        const T gr = fma_rn<T>(a, rho.x, col.x - row.x);
        const T gi = fma_rn<T>(a, rho.y, col.y - row.y);
        f.x = -gi;
        f.y = gr;
        return f;
    }
    return rhs_element<T>(col, row, rho, t, a);
}

// The element's own slot offset from its descriptor.
__device__ __forceinline__ uint32_t own_off(const ResDesc& d) { return d.a.w; }
__device__ __forceinline__ uint32_t own_off(const uint4& w) { return lo16x8(w.w); }
// Its two diagonal offsets (i's and j's; the wide descriptors of the shared
// blocks only, where they do not depend on the general form).
__device__ __forceinline__ uint32_t own_di(const ResDesc& d) { return d.b.w & 0xffffu; }
__device__ __forceinline__ uint32_t own_dj(const ResDesc& d) { return d.b.w >> 16; }
__device__ __forceinline__ uint32_t own_di(const uint4&) { return 0; }
__device__ __forceinline__ uint32_t own_dj(const uint4&) { return 0; }

// The same with the variant chosen by a (compile-time) slot condition.
template <typename T, bool OWN_REG, bool T1, typename DT, bool POT = false, bool HOP = false,
          bool WPRE = false>
__device__ __forceinline__ cplx_t<T> element_rhs_sel(bool gen, const unsigned char* Yb,
                                                     const unsigned char* Yd, const DT& d,
                                                     T t, T U, cplx_t<T> own,
                                                     const unsigned char* Vd = nullptr, T Aw = 0,
                                                     bool pot_on = false,
                                                     HopTab Wt = {},
                                                     const cplx_t<T>* wpre = nullptr) {
    return gen ? element_rhs<T, OWN_REG, true, T1, POT, HOP, WPRE>(Yb, Yd, decode<true>(d), t, U,
                                                                    own, Vd, Aw, pot_on, Wt, wpre)
               : element_rhs<T, OWN_REG, false, T1, POT, HOP, WPRE>(Yb, Yd, decode<false>(d), t,
                                                                     U, own, Vd, Aw, pot_on, Wt,
                                                                     wpre);
}

// One Runge-Kutta stage update of an element from its slope k:
//   stage 1: acc = k;                 next = fma(c, k, y)
//   stage 2, 3: acc = fma(2, k, acc); next = fma(c, k, y)
//   stage 4: acc = acc + k;           y = fma(c, acc, y); next = y
template <int STAGE, typename T>
__device__ __forceinline__ cplx_t<T> rk_update(T c, cplx_t<T> k, cplx_t<T>& y, cplx_t<T>& acc) {
    cplx_t<T> nx;
    if constexpr (STAGE == 1) {
        acc = k;
    } else if constexpr (STAGE < 4) {
        acc.x = fma_rn<T>((T)2, k.x, acc.x);
        acc.y = fma_rn<T>((T)2, k.y, acc.y);
    } else {
        acc.x = acc.x + k.x;
        acc.y = acc.y + k.y;
    }
    if constexpr (STAGE < 4) {
        nx.x = fma_rn<T>(c, k.x, y.x);
        nx.y = fma_rn<T>(c, k.y, y.y);
    } else {
        y.x = fma_rn<T>(c, acc.x, y.x);
        y.y = fma_rn<T>(c, acc.y, y.y);
        nx = y;
    }
    return nx;
}

template <typename T> __device__ __forceinline__ unsigned to_bits(T v);
template <> __device__ __forceinline__ unsigned to_bits<float>(float v) { return __float_as_uint(v); }
template <typename T> __device__ __forceinline__ T from_bits(unsigned v);
template <> __device__ __forceinline__ float from_bits<float>(unsigned v) { return __uint_as_float(v); }

template <int V> using stage_c = std::integral_constant<int, V>;

// Pins a register value at this point of the program: it is computed here
// (not sunk past a barrier, where it would be live together with the next
// phase's values).
template <typename C> __device__ __forceinline__ void pin(C& v) {
    __asm__ volatile("" : "+v"(v.x), "+v"(v.y));
}

// Generic pointer to LDS byte address `a` (the kernel's dynamic LDS block
// starts at address 0).
__device__ __forceinline__ unsigned char* lds_ptr(uint32_t a) {
    return (unsigned char*)(__attribute__((address_space(3))) unsigned char*)(uintptr_t)a;
}

// T1: every instance of the launch has t = 1 (the usual unit of energy).
// POT: entries may carry an external on-site potential; its profile sits in
// LDS in the layout of the diagonal that the descriptors index (spin split:
// after the partner's diagonal copies; shared blocks: after the blocks, site
// i at i sizeof(C)).
// HOP: every entry carries complex hopping (ResidentInst::hop: the ratio
// table hop_table_kernel prepared; spin split: each stage's first kHopLds
// places copied into LDS, the rest read from global memory; shared blocks:
// the whole stage table in LDS, an element's ratios read once for both
// spins).
// GINT: every entry carries a general interaction u_ij (ResidentInst::umat,
// u rounded to T, blocked by four along k: [k/4][i][4]): each stage starts
// with D_i = sum_k u_ki (d_k + 1/2) over the partner's diagonal, one
// ascending fused chain per site (and spin, shared blocks), into LDS (spin
// split: after the diagonal copies, in their layout; shared blocks: after
// the blocks, at the element stride), and the U factor of an element is
// D_i - D_j (U = 1 exactly).
// Places whose complex-hopping ratios (three FP32 complex numbers, 24 bytes)
// a stage keeps in LDS: the most that fit beside a 198-site spin block (its
// elements, the two diagonal copies and the record sums leave 3,712 bytes of
// the 160 KB); the table's later places are read from global memory.
constexpr int kHopLds = 152;

// Minimum waves per SIMD the compiler must leave room for.  The FP32 tiles of
// units of 64 threads (lattices up to 15 sites) hold little state per
// thread: at 64 registers eight waves share a SIMD instead of four (with 16
// units: 10 % faster at 12 sites with eight scratch accesses per lane and
// RK4 step).  Its Hamiltonian variants (VAR) spill two to three times
// as much there and keep four waves.  Every other tile keeps the register
// file for its state (the same hint spills FP64 and larger tiles and makes
// them 2-5x slower).
template <typename T, int S, int NTU, int UNITS, bool VAR>
constexpr int resident_min_waves() {
    return std::is_same<T, float>::value && S == 2 && NTU == 64 && !VAR ? 8 : 1;
}

template <typename T, int S, int NTU, int UNITS, int UE, int UO, int GE, int GO, bool T1,
          bool POT = false, bool HOP = false, bool GINT = false>
__global__ __launch_bounds__(NTU * UNITS)
__attribute__((amdgpu_waves_per_eu(resident_min_waves<T, S, NTU, UNITS, POT || HOP || GINT>(), 8)))
void rk4_resident(ResidentArgs A) {
    using C = cplx_t<T>;
    // descriptor form: compact for the spin split, wide otherwise
    using DT = std::conditional_t<S == 1, uint4, ResDesc>;
    static_assert(S == 2 || UNITS == 1, "the spin split holds one spin block per workgroup");
    static_assert(!HOP || !POT, "complex hopping without a potential");
    static_assert(!GINT || (!POT && !HOP), "a general interaction alone");
    constexpr int kEvenPad = NTU * UE;
    constexpr int CB = (int)sizeof(C);
    constexpr int TB = (int)sizeof(T);
    constexpr uint32_t kDiagCopy = 256 * TB;  // S = 1: one copy of the partner's diagonal
    constexpr int kTail = S == 1 ? 33 : 2;    // slots after the elements: zero(s), scratch
    extern __shared__ __align__(16) unsigned char smem[];  // dynamic LDS, at address 0
    (void)smem;
    const int tid0 = threadIdx.x;

    // Persistent schedule.  S = 2: workgroup b takes items b, b + grid, ...
    // (an item is UNITS consecutive trajectories of one table entry).  S = 1:
    // the two workgroups of pair p (same XCD: blocks b and b + 8 of a group of
    // 16) take items p, p + n_pairs, ... (an item is one trajectory), in the
    // same order, so their stage counters stay equal.
    int spin0 = 0;
    int pair = 0;
    int64_t first, stride;
    if constexpr (S == 1) {
        const int b = blockIdx.x, xcd = b % 8, k = b / 8;
        spin0 = k % 2;
        pair = (k / 2) * 8 + xcd;
        first = pair;
        stride = gridDim.x / 2;
    } else {
        first = blockIdx.x;
        stride = gridDim.x;
    }
    if (tid0 == 0) *reinterpret_cast<int*>(lds_ptr(A.tail_off + (NTU * UNITS / 64) * 2 * S * 8)) = 0;
    uint64_t* const mb = A.mailbox;
    int64_t g = 0;  // stage counter (continues across items)

    C y[S][UE + UO], acc[S][UE + UO], hold[S][UE];

    for (int64_t item = first; item < A.n_items; item += stride) {
        // thread coordinates are re-derived every item (an opaque copy of the
        // thread index), so that per-slot offsets are not hoisted out of the
        // item loop and kept in registers across it
        const int tid = tid0;
        const int unit = UNITS == 1 ? 0 : tid / NTU;
        const int t = UNITS == 1 ? tid : tid % NTU;
        const uint32_t toff = (uint32_t)t * (uint32_t)sizeof(DT);
        const int lane = tid % 64;
        const int wave = tid / 64;

        // table entry of this item (uniform: scalar loads)
        int ent = 0;
        while (ent + 1 < A.n_entries && A.table[ent + 1].item0 <= item) ++ent;
        ent = __builtin_amdgcn_readfirstlane(ent);
        const ResidentInst& E = A.table[ent];
        const int N = E.N;
        const int P = E.P;
        const int Pb = P + kTail;  // per block: P elements, the zero slot(s), the scratch slot
        // LDS: UNITS x S blocks of Pb complex slots; S = 1: two copies of the
        // partner's diagonal (N reals, sublattice-major, kDiagCopy bytes
        // apart) first, then the block.  The launch has no static LDS, so the
        // dynamic block starts at LDS address 0 and offsets are addresses (no
        // base register; constant offsets go into the instructions).
        // S = 1: two diagonal copies, then the potential's profile (POT), or
        // D and two site-ordered copies of the partner's diagonal (GINT), or
        // the first kHopLds places' ratios of the stage's table (HOP)
        constexpr uint32_t kPre =
            S == 1 ? (HOP ? 2 * kDiagCopy + kHopLds * 6 * TB
                          : (GINT ? 5 : POT ? 3 : 2) * kDiagCopy)
                   : 0;
        unsigned char* const Yunit = lds_ptr((uint32_t)(kPre + (size_t)unit * S * Pb * CB));
        // S = 2: after the blocks of all units, D of every unit and spin
        // (GINT: [unit][spin][site] at the element stride, so that the
        // descriptors' diagonal offsets index it), the stage's ratio table in
        // site order (HOP) or the potential's profile (POT, [site] at the
        // element stride)
        unsigned char* const xarea = lds_ptr(((uint32_t)(UNITS * S * Pb * CB) + 15u) & ~15u);
        // S = 2 with a general interaction: then a copy of u in its staged
        // layout and h = d + 1/2 of every unit's two diagonals in site order
        // ([unit][spin][k], zero from N up to u's padded row count KU), where
        // the plan made room for them (E.u_lds)
        unsigned char* const uarea = xarea + ((UNITS * 2 * N * CB + 15) & ~15);
        const int KU = umat_rows(N);
        T* const hsv = reinterpret_cast<T*>(uarea + (size_t)KU * N * TB);
        // GINT: h_k = d_k + 1/2 of the partner's diagonal in site order, copy c
        // (stage parity), zero from N up to the u table's padded row count
        auto dsite = [&](int c) { return reinterpret_cast<T*>(lds_ptr((3 + c) * kDiagCopy)); };
        unsigned char* const dpart = lds_ptr(0);
        // per-wave partial sums of the records and the abort flag follow
        // (placed after the largest blocks of the launch: A.tail_off)
        double (*red)[2 * S] = reinterpret_cast<double (*)[2 * S]>(lds_ptr(A.tail_off));
        int& abort_flag = *reinterpret_cast<int*>(lds_ptr(A.tail_off + (NTU * UNITS / 64) * 2 * S * 8));
        const int64_t Mc = E.Mc;
        const int64_t m = (item - E.item0) * (S == 1 ? 1 : UNITS) + (S == 1 ? 0 : unit);
        const bool active = m < Mc;
        C* const rho = reinterpret_cast<C*>(uniform64((uint64_t)E.rho));
        const int64_t ldr = E.ldr;
        double* const Xrec = E.X;
        double* const inv_parts = E.inv_parts;
        gdesc_t desc = (gdesc_t)uniform64((uint64_t)E.desc);
        // LDS byte offset (within its spin block) of the element in
        // descriptor entry e
        auto own_at = [&](gdesc_t dt, int e) -> uint32_t {
            if constexpr (S == 1)
                return (reinterpret_cast<const uint4*>((uint64_t)dt)[e].w & 0xffffu) *
                       (uint32_t)CB;
            else
                return dt[e].a.w;
        };
        auto own_of = [&](int e) -> uint32_t { return own_at(desc, e); };
        __syncthreads();  // the previous item is done with LDS and `red`

        // packed index of the element a descriptor describes (its LDS slot
        // through the class-order table), for the state in HBM
        const uint32_t* const ord = reinterpret_cast<const uint32_t*>(uniform64((uint64_t)E.ord));
        const int32_t* const nbt = reinterpret_cast<const int32_t*>(uniform64((uint64_t)E.nb));

        // (the LDS holds rho_ab; rho_ba when b < a is the packed element, so
        // it is conjugated on the way in and out)
        auto packed_of = [&](uint32_t own, bool& transposed) -> int64_t {
            const uint32_t ab = ord[own / CB];
            const int a = (int)(ab & 0xffffu), b = (int)(ab >> 16);
            const int i = a < b ? a : b, j = a < b ? b : a;
            transposed = a > b;
            return (int64_t)i * N - (int64_t)i * (i - 1) / 2 + (j - i);
        };
        // ---- load the trajectory into registers and LDS
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int gs = spin0 + s;
#pragma unroll
            for (int u = 0; u < UE + UO; ++u) {
                const int e = u < UE ? t + NTU * u : kEvenPad + t + NTU * (u - UE);
                const uint32_t own = own_of(e);
                C v;
                v.x = 0;
                v.y = 0;
                if (active && own < (uint32_t)P * CB) {
                    bool tr;
                    const int64_t p = packed_of(own, tr);
                    v = rho[((int64_t)gs * P + p) * ldr + m];
                    if (tr) v.y = -v.y;
                }
                *reinterpret_cast<C*>(Yunit + s * Pb * CB + own) = v;  // dummies: scratch slot
                y[s][u] = v;
                acc[s][u] = v;
                if (u < UE) hold[s][u] = v;  // S = 1 writes held values in phase 1
            }
            // the zero slot(s) and the scratch slot after the elements (the
            // compact descriptors of the spin split use 32 zero slots)
            if (t < kTail) {
                C z;
                z.x = 0;
                z.y = 0;
                reinterpret_cast<C*>(Yunit + s * Pb * CB)[P + t] = z;
            }
        }
        const int32_t* const dpos = reinterpret_cast<const int32_t*>(uniform64((uint64_t)E.dpos));
        const int qdiag = (S == 1 && tid < N) ? dpos[tid] : 0;  // this thread's polled site
        // external potential of this entry: its profile in the diagonal's
        // layout (spin split: after the diagonal copies; shared blocks: in the
        // area after the blocks, one value per site at the element stride),
        // the envelope read per stage
        const double* const venv = POT ? reinterpret_cast<const double*>(uniform64((uint64_t)E.v_env))
                                       : nullptr;
        const bool pot_on = POT && E.v_site != nullptr;
        unsigned char* const vpart = S == 1 ? lds_ptr(2 * kDiagCopy) : xarea;
        if constexpr (POT) {
            const double* const vs = reinterpret_cast<const double*>(uniform64((uint64_t)E.v_site));
            if constexpr (S == 1) {
                for (int i = t; i < N; i += NTU)
                    reinterpret_cast<T*>(vpart)[dpos[i]] = pot_on ? (T)vs[i] : (T)0;
            } else {
                for (int i = tid; i < N; i += NTU * UNITS)
                    *reinterpret_cast<T*>(vpart + (size_t)i * CB) = pot_on ? (T)vs[i] : (T)0;
            }
        }
        // complex hopping: the prepared ratio tables, [2 n_steps + 1][N][3]
        const unsigned char* const hop_tab =
            HOP ? reinterpret_cast<const unsigned char*>(uniform64((uint64_t)E.hop)) : nullptr;
        // general interaction: u in T, blocked [k/4][i][4] (spin split: D goes
        // where the profile would)
        const T* const utab = GINT ? reinterpret_cast<const T*>(uniform64((uint64_t)E.umat)) : nullptr;
        const bool u_lds = GINT && S == 2 && E.u_lds != 0;
        if constexpr (GINT && S == 2) {
            // u into LDS once per item (16-byte words; visible after the
            // barrier that follows the first record)
            if (u_lds) {
                const uint4* src = reinterpret_cast<const uint4*>(utab);
                const int n16 = KU * N * TB / 16;
                for (int k = tid; k < n16; k += NTU * UNITS)
                    reinterpret_cast<uint4*>(uarea)[k] = src[k];
                // h of the first stage input (slot 0 of thread t < N holds
                // site t's diagonal)
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (t < N) hsv[(unit * 2 + s) * KU + t] = y[s][0].x + (T)0.5;
                    for (int k = N + t; k < KU; k += NTU) hsv[(unit * 2 + s) * KU + k] = (T)0;
                }
            }
        }
        if constexpr (S == 1) {
            // the partner's diagonal in two alternating copies (stage parity),
            // reals in sublattice-major order; the current one from HBM
            for (int i = t; i < N; i += NTU) {
                const int64_t p = (int64_t)i * N - (int64_t)i * (i - 1) / 2;
                const int q = dpos[i];
                const T v = active ? rho[((int64_t)(1 - spin0) * P + p) * ldr + m].x : (T)0;
                reinterpret_cast<T*>(dpart + (size_t)(g & 1) * kDiagCopy)[q] = v;
                reinterpret_cast<T*>(dpart + (size_t)((g + 1) & 1) * kDiagCopy)[q] = (T)0;
                if constexpr (GINT) {
                    dsite((int)(g & 1))[i] = v + (T)0.5;
                    dsite((int)((g + 1) & 1))[i] = (T)0;
                }
            }
            if constexpr (GINT) {
                for (int i = N + t; i < umat_rows(N); i += NTU) {
                    dsite(0)[i] = (T)0;
                    dsite(1)[i] = (T)0;
                }
            }
        }
        // records: the first N even elements are the diagonal (i = position)
        // (every configuration has N <= NTU, so only slot 0 can hold them)
        auto record = [&](int64_t r) {
            if (active && t < N) {
#pragma unroll
                for (int s = 0; s < S; ++s)
                    Xrec[(r * 2 * N + (int64_t)(spin0 + s) * N + t) * Mc + m] = (double)y[s][0].x;
            }
            if (inv_parts) {
                // per-trajectory sums for the invariant checks, in FP64:
                // hop = sum_i sum_{k in nb(i)} Re rho_ik (each bond twice),
                // frob = sum_ij |rho_ij|^2 (off-diagonal elements twice)
                double hop[S], frob[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    hop[s] = 0.0;
                    frob[s] = 0.0;
#pragma unroll
                    for (int u = 0; u < UE + UO; ++u) {
                        const int e = u < UE ? t + NTU * u : kEvenPad + t + NTU * (u - UE);
                        const uint32_t own = own_of(e);
                        const double re = (double)y[s][u].x, im = (double)y[s][u].y;
                        const bool diag = u < UE && e < N;
                        frob[s] += diag ? re * re : 2.0 * (re * re + im * im);
                        if (own < (uint32_t)P * CB) {  // bond: j a neighbour of i
                            const uint32_t ij = ord[own / CB];
                            const int i = (int)(ij & 0xffffu), j = (int)(ij >> 16);
                            bool bond = false;
                            for (int n = 0; n < 3; ++n) bond = bond || nbt[i * 4 + n] == j;
                            if (bond) hop[s] += 2.0 * re;
                        }
                    }
                    for (int off = 32; off > 0; off /= 2) {
                        hop[s] += __shfl_xor(hop[s], off, 64);
                        frob[s] += __shfl_xor(frob[s], off, 64);
                    }
                }
                if (lane == 0)
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        red[wave][2 * s] = hop[s];
                        red[wave][2 * s + 1] = frob[s];
                    }
                __syncthreads();
                if (t == 0 && active) {
                    constexpr int kWavesPerUnit = NTU / 64;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        double h = 0.0, f = 0.0;
                        for (int w = 0; w < kWavesPerUnit; ++w) {
                            h += red[unit * kWavesPerUnit + w][2 * s];
                            f += red[unit * kWavesPerUnit + w][2 * s + 1];
                        }
                        const int64_t base = ((r * 2 + spin0 + s) * 2) * Mc + m;
                        inv_parts[base] = h;
                        inv_parts[base + Mc] = f;
                    }
                }
            }
        };
        record(0);
        __syncthreads();

        const T tw = uniform_real<T>((T)E.t), Uw = uniform_real<T>((T)E.U);
        const T c_half = uniform_real<T>((T)(0.5 * A.dt));
        const T c_full = uniform_real<T>((T)A.dt);
        const T c_sixth = uniform_real<T>((T)(A.dt / 6.0));
        int64_t cur_step = 0;  // index of the step being taken (the envelope's sample 2 cur_step)

        // One Runge-Kutta stage (STAGE = 1..4) of every element of the unit.
        // Returns false when a spin-split wait timed out.
        auto run_stage = [&](auto stage_tag) -> bool {
            constexpr int STAGE = decltype(stage_tag)::value;
            const T c = STAGE <= 2 ? c_half : (STAGE == 3 ? c_full : c_sixth);
            // S = 1: the partner's diagonal of this stage's input (the copy
            // of the stage counter's parity, which is that of STAGE - 1: every
            // step advances the counter by four)
            const unsigned char* dcur = dpart + ((STAGE - 1) & 1) * kDiagCopy;
            // envelope at this stage's time: t_n, t_n + h/2 (twice), t_n + h
            T Aw = 0;
            if constexpr (POT) {
                if (pot_on)
                    Aw = uniform_real<T>((T)venv[2 * cur_step + (STAGE == 1 ? 0 : STAGE == 4 ? 2 : 1)]);
            }
            // the ratio table of this stage's time (the same half-step samples)
            // (spin split: the first kHopLds places in LDS; shared blocks: the
            // whole table, in site order)
            const int n_lds = S == 2 ? N : (N < kHopLds ? N : kHopLds);
            const HopTab Wt{
                HOP ? hop_tab + (size_t)(2 * cur_step + (STAGE == 1 ? 0 : STAGE == 4 ? 2 : 1)) *
                                    (size_t)N * 3 * CB
                    : nullptr,
                N * 3 * CB, S == 2 ? xarea : lds_ptr(2 * kDiagCopy),
                (uint32_t)n_lds * (S == 2 ? CB : TB), S == 2 ? 3u : 6u};
            if constexpr (HOP) {
                // a new table at stages 2 and 4 (stage 1 reuses the previous
                // step's stage-4 table, except at an item's first step); the
                // previous stage ended with a barrier, so no thread still reads
                // the old copy
                if (STAGE == 2 || STAGE == 4 || cur_step == 0) {
                    const T* src = reinterpret_cast<const T*>(Wt.p);
                    for (int k = tid; k < 6 * n_lds; k += NTU * UNITS)
                        reinterpret_cast<T*>(const_cast<unsigned char*>(Wt.lds))[k] = src[k];
                    __syncthreads();
                }
            }
            // general interaction: D of this stage's input (the partner's
            // diagonal in dcur is complete: the previous stage ended with a
            // barrier after it landed), then the elements take D in place of
            // the diagonal and 1 in place of U
            const unsigned char* Ud = dcur;
            T Uu = Uw;
            if constexpr (GINT && S == 1) {
                if (tid < N) {
                    // u blocked by four along k ([k/4][i][4], zero rows up to a
                    // multiple of 32): one 16-byte buffer load per lane carries
                    // four terms of the chain and a wave reads one contiguous
                    // segment; four such loads are in flight per batch of 16
                    // terms (eight spill registers of the held state at 13 + 13
                    // slots and ran 4 % slower).  h_k = d_k + 1/2 comes from the
                    // site-ordered copy (one wave-uniform 16-byte LDS read per
                    // four terms).  The padded terms are fma(0, 0, D) = D + 0 = D
                    // exactly (D never holds -0: it starts at +0 and a
                    // round-to-nearest sum is -0 only when both addends are).
                    constexpr int B = 4;
                    const int K = umat_rows(N);
                    const T* const hs = dsite((STAGE - 1) & 1);
                    const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)utab, (short)0, (int)(K * N * TB), 0x00020000);
                    T accD = 0;
                    for (int k0 = 0; k0 < K; k0 += 4 * B) {
                        float4 ub[B];
#pragma unroll
                        for (int b = 0; b < B; ++b)
                            ub[b] = __builtin_bit_cast(
                                float4, __builtin_amdgcn_raw_buffer_load_b128(
                                            urs, (uint32_t)(tid * 16), (k0 / 4 + b) * N * 16, 0));
#pragma unroll
                        for (int b = 0; b < B; ++b) {
                            const float4 h = *reinterpret_cast<const float4*>(hs + k0 + 4 * b);
                            accD = fma_rn<T>(ub[b].x, h.x, accD);
                            accD = fma_rn<T>(ub[b].y, h.y, accD);
                            accD = fma_rn<T>(ub[b].z, h.z, accD);
                            accD = fma_rn<T>(ub[b].w, h.w, accD);
                        }
                    }
                    reinterpret_cast<T*>(vpart)[qdiag] = accD;
                }
                __syncthreads();
                Ud = vpart;
                Uu = (T)1;
            }
            if constexpr (GINT && S == 2) {
                // shared blocks: D of both spins of this unit's trajectory,
                // one ascending chain per (spin, site) on threads t < 2N, from
                // the partner block's diagonal (slot k holds rho_kk) and u
                // blocked by four along k (terms k >= N skipped: those slots
                // hold other elements)
                for (int cs = t; cs < 2 * N; cs += NTU) {
                    const int s = cs >= N ? 1 : 0;
                    const int i = cs - s * N;
                    const unsigned char* const dsrc = Yunit + (1 - s) * Pb * CB;
                    T accD = 0;
                    if (u_lds) {
                        // u and h from their LDS copies, four terms per 16
                        // (FP32) or 32 (FP64) bytes (u: a wave's lanes on
                        // consecutive sites; h: the same address on every
                        // lane), in batches of 16 terms whose reads are all
                        // issued before the chain uses them; up to N rounded
                        // up to 16 (<= KU) the terms k >= N are fma(0, 0, D) =
                        // D + 0 (exact: the chain starts at +0 and never holds
                        // -0)
                        const unsigned char* const ui = uarea + (size_t)i * 4 * TB;
                        const T* const hp = hsv + (unit * 2 + (1 - s)) * KU;
                        for (int k0 = 0; k0 < N; k0 += 16) {
                            T ub[16], hb[16];
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                quad_lds<T>(ui + (size_t)(k0 / 4 + b) * N * 4 * TB, ub + 4 * b);
                                quad_lds<T>(reinterpret_cast<const unsigned char*>(hp + k0 + 4 * b),
                                            hb + 4 * b);
                            }
#pragma unroll
                            for (int q = 0; q < 16; ++q) accD = fma_rn<T>(ub[q], hb[q], accD);
                        }
                        *reinterpret_cast<T*>(xarea + ((unit * 2 + s) * N + i) * CB) = accD;
                        continue;
                    }
                    const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)utab, (short)0, (int)(umat_rows(N) * N * TB), 0x00020000);
#pragma unroll 2
                    for (int k0 = 0; k0 < N; k0 += 4) {
                        T ub[4];
                        if constexpr (TB == 4) {
                            const float4 v = __builtin_bit_cast(
                                float4, __builtin_amdgcn_raw_buffer_load_b128(
                                            urs, (uint32_t)(i * 16), (k0 / 4) * N * 16, 0));
                            ub[0] = v.x; ub[1] = v.y; ub[2] = v.z; ub[3] = v.w;
                        } else {
                            const double2 v0 = __builtin_bit_cast(
                                double2, __builtin_amdgcn_raw_buffer_load_b128(
                                             urs, (uint32_t)(i * 32), (k0 / 4) * N * 32, 0));
                            const double2 v1 = __builtin_bit_cast(
                                double2, __builtin_amdgcn_raw_buffer_load_b128(
                                             urs, (uint32_t)(i * 32 + 16), (k0 / 4) * N * 32, 0));
                            ub[0] = v0.x; ub[1] = v0.y; ub[2] = v1.x; ub[3] = v1.y;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (k0 + q < N)
                                accD = fma_rn<T>(ub[q],
                                                 *reinterpret_cast<const T*>(dsrc + (k0 + q) * CB) +
                                                     (T)0.5,
                                                 accD);
                    }
                    *reinterpret_cast<T*>(xarea + ((unit * 2 + s) * N + i) * CB) = accD;
                }
                __syncthreads();
            }
            desc = launder(desc);  // descriptors are re-read every phase
            // ---------------- phase 1: even elements (next values held in
            // registers); descriptors are loaded KP slots ahead.
            // S = 1: the held values of the previous stage are written to LDS
            // here (nothing reads an even element in phase 1: its own value
            // comes from the register, the diagonal of the U term from the
            // partner's copy), which saves a barrier per stage.
            const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)desc, (short)0, (int)((kEvenPad + NTU * UO) * sizeof(DT)), 0x00020000);
            // descriptors in flight: two for the spin split (the L2 latency
            // exceeds one element's time), one where registers are scarcer
            constexpr int KP = S == 1 && NTU * UNITS <= 768 ? 2 : 1;
            auto entry_of = [](int v) { return v < UE ? NTU * v : kEvenPad + NTU * (v - UE); };
            DT dq[KP];
#pragma unroll
            for (int v = 0; v < KP; ++v) dq[v] = slot_desc_buf<DT>(drs, entry_of(v < UE + UO ? v : UE + UO - 1), toff);
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                const DT d = dq[u % KP];
                if (u + KP < UE + UO) dq[u % KP] = slot_desc_buf<DT>(drs, entry_of(u + KP), toff);
                // shared blocks with complex hopping: the element's ratios,
                // the same for both spins, read once
                C wsh[HOP && S == 2 ? 6 : 1];
                if constexpr (HOP && S == 2) ratios_lds<T>(Wt, own_di(d), own_dj(d), wsh);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    unsigned char* Yb = Yunit + s * Pb * CB;
                    C k;
                    if constexpr (S == 1) {
                        // the stage input of this element: after a full step it
                        // is y itself, so nothing is held across steps
                        const C own = STAGE == 1 ? y[s][u] : hold[s][u];
                        *reinterpret_cast<C*>(Yb + own_off(d)) = own;
                        k = element_rhs_sel<T, true, T1, DT, POT, HOP>(u < GE, Yb, Ud, d, tw,
                                                                       Uu, own, vpart, Aw, pot_on,
                                                                       Wt);
                    } else {
                        // the U term from the partner block's diagonal, or
                        // (GINT) from this unit's D of spin s with U = 1
                        const unsigned char* Yd2 =
                            GINT ? xarea + (size_t)(unit * 2 + s) * N * CB
                                 : Yunit + (1 - s) * Pb * CB;
                        k = element_rhs_sel<T, false, T1, DT, POT, HOP, HOP>(
                            u < GE, Yb, Yd2, d, tw, GINT ? (T)1 : Uw, hold[s][u], vpart, Aw,
                            pot_on, Wt, wsh);
                    }
                    hold[s][u] = rk_update<STAGE, T>(c, k, y[s][u], acc[s][u]);
                    pin(hold[s][u]);
                    pin(acc[s][u]);
                    if constexpr (STAGE == 4) pin(y[s][u]);
                }
                if constexpr (S == 1) {
                    if (u == 0 && t < N) {
                        // publish the next-stage diagonal for the partner: one
                        // 64-bit word per site, (stage number << 32) | value bits,
                        // a single relaxed agent-scope atomic store
                        uint64_t* slot =
                            mb + ((size_t)(pair * 2 + spin0) * 2 + ((g + 1) & 1)) * A.Nmax;
                        const uint64_t word = ((uint64_t)(g + 1) << 32) | to_bits<T>(hold[0][0].x);
                        __hip_atomic_store(slot + t, word, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                // one element per scheduling region: the scheduler may not pull
                // later slots' loads forward (their registers would not fit)
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            // ---------------- phase 2: odd elements (written straight to LDS)
#pragma unroll
            for (int u = UE; u < UE + UO; ++u) {
                const DT d = dq[u % KP];
                if (u + KP < UE + UO) dq[u % KP] = slot_desc_buf<DT>(drs, entry_of(u + KP), toff);
                C wsh[HOP && S == 2 ? 6 : 1];
                if constexpr (HOP && S == 2) ratios_lds<T>(Wt, own_di(d), own_dj(d), wsh);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    unsigned char* Yb = Yunit + s * Pb * CB;
                    const unsigned char* Yd =
                        S == 1 ? Ud
                               : (GINT ? xarea + (size_t)(unit * 2 + s) * N * CB
                                       : Yunit + (1 - s) * Pb * CB);
                    const T Us = S == 1 ? Uu : (GINT ? (T)1 : Uw);
                    // stage 1 reads the element's own value from y (the
                    // stage input of a full step is its base point)
                    constexpr bool WP = HOP && S == 2;
                    const C k = STAGE == 1
                        ? element_rhs_sel<T, true, T1, DT, POT, HOP, WP>(u - UE < GO, Yb, Yd, d,
                                                                          tw, Us, y[s][u], vpart,
                                                                          Aw, pot_on, Wt, wsh)
                        : element_rhs_sel<T, false, T1, DT, POT, HOP, WP>(u - UE < GO, Yb, Yd, d,
                                                                           tw, Us, y[s][u], vpart,
                                                                           Aw, pot_on, Wt, wsh);
                    *reinterpret_cast<C*>(Yb + own_off(d)) = rk_update<STAGE, T>(c, k, y[s][u], acc[s][u]);
                    pin(acc[s][u]);
                    if constexpr (STAGE == 4) pin(y[s][u]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (S == 1) {
                // the partner's diagonal of the next stage into the other copy
                // (not read in this stage): thread i < N polls word i until it
                // carries stage g+1 (bounded; the two mailbox slots alternate
                // by parity, so a word is never overwritten before it is read)
                if (tid < N) {
                    const int q = qdiag;
                    const uint64_t* slot =
                        mb + ((size_t)(pair * 2 + (1 - spin0)) * 2 + ((g + 1) & 1)) * A.Nmax;
                    const uint32_t want = (uint32_t)(g + 1);
                    uint64_t w = __hip_atomic_load(slot + tid, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    unsigned it = 0;
                    while ((uint32_t)(w >> 32) != want) {
                        if (++it >= A.spin_limit) {
                            abort_flag = 1;
                            atomicExch(A.error, 1);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        w = __hip_atomic_load(slot + tid, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    }
                    reinterpret_cast<T*>(dpart + (STAGE & 1) * kDiagCopy)[q] =
                        from_bits<T>((uint32_t)w);
                    if constexpr (GINT) dsite(STAGE & 1)[tid] = from_bits<T>((uint32_t)w) + (T)0.5;
                }
            } else {
                __syncthreads();
                desc = launder(desc);
                // ---------------- held even values (slot t + NTU*u; padding
                // entries write the scratch slot)
#pragma unroll
                for (int u = 0; u < UE; ++u) {
                    const uint32_t own = slot_desc(desc, NTU * u, toff).a.w;
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        *reinterpret_cast<C*>(Yunit + s * Pb * CB + own) = hold[s][u];
                }
                if constexpr (GINT) {
                    // the next stage input's h (read after the barrier)
                    if (u_lds && t < N) {
#pragma unroll
                        for (int s = 0; s < S; ++s)
                            hsv[(unit * 2 + s) * KU + t] = hold[s][0].x + (T)0.5;
                    }
                }
            }
            __syncthreads();
            ++g;
            if constexpr (S == 1) return abort_flag == 0;
            return true;
        };

        // the state y of every element to `out` (same layout as rho; stored
        // elements are conjugated back to the upper triangle).  Addresses are
        // recomputed, not kept alive across the time loop.
        auto store_state = [&](C* out) {
            const gdesc_t dl = launder(desc);  // a local copy: desc itself stays uniform
            out = reinterpret_cast<C*>(uniform64((uint64_t)out));
            if (!active) return;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int gs = spin0 + s;
#pragma unroll
                for (int u = 0; u < UE + UO; ++u) {
                    const int e = u < UE ? t + NTU * u : kEvenPad + t + NTU * (u - UE);
                    const uint32_t own = own_at(dl, e);
                    if (own < (uint32_t)P * CB) {
                        bool tr;
                        const int64_t p = packed_of(own, tr);
                        C v = y[s][u];
                        if (tr) v.y = -v.y;
                        out[((int64_t)gs * P + p) * ldr + m] = v;
                    }
                }
            }
        };

        for (int64_t step = 1; step <= A.n_steps; ++step) {
            cur_step = step - 1;
            if (!run_stage(stage_c<1>{})) return;
            if (!run_stage(stage_c<2>{})) return;
            if (!run_stage(stage_c<3>{})) return;
            if (!run_stage(stage_c<4>{})) return;
            if (step % A.record_every == 0) {
                const int64_t r = step / A.record_every;
                record(r);
                // optional stored state at every record (the adjoint's
                // checkpoints and segment states; general kernels only, so
                // that the unit-hopping variant's time loop carries no such
                // code)
                if constexpr (!T1) {
                    C* const dump = reinterpret_cast<C*>(uniform64((uint64_t)E.dump));
                    if (dump) store_state(dump + (r - 1) * E.dump_stride);
                }
            }
        }

        // ---- final state back to HBM
        store_state(rho);
    }
}

// ---------------------------------------------------------------- split kernel
// A spin block too large for one CU (the 198-site block in FP64: 315 KB)
// spread over G workgroups ("parts") placed on one XCD: part p owns the stored
// elements of a strip of rows (sites in rank order, strips of nearly equal
// element count) and keeps, besides its own elements, the "halo" its stencils
// read from the neighbouring strips in LDS.  Every stage each part publishes
// the next values of its exported elements (those another part reads, and
// the diagonal, which the other spin's parts read for the U term) into a
// per-part area of global memory, and copies in its halo and the partner
// spin's diagonal.  Every published 32-bit word travels with the number of
// the stage it belongs to in one 64-bit relaxed agent-scope atomic (two
// areas alternating by stage parity), so no fences are needed; a word is
// never overwritten before it is read because the stencil relation is
// symmetric (a part that reads a neighbour's element is read back by it in
// the other class) and the diagonal exchange is all-to-all, so no member of
// a group runs two stages ahead of a reader.  Waits are bounded.
//
// The two-phase stage stays, with the waits placed where their data has had
// the most time to arrive: the even elements of a part are ordered interior
// (they read no other part's element) before boundary (the diagonal and the
// exported ones).  The reads of both halos of a stage's input are issued at
// the start of the stage; the odd halo (published early in the producers'
// previous phase 2: exported odd elements come first) is needed only from the
// boundary slots on, after a barrier; the even halo (published in the
// producers' previous phase 1) before phase 2; the partner's diagonal of the
// next stage's input is read during phase 2.

// Sub-dword-select shifts with the shift as a template argument.
template <int SH> __device__ __forceinline__ uint32_t lo16_shl(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:WORD_0" : "=v"(r) : "v"(w), "i"(SH));
    return r;
}
template <int SH> __device__ __forceinline__ uint32_t hi16_shl(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:WORD_1" : "=v"(r) : "v"(w), "i"(SH));
    return r;
}
template <int SH> __device__ __forceinline__ uint32_t b2_shl(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:BYTE_2" : "=v"(r) : "v"(w), "i"(SH));
    return r;
}
template <int SH> __device__ __forceinline__ uint32_t b3_shl(uint32_t w) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD "
            "src1_sel:BYTE_3" : "=v"(r) : "v"(w), "i"(SH));
    return r;
}

// Compact descriptor of the split kernel: slot numbers x 2^SH bytes, diagonal
// positions x 2^DSH bytes; xp (constant once the slot loop is unrolled): the
// own field may carry the export flag (bit 15).
template <int SH, int DSH, bool GEN>
__device__ __forceinline__ Stencil decode_split(const uint4& w, bool xp) {
    Stencil e;
    const uint32_t f[3] = {w.x, w.y, w.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if constexpr (GEN) {
            e.n[2 * k] = ((f[k] & 0x7fffu) << SH) | ((f[k] & 0x8000u) << 16);
            e.n[2 * k + 1] = (((f[k] >> 16) & 0x7fffu) << SH) | (f[k] & 0x80000000u);
        } else {
            e.n[2 * k] = lo16_shl<SH>(f[k]);
            e.n[2 * k + 1] = hi16_shl<SH>(f[k]);
        }
    }
    e.own = xp ? (w.w & 0x7fffu) << SH : lo16_shl<SH>(w.w);
    e.di = b2_shl<DSH>(w.w);
    e.dj = b3_shl<DSH>(w.w);
    return e;
}

template <typename T, bool OWN_REG, bool T1, int SH, int DSH, bool POT = false, bool HOP = false>
__device__ __forceinline__ cplx_t<T> element_rhs_split(bool gen, bool xp, const unsigned char* Yb,
                                                       const unsigned char* Yd, const uint4& d,
                                                       T t, T U, cplx_t<T> own,
                                                       const unsigned char* Vd = nullptr,
                                                       T Aw = 0, bool pot_on = false,
                                                       HopTab Wt = {}) {
    return gen ? element_rhs<T, OWN_REG, true, T1, POT, HOP>(Yb, Yd, decode_split<SH, DSH, true>(d, xp),
                                                             t, U, own, Vd, Aw, pot_on, Wt)
               : element_rhs<T, OWN_REG, false, T1, POT, HOP>(Yb, Yd,
                                                              decode_split<SH, DSH, false>(d, xp),
                                                              t, U, own, Vd, Aw, pot_on, Wt);
}

// A complex value as 32-bit payload words and back.
template <typename T> struct Payload {
    static constexpr int W = (int)sizeof(cplx_t<T>) / 4;
    uint32_t w[W];
};
template <typename T> __device__ __forceinline__ Payload<T> to_payload(cplx_t<T> v) {
    return __builtin_bit_cast(Payload<T>, v);
}
template <typename T> __device__ __forceinline__ cplx_t<T> from_payload(const Payload<T>& p) {
    return __builtin_bit_cast(cplx_t<T>, p);
}

// Publishes a value: every payload word with the stage number in the high
// half, each a relaxed agent-scope atomic (a reader sees the old or the new
// stage of a word, never a mixture); word k at dst + k * stride (word-major
// areas: the threads of a wave write consecutive words).
template <typename T>
__device__ __forceinline__ void publish(uint64_t* dst, int stride, cplx_t<T> v, uint32_t stamp) {
    const Payload<T> p = to_payload<T>(v);
#pragma unroll
    for (int k = 0; k < Payload<T>::W; ++k)
        __hip_atomic_store(dst + (size_t)k * stride, ((uint64_t)stamp << 32) | p.w[k],
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t peek(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr unsigned kSplitSpinLimit = 1u << 22;  // default: ~3.5 s at the longer sleeps below

// Waits until NW published words carry stage `want`: w[k] was read from
// src[k / WPE] + (k % WPE) * stride (WPE = NW / NP, null pointers are
// skipped); while any word is stale, all of them are read again (one round
// trip per retry).
// Bounded: false (abort flag and error word set) when the stage never comes
// or another wait of the workgroup gave up.
template <int NW, int NP>
__device__ __forceinline__ bool settle_words(const uint64_t* const* src, int stride, uint64_t* w,
                                             uint32_t want, int& abort_flag, int* error,
                                             unsigned limit) {
    constexpr int WPE = NW / NP;
    unsigned it = 0;
    while (true) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < NW; ++k)
            ok = ok && (src[k / WPE] == nullptr || (uint32_t)(w[k] >> 32) == want);
        if (ok) return true;
        if (*reinterpret_cast<volatile int*>(&abort_flag)) return false;
        if (++it >= limit) {
            abort_flag = 1;
            atomicExch(error, 1);
            return false;
        }
        // ~2000 cycles: polling less often leaves the memory system to the
        // producers (a shorter sleep is slower overall)
        __builtin_amdgcn_s_sleep(32);
#pragma unroll
        for (int k = 0; k < NW; ++k)
            if (src[k / WPE]) w[k] = peek(src[k / WPE] + (size_t)(k % WPE) * stride);
    }
}

// T1: every instance of the launch has t = 1.  Even slots: interior elements
// in u < UB (the first GE1 slots read transposes), boundary elements from UB
// (the diagonal first; slots UB .. UB + GE2 - 1 read transposes); odd slots:
// the first GO read transposes, exported elements in the first XO.  KB: halo
// entries per thread whose reads are issued a phase ahead.  POT: entries may
// carry an external potential (its profile after the two diagonal copies, in
// their layout; the element slots follow it).  GINT: every entry carries a
// general interaction u_ij (ResidentInst::umat, as the spin-split kernels
// read it): every part forms D_i = sum_k u_ki (d_k + 1/2) for all sites at
// the start of each stage from the partner's whole diagonal (which every
// part receives), into LDS after the diagonal copies, and the U factor of an
// element is D_i - D_j (U = 1 exactly).  HOP: every entry carries complex
// hopping (ResidentInst::hop, as the spin-split kernels read it); each stage
// keeps the whole ratio table of its time in LDS after the diagonal copies.
template <typename T, int G, int NTU, int UE, int UO, int UB, int GE1, int GE2, int GO, int XO,
          int KB, bool T1, bool POT = false, bool GINT = false, bool HOP = false>
__global__ __launch_bounds__(NTU) void rk4_split(ResidentArgs A) {
    using C = cplx_t<T>;
    constexpr int CB = (int)sizeof(C);
    constexpr int TB = (int)sizeof(T);
    constexpr int SH = CB == 8 ? 3 : 4;   // slot number -> byte offset
    constexpr int DSH = TB == 4 ? 2 : 3;  // diagonal position -> byte offset
    constexpr int W = Payload<T>::W;      // published words per element
    constexpr int DW = TB / 4;            // words of the real part
    constexpr int kEnt = NTU * (UE + UO); // descriptor entries of a part
    constexpr int kEvenPad = NTU * UE;
    constexpr uint32_t kDiagCopy = 256 * TB;
    static_assert(GE1 <= UB && UB < UE && UB + GE2 <= UE && GO <= UO && XO <= UO,
                  "slot groups within their class");
    static_assert((POT ? 1 : 0) + (GINT ? 1 : 0) + (HOP ? 1 : 0) <= 1,
                  "one of a potential, a general interaction and complex hopping");
    extern __shared__ __align__(16) unsigned char smem[];
    (void)smem;
    const int tid0 = threadIdx.x;

    // groups of 2G workgroups on one XCD (blocks b = xcd + 8 k; members k =
    // 2G c .. 2G c + 2G - 1): spin = member / G, part = member % G; the
    // groups take items (trajectories) in the same order
    const int b = blockIdx.x, xcd = b % 8, k = b / 8;
    const int member = k % (2 * G);
    const int spin0 = member / G, part = member % G;
    const int group = (k / (2 * G)) * 8 + xcd;
    const int64_t n_groups = gridDim.x / (2 * G);
    if (tid0 == 0) *reinterpret_cast<int*>(lds_ptr(A.tail_off + (NTU / 64) * 2 * 8)) = 0;
    // published words of this group: [2 spins][G parts][2 parities][W][kEnt]
    uint64_t* const xg = A.mailbox + (size_t)group * 2 * G * 2 * kEnt * W;
    auto xslot = [&](int spin, int q, uint32_t stamp) {
        return xg + ((size_t)(spin * G + q) * 2 + (stamp & 1)) * kEnt * W;
    };
    int64_t g = 0;  // stage counter (continues across items)

    C y[UE + UO], acc[UE + UO], hold[UE];

    for (int64_t item = group; item < A.n_items; item += n_groups) {
        const int t = tid0;
        const uint32_t toff = (uint32_t)t * 16u;
        int ent = 0;
        while (ent + 1 < A.n_entries && A.table[ent + 1].item0 <= item) ++ent;
        ent = __builtin_amdgcn_readfirstlane(ent);
        const ResidentInst& E = A.table[ent];
        const int N = E.N;
        const int P = E.P;
        const int pw = __builtin_amdgcn_readfirstlane(E.part_words);
        const int hmax = __builtin_amdgcn_readfirstlane(E.hmax);
        const uint32_t* const blob = reinterpret_cast<const uint32_t*>(uniform64((uint64_t)E.desc));
        const uint32_t* const pb = blob + (size_t)part * pw;
        const int n_own = __builtin_amdgcn_readfirstlane((int)pb[1]);
        const int n_ie = __builtin_amdgcn_readfirstlane((int)pb[2]);
        const int n_io = __builtin_amdgcn_readfirstlane((int)pb[3]);
        const int n_diag = __builtin_amdgcn_readfirstlane((int)pb[4]);
        gdesc_t desc = (gdesc_t)uniform64((uint64_t)(pb + 8));
        const uint32_t* const pord = pb + 8 + 4 * kEnt;
        const uint32_t* const imp = pord + kEnt;
        const uint32_t* const dsite = imp + hmax;
        const uint32_t* const dsrc = blob + (size_t)G * pw;
        // LDS: two copies of the partner's diagonal (sublattice-major), then
        // the potential's profile (POT) or D and two site-ordered copies of
        // h_k = d_k + 1/2, zero from N up to the u table's row count (GINT),
        // then the part's elements; HOP: the stage's ratio table (256 places)
        // in place of those
        unsigned char* const Yb =
            lds_ptr(HOP ? 2 * kDiagCopy + 256 * 6 * TB : (GINT ? 5 : POT ? 3 : 2) * kDiagCopy);
        unsigned char* const dpart = lds_ptr(0);
        auto hsite = [&](int c) { return reinterpret_cast<T*>(lds_ptr((3 + c) * kDiagCopy)); };
        int& abort_flag = *reinterpret_cast<int*>(lds_ptr(A.tail_off + (NTU / 64) * 2 * 8));
        const int64_t Mc = E.Mc;
        const int64_t m = item - E.item0;
        const bool active = m < Mc;
        C* const rho = reinterpret_cast<C*>(uniform64((uint64_t)E.rho));
        const int64_t ldr = E.ldr;
        double* const Xrec = E.X;
        auto own_slot_at = [&](gdesc_t dt, int e) -> uint32_t {
            return reinterpret_cast<const uint4*>((uint64_t)dt)[e].w & 0x7fffu;
        };
        // packed index of stored element a | b << 16 (conjugated when b < a)
        auto packed_ab = [&](uint32_t ab, bool& transposed) -> int64_t {
            const int a = (int)(ab & 0xffffu), bb = (int)(ab >> 16);
            const int i = a < bb ? a : bb, j = a < bb ? bb : a;
            transposed = a > bb;
            return (int64_t)i * N - (int64_t)i * (i - 1) / 2 + (j - i);
        };
        auto load_elem = [&](uint32_t ab) -> C {
            C v;
            v.x = 0;
            v.y = 0;
            if (active) {
                bool tr;
                const int64_t p = packed_ab(ab, tr);
                v = rho[((int64_t)spin0 * P + p) * ldr + m];
                if (tr) v.y = -v.y;
            }
            return v;
        };
        __syncthreads();  // the previous item is done with LDS

        // ---- the trajectory's own elements, the halo, the zero and scratch
        // slots, and the partner's diagonal
#pragma unroll
        for (int u = 0; u < UE + UO; ++u) {
            const int e = u < UE ? t + NTU * u : kEvenPad + t + NTU * (u - UE);
            const uint32_t own = own_slot_at(desc, e);
            C v;
            v.x = 0;
            v.y = 0;
            if (own < (uint32_t)n_own) v = load_elem(pord[own]);
            reinterpret_cast<C*>(Yb)[own] = v;
            y[u] = v;
            acc[u] = v;
            if (u < UE) hold[u] = v;
        }
        for (int h = t; h < n_ie + n_io; h += NTU) {
            const uint32_t qs = imp[h];
            const uint32_t* const pq = blob + (size_t)(qs >> 16) * pw + 8 + 4 * kEnt;
            reinterpret_cast<C*>(Yb)[n_own + h] = load_elem(pq[qs & 0xffffu]);
        }
        if (t < 33) {
            C z;
            z.x = 0;
            z.y = 0;
            reinterpret_cast<C*>(Yb)[n_own + n_ie + n_io + t] = z;
        }
        const int32_t* const dpos = reinterpret_cast<const int32_t*>(uniform64((uint64_t)E.dpos));
        for (int i = t; i < N; i += NTU) {
            const int64_t p = (int64_t)i * N - (int64_t)i * (i - 1) / 2;
            const int q = dpos[i];
            reinterpret_cast<T*>(dpart + (size_t)(g & 1) * kDiagCopy)[q] =
                active ? rho[((int64_t)(1 - spin0) * P + p) * ldr + m].x : (T)0;
            reinterpret_cast<T*>(dpart + (size_t)((g + 1) & 1) * kDiagCopy)[q] = (T)0;
            if constexpr (GINT) {
                hsite((int)(g & 1))[i] =
                    (active ? rho[((int64_t)(1 - spin0) * P + p) * ldr + m].x : (T)0) + (T)0.5;
                hsite((int)((g + 1) & 1))[i] = (T)0;
            }
        }
        if constexpr (GINT) {
            for (int i = N + t; i < umat_rows(N); i += NTU) {
                hsite(0)[i] = (T)0;
                hsite(1)[i] = (T)0;
            }
        }
        // general interaction: u in T, blocked by four along k
        const T* const utab = GINT ? reinterpret_cast<const T*>(uniform64((uint64_t)E.umat)) : nullptr;
        // complex hopping: the prepared ratio tables, [2 n_steps + 1][N][3]
        const unsigned char* const hop_tab =
            HOP ? reinterpret_cast<const unsigned char*>(uniform64((uint64_t)E.hop)) : nullptr;
        // external potential of this entry: the profile v (zero without one)
        // and the envelope, read per stage
        const double* const venv = POT ? reinterpret_cast<const double*>(uniform64((uint64_t)E.v_env))
                                       : nullptr;
        const bool pot_on = POT && E.v_site != nullptr;
        unsigned char* const vpart = lds_ptr(2 * kDiagCopy);
        if constexpr (POT) {
            const double* const vs = reinterpret_cast<const double*>(uniform64((uint64_t)E.v_site));
            for (int i = t; i < N; i += NTU)
                reinterpret_cast<T*>(vpart)[dpos[i]] = pot_on ? (T)vs[i] : (T)0;
        }
        int64_t cur_step = 0;  // index of the step being taken (the envelope's sample 2 cur_step)
        // records: boundary entry t < n_diag (slot UB) is the diagonal element
        // of site dsite[t]
        auto record = [&](int64_t r) {
            if (active && t < n_diag)
                Xrec[(r * 2 * N + (int64_t)spin0 * N + (int64_t)dsite[t]) * Mc + m] = (double)y[UB].x;
        };
        record(0);
        __syncthreads();

        const T tw = uniform_real<T>((T)E.t), Uw = uniform_real<T>((T)E.U);
        const T c_half = uniform_real<T>((T)(0.5 * A.dt));
        const T c_full = uniform_real<T>((T)A.dt);
        const T c_sixth = uniform_real<T>((T)(A.dt / 6.0));
        bool first = true;  // the item's first stage: its halo came from HBM

        // Halo copies: the reads of this thread's first KB entries of [h0, h1)
        // are issued early (issue), the values land in their slots later
        // (land; further entries, if any, are read there).
        struct Batch {
            uint64_t w[KB * W];
            const uint64_t* src[KB];
        };
        auto issue = [&](Batch& bt, int h0, int h1, uint32_t want) {
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                const int h = h0 + t + j * NTU;
                bt.src[j] = nullptr;
                if (h < h1) {
                    const uint32_t qs = imp[h];
                    bt.src[j] = xslot(spin0, (int)(qs >> 16), want) + (qs & 0xffffu);
#pragma unroll
                    for (int kk = 0; kk < W; ++kk) bt.w[j * W + kk] = peek(bt.src[j] + (size_t)kk * kEnt);
                }
            }
        };
        auto land = [&](Batch& bt, int h0, int h1, uint32_t want) {
            for (int hb = h0;; ) {
                if (!settle_words<KB * W, KB>(bt.src, kEnt, bt.w, want, abort_flag, A.error,
                                              A.spin_limit))
                    return;
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    if (bt.src[j]) {
                        Payload<T> pl;
#pragma unroll
                        for (int kk = 0; kk < W; ++kk) pl.w[kk] = (uint32_t)bt.w[j * W + kk];
                        reinterpret_cast<C*>(Yb)[n_own + hb + t + j * NTU] = from_payload<T>(pl);
                    }
                }
                hb += KB * NTU;
                if (hb >= h1) return;
                issue(bt, hb, h1, want);
            }
        };

        auto run_stage = [&](auto stage_tag) -> bool {
            constexpr int STAGE = decltype(stage_tag)::value;
            const T c = STAGE <= 2 ? c_half : (STAGE == 3 ? c_full : c_sixth);
            const unsigned char* dcur = dpart + ((STAGE - 1) & 1) * kDiagCopy;
            // envelope at this stage's time: t_n, t_n + h/2 (twice), t_n + h
            T Aw = 0;
            if constexpr (POT) {
                if (pot_on)
                    Aw = uniform_real<T>((T)venv[2 * cur_step + (STAGE == 1 ? 0 : STAGE == 4 ? 2 : 1)]);
            }
            // general interaction: D of this stage's input from the
            // site-ordered copy (complete: the previous stage ended with a
            // barrier after it landed), one ascending fused chain per site on
            // threads t < N; u blocked by four along k, two 16-byte loads per
            // lane and block (FP64), four blocks in flight; padded terms add
            // exactly +0 (the chain starts at +0 and never holds -0)
            // complex hopping: this stage's ratio table, all of it in LDS
            // (copied when the table changes: stages 2 and 4, and an item's
            // first stage; the previous stage ended with a barrier)
            const HopTab Wt{
                HOP ? hop_tab + (size_t)(2 * cur_step + (STAGE == 1 ? 0 : STAGE == 4 ? 2 : 1)) *
                                    (size_t)N * 3 * CB
                    : nullptr,
                N * 3 * CB, lds_ptr(2 * kDiagCopy), (uint32_t)N * TB};
            if constexpr (HOP) {
                if (STAGE == 2 || STAGE == 4 || cur_step == 0) {
                    const T* src = reinterpret_cast<const T*>(Wt.p);
                    for (int k = t; k < 6 * N; k += NTU)
                        reinterpret_cast<T*>(lds_ptr(2 * kDiagCopy))[k] = src[k];
                    __syncthreads();
                }
            }
            const unsigned char* Ud = dcur;
            T Uu = Uw;
            if constexpr (GINT) {
                if (t < N) {
                    constexpr int B = 4;
                    const int K = umat_rows(N);
                    const T* const hs = hsite((STAGE - 1) & 1);
                    const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)utab, (short)0, (int)(K * N * TB), 0x00020000);
                    T accD = 0;
                    for (int k0 = 0; k0 < K; k0 += 4 * B) {
                        double2 ua[B], ub[B];
#pragma unroll
                        for (int b = 0; b < B; ++b) {
                            const int so = (k0 / 4 + b) * N * 32;
                            ua[b] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(
                                                                    urs, (uint32_t)(t * 32), so, 0));
                            ub[b] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(
                                                                    urs, (uint32_t)(t * 32 + 16), so, 0));
                        }
#pragma unroll
                        for (int b = 0; b < B; ++b) {
                            const double2 h0 = *reinterpret_cast<const double2*>(hs + k0 + 4 * b);
                            const double2 h1 = *reinterpret_cast<const double2*>(hs + k0 + 4 * b + 2);
                            accD = fma_rn<T>(ua[b].x, h0.x, accD);
                            accD = fma_rn<T>(ua[b].y, h0.y, accD);
                            accD = fma_rn<T>(ub[b].x, h1.x, accD);
                            accD = fma_rn<T>(ub[b].y, h1.y, accD);
                        }
                    }
                    reinterpret_cast<T*>(vpart)[dpos[t]] = accD;
                }
                __syncthreads();
                Ud = vpart;
                Uu = (T)1;
            }
            const uint32_t stamp = (uint32_t)(g + 1);
            uint64_t* const mine = xslot(spin0, part, stamp);
            desc = launder(desc);
            const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)desc, (short)0, (int)(kEnt * 16), 0x00020000);
            constexpr int KP = 2;
            auto entry_of = [](int v) { return v < UE ? NTU * v : kEvenPad + NTU * (v - UE); };
            uint4 dq[KP];
#pragma unroll
            for (int v = 0; v < KP; ++v) dq[v] = slot_desc_buf<uint4>(drs, entry_of(v < UE + UO ? v : UE + UO - 1), toff);
            // the halo of this stage's input (published in the producers'
            // previous stage): reads issued now, landed before the elements
            // that need them (the odd halo before the boundary, the even halo
            // before phase 2)
            Batch bo, be;
            if (!first) {
                issue(bo, n_ie, n_ie + n_io, (uint32_t)g);
                issue(be, 0, n_ie, (uint32_t)g);
            }
            // ---------------- phase 1: even elements (next values held)
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                if (u == UB) {
                    // the boundary elements read the odd halo
                    if (!first) land(bo, n_ie, n_ie + n_io, (uint32_t)g);
                    __syncthreads();
                }
                const uint4 d = dq[u % KP];
                if (u + KP < UE + UO) dq[u % KP] = slot_desc_buf<uint4>(drs, entry_of(u + KP), toff);
                const C own = STAGE == 1 ? y[u] : hold[u];
                const bool xp = u >= UB;
                const bool gen = u < GE1 || (u >= UB && u < UB + GE2);
                const uint32_t ob = xp ? (d.w & 0x7fffu) << SH : lo16_shl<SH>(d.w);
                *reinterpret_cast<C*>(Yb + ob) = own;
                const C kk = element_rhs_split<T, true, T1, SH, DSH, POT, HOP>(
                    gen, xp, Yb, Ud, d, tw, Uu, own, vpart, Aw, pot_on, Wt);
                hold[u] = rk_update<STAGE, T>(c, kk, y[u], acc[u]);
                pin(hold[u]);
                pin(acc[u]);
                if constexpr (STAGE == 4) pin(y[u]);
                if (xp && (d.w & 0x8000u))
                    publish<T>(mine + (d.w & 0x7fffu), kEnt, hold[u], stamp);
                __builtin_amdgcn_sched_barrier(0);
            }
            // phase 2 reads the even halo
            if (!first) land(be, 0, n_ie, (uint32_t)g);
            __syncthreads();
            // ---------------- phase 2: odd elements (written straight to LDS);
            // the partner's diagonal of the next stage's input is read
            // meanwhile (into the copy this stage does not read)
            const uint64_t* dsrcp[1] = {nullptr};
            uint64_t dw[DW];
            if (t < N) {
                const uint32_t qs = dsrc[t];
                dsrcp[0] = xslot(1 - spin0, (int)(qs >> 16), stamp) + (qs & 0xffffu);
#pragma unroll
                for (int kk = 0; kk < DW; ++kk) dw[kk] = peek(dsrcp[0] + (size_t)kk * kEnt);
            }
#pragma unroll
            for (int u = UE; u < UE + UO; ++u) {
                const uint4 d = dq[u % KP];
                if (u + KP < UE + UO) dq[u % KP] = slot_desc_buf<uint4>(drs, entry_of(u + KP), toff);
                const bool xp = u - UE < XO;
                const bool gen = u - UE < GO;
                const C kk = STAGE == 1
                    ? element_rhs_split<T, true, T1, SH, DSH, POT, HOP>(gen, xp, Yb, Ud, d, tw, Uu,
                                                                        y[u], vpart, Aw, pot_on, Wt)
                    : element_rhs_split<T, false, T1, SH, DSH, POT, HOP>(gen, xp, Yb, Ud, d, tw, Uu,
                                                                         y[u], vpart, Aw, pot_on, Wt);
                const C nx = rk_update<STAGE, T>(c, kk, y[u], acc[u]);
                const uint32_t ob = xp ? (d.w & 0x7fffu) << SH : lo16_shl<SH>(d.w);
                *reinterpret_cast<C*>(Yb + ob) = nx;
                pin(acc[u]);
                if constexpr (STAGE == 4) pin(y[u]);
                if (xp && (d.w & 0x8000u)) publish<T>(mine + (d.w & 0x7fffu), kEnt, nx, stamp);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (t < N && settle_words<DW, 1>(dsrcp, kEnt, dw, stamp, abort_flag, A.error,
                                             A.spin_limit)) {
                Payload<T> pl;
#pragma unroll
                for (int kk = 0; kk < W; ++kk) pl.w[kk] = kk < DW ? (uint32_t)dw[kk] : 0u;
                reinterpret_cast<T*>(dpart + (STAGE & 1) * kDiagCopy)[dpos[t]] = from_payload<T>(pl).x;
                if constexpr (GINT) hsite(STAGE & 1)[t] = from_payload<T>(pl).x + (T)0.5;
            }
            __syncthreads();
            ++g;
            first = false;
            return abort_flag == 0;
        };

        auto store_state = [&](C* out) {
            const gdesc_t dl = launder(desc);
            out = reinterpret_cast<C*>(uniform64((uint64_t)out));
            if (!active) return;
#pragma unroll
            for (int u = 0; u < UE + UO; ++u) {
                const int e = u < UE ? t + NTU * u : kEvenPad + t + NTU * (u - UE);
                const uint32_t own = own_slot_at(dl, e);
                if (own < (uint32_t)n_own) {
                    bool tr;
                    const int64_t p = packed_ab(pord[own], tr);
                    C v = y[u];
                    if (tr) v.y = -v.y;
                    out[((int64_t)spin0 * P + p) * ldr + m] = v;
                }
            }
        };

        for (int64_t step = 1; step <= A.n_steps; ++step) {
            cur_step = step - 1;
            if (!run_stage(stage_c<1>{})) return;
            if (!run_stage(stage_c<2>{})) return;
            if (!run_stage(stage_c<3>{})) return;
            if (!run_stage(stage_c<4>{})) return;
            if (step % A.record_every == 0) {
                const int64_t r = step / A.record_every;
                record(r);
                if constexpr (!T1) {
                    C* const dump = reinterpret_cast<C*>(uniform64((uint64_t)E.dump));
                    if (dump) store_state(dump + (r - 1) * E.dump_stride);
                }
            }
        }
        store_state(rho);
    }
}

// ---------------------------------------------------------------- configurations
// GE, GO: the leading even and odd slots that take the general path (the
// elements that read a transpose must fit in them).
// fn_t1: the variant for launches whose instances all have t = 1 (FP32).
struct Config {
    ftwa_dtype dtype;
    int S, NTU, UNITS, UE, UO, GE, GO;
    const void* fn;
    const void* fn_t1;
    // split kernel (G > 1 workgroups per spin block): GE = GE1; boundary
    // from slot UB, its first GE2 slots read transposes; exported odd
    // elements in the first XO odd slots; KB halo reads issued ahead
    int G = 1;
    int UB = 0, GE2 = 0, XO = 0, KB = 0;
    bool auto_pick = true;  // false: chosen only when forced or by the autotuner
    // variants (the FP32 spin split and the FP64 split kernel; _t1: the same
    // for launches with t = 1, FP32 only): external potential, complex
    // hopping, general interaction
    const void* fn_pot = nullptr;
    const void* fn_pot_t1 = nullptr;
    const void* fn_hop = nullptr;
    const void* fn_hop_t1 = nullptr;
    const void* fn_gint = nullptr;
    const void* fn_gint_t1 = nullptr;
};

template <typename T, int S, int NTU, int UNITS, int UE, int UO, int GE, int GO>
constexpr const void* unit_hop_fn() {
    if constexpr (std::is_same<T, float>::value)
        return (const void*)&rk4_resident<T, S, NTU, UNITS, UE, UO, GE, GO, true>;
    else
        return nullptr;
}

// the potential variant: spin split (FP32) and shared blocks (FP32 and FP64;
// t = 1: FP32)
template <typename T, int S, int NTU, int UNITS, int UE, int UO, int GE, int GO>
constexpr const void* potential_fn() {
    return (const void*)&rk4_resident<T, S, NTU, UNITS, UE, UO, GE, GO, false, true>;
}

template <typename T, int S, int NTU, int UNITS, int UE, int UO, int GE, int GO>
constexpr const void* potential_t1_fn() {
    if constexpr (std::is_same<T, float>::value)
        return (const void*)&rk4_resident<T, S, NTU, UNITS, UE, UO, GE, GO, true, true>;
    else
        return nullptr;
}

template <typename T, int S, int NTU, int UNITS, int UE, int UO, int GE, int GO, bool T1>
constexpr const void* hopping_fn() {
    // spin split (FP32) and shared blocks (FP32 and FP64; t = 1: FP32)
    if constexpr (std::is_same<T, float>::value || !T1)
        return (const void*)&rk4_resident<T, S, NTU, UNITS, UE, UO, GE, GO, T1, false, true>;
    else
        return nullptr;
}

template <typename T, int S, int NTU, int UNITS, int UE, int UO, int GE, int GO, bool T1>
constexpr const void* interaction_fn() {
    if constexpr (std::is_same<T, float>::value || !T1)
        return (const void*)&rk4_resident<T, S, NTU, UNITS, UE, UO, GE, GO, T1, false, false,
                                          true>;
    else
        return nullptr;
}

#define FTWA_RES_CFG(T, DT, S, NTU, UNITS, UE, UO, GE, GO)                    \
    Config{DT, S, NTU, UNITS, UE, UO, GE, GO,                                    \
           (const void*)&rk4_resident<T, S, NTU, UNITS, UE, UO, GE, GO, false>, \
           unit_hop_fn<T, S, NTU, UNITS, UE, UO, GE, GO>(), 1, 0, 0, 0, 0, true, \
           potential_fn<T, S, NTU, UNITS, UE, UO, GE, GO>(),                     \
           potential_t1_fn<T, S, NTU, UNITS, UE, UO, GE, GO>(),                  \
           hopping_fn<T, S, NTU, UNITS, UE, UO, GE, GO, false>(),                \
           hopping_fn<T, S, NTU, UNITS, UE, UO, GE, GO, true>(),                 \
           interaction_fn<T, S, NTU, UNITS, UE, UO, GE, GO, false>(),            \
           interaction_fn<T, S, NTU, UNITS, UE, UO, GE, GO, true>()}

template <typename T, int G, int NTU, int UE, int UO, int UB, int GE1, int GE2, int GO, int XO,
          int KB>
constexpr const void* split_unit_hop_fn() {
    if constexpr (std::is_same<T, float>::value)
        return (const void*)&rk4_split<T, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB, true>;
    else
        return nullptr;
}

#define FTWA_SPLIT_CFG(T, DT, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB, AUTO)              \
    Config{DT, 1, NTU, 1, UE, UO, GE1, GO,                                                   \
           (const void*)&rk4_split<T, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB, false>,     \
           split_unit_hop_fn<T, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB>(), G, UB, GE2, XO, KB, \
           AUTO, (const void*)&rk4_split<T, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB, false, true>, \
           nullptr,                                                                          \
           (const void*)&rk4_split<T, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB, false, false, false, \
                                   true>,                                                    \
           nullptr,                                                                          \
           (const void*)&rk4_split<T, G, NTU, UE, UO, UB, GE1, GE2, GO, XO, KB, false, false, true>, \
           nullptr}

const Config kConfigs[] = {
    FTWA_RES_CFG(double, FTWA_F64, 2, 64, 16, 1, 1, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 128, 8, 2, 2, 2, 2),
    FTWA_RES_CFG(double, FTWA_F64, 2, 256, 3, 3, 3, 3, 3),
    FTWA_RES_CFG(double, FTWA_F64, 2, 512, 1, 5, 5, 5, 5),
    FTWA_RES_CFG(float, FTWA_F32, 2, 64, 16, 1, 1, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 128, 8, 2, 2, 2, 2),
    FTWA_RES_CFG(float, FTWA_F32, 2, 256, 4, 3, 3, 3, 3),
    FTWA_RES_CFG(float, FTWA_F32, 2, 512, 1, 5, 5, 5, 5),
    FTWA_RES_CFG(float, FTWA_F32, 1, 768, 1, 8, 8, 2, 2),
    FTWA_RES_CFG(float, FTWA_F32, 1, 768, 1, 13, 13, 2, 2),
    FTWA_RES_CFG(float, FTWA_F32, 1, 1024, 1, 10, 10, 2, 2),
    FTWA_RES_CFG(float, FTWA_F32, 1, 512, 1, 20, 20, 2, 2),
    FTWA_RES_CFG(float, FTWA_F32, 1, 768, 1, 13, 13, 13, 13),
    // the shared-block tiles with only the first slot of each class general
    FTWA_RES_CFG(double, FTWA_F64, 2, 128, 8, 2, 2, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 256, 3, 3, 3, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 512, 1, 5, 5, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 128, 8, 2, 2, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 256, 4, 3, 3, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 512, 1, 5, 5, 1, 1),
    // spin blocks split over workgroups (FP64 blocks larger than one CU)
    FTWA_SPLIT_CFG(double, FTWA_F64, 2, 512, 6, 6, 4, 1, 2, 1, 2, 1, true),
    FTWA_SPLIT_CFG(double, FTWA_F64, 3, 512, 7, 7, 4, 1, 1, 2, 4, 2, true),
    FTWA_SPLIT_CFG(double, FTWA_F64, 4, 512, 5, 5, 2, 1, 1, 1, 4, 3, true),
    // two parts of 768 threads (three waves per SIMD): 12 % faster than 512
    // threads at N = 150; at three and four parts the extra waves spill
    FTWA_SPLIT_CFG(double, FTWA_F64, 2, 768, 4, 4, 3, 1, 1, 1, 2, 1, true),
    // FP64 shared-block tiles of 384 threads x 2 units with (2, 2) slots: the
    // same 768 entries per class as 256 x (3, 3), with two thirds of its
    // registers per thread (the wider tiles spill in FP64)
    FTWA_RES_CFG(double, FTWA_F64, 2, 384, 2, 2, 2, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 384, 2, 2, 2, 2, 2),
    // fewer units per workgroup: the per-stage barriers span fewer waves and
    // more workgroups share a CU, so one workgroup's barrier wait overlaps
    // the others' work (a single-wave workgroup's barrier is nearly free):
    // 12 sites FP32 6.1e8 -> 1.06e9 (64 x 1), 24 sites 1.6e8 -> 2.5e8
    // (128 x 1), 54 sites 4.7e7 -> 5.9e7 (256 x 1); FP64 12 sites 4.3e8 ->
    // 5.8e8, 24 sites 7.9e7 -> 1.26e8 (FP64 384 x 1 is slower than 384 x 2)
    FTWA_RES_CFG(double, FTWA_F64, 2, 64, 8, 1, 1, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 64, 8, 1, 1, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 64, 4, 1, 1, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 64, 4, 1, 1, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 64, 2, 1, 1, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 64, 2, 1, 1, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 64, 1, 1, 1, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 64, 1, 1, 1, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 128, 1, 2, 2, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 128, 1, 2, 2, 1, 1),
    FTWA_RES_CFG(double, FTWA_F64, 2, 384, 1, 2, 2, 1, 1),
    FTWA_RES_CFG(float, FTWA_F32, 2, 256, 1, 3, 3, 1, 1),
};

// Order of preference of the first-fit choice (of tiles with the same slots,
// fewer units per workgroup first, then fewer general slots; indices are
// those of kConfigs).
const int kPreference[] = {31, 29, 27, 25, 0, 33, 13, 1, 23, 24, 35, 14, 2, 15, 3,
                           32, 30, 28, 26, 4, 34, 16, 5, 36, 17, 6, 18, 7,
                           8, 9, 10, 11, 12, 22, 19, 20, 21};
static_assert(sizeof(kPreference) == sizeof(kConfigs) / sizeof(kConfigs[0]) * sizeof(int),
              "every configuration has a place in the preference order");

constexpr size_t kMaxLds = 160 * 1024;  // the kernel declares no static LDS

// Dynamic LDS of a launch: the state blocks (S = 1: after two copies of the
// partner's diagonal, room for 256 reals each), then the per-wave record sums
// and the abort flag.
size_t lds_blocks(const Config& c, int N, int P) {
    (void)N;
    const size_t cb = c.dtype == FTWA_F64 ? 16 : 8;
    const size_t tail = c.S == 1 ? 33 : 2;  // zero slot(s) and scratch slot
    const size_t b = (size_t)c.UNITS * c.S * (P + tail) * cb + (c.S == 1 ? 2 * 256 * (cb / 2) : 0);
    return (b + 15) / 16 * 16;
}
size_t lds_tail(const Config& c) { return (size_t)(c.NTU * c.UNITS / 64) * 2 * c.S * 8 + 16; }
size_t lds_bytes(const Config& c, int N, int P) { return lds_blocks(c, N, P) + lds_tail(c); }
// The split kernel: two copies of the partner's diagonal, then the owned and
// halo elements, 32 zero slots and the scratch slot of the largest part.
size_t split_lds_bytes(const Config& c, int max_slots) {
    const size_t cb = c.dtype == FTWA_F64 ? 16 : 8;
    const size_t b = 2 * 256 * (cb / 2) + (size_t)(max_slots + 33) * cb;
    return (b + 15) / 16 * 16 + lds_tail(c);
}
// Published words per element of the split kernel, and per group of 2G
// workgroups: [2 spins][G parts][2 parities][entries][words].
int64_t split_words(const Config& c) {
    const int64_t w = c.dtype == FTWA_F64 ? 4 : 2;
    return 2 * (int64_t)c.G * 2 * (int64_t)c.NTU * (c.UE + c.UO) * w;
}

}  // namespace

bool resident_plan(int N, ftwa_dtype dtype, const DeviceTables& tab, ResidentPlan* plan,
                   int force_config, bool allow_split, bool need_potential, bool need_hop,
                   bool need_interaction) {
    if (!tab.bipartite) return false;
    const int P = (int)packed_count(N);
    const int n_even = (int)tab.n_even, n_odd = P - n_even;
    const int n_cfg = (int)(sizeof(kConfigs) / sizeof(kConfigs[0]));
    for (int o = 0; o < n_cfg; ++o) {
        const int k = kPreference[o];
        if (force_config >= 0 && k != force_config) continue;
        const Config& c = kConfigs[k];
        bool u_lds = false;
        if (c.dtype != dtype) continue;
        if (!c.auto_pick && force_config < 0) continue;
        if (need_potential && !c.fn_pot) continue;
        if (need_hop && !c.fn_hop) continue;
        if (need_interaction && !c.fn_gint) continue;
        if (N > c.NTU) continue;  // the diagonal must sit in slot 0
        size_t lds;
        if (c.G > 1) {
            // the split kernel: every part must fit (no invariant sums)
            if (!allow_split || N > 256) continue;
            const SplitShape& sh = tab.split[c.G];
            const int64_t n = c.NTU;
            if (n * c.UE < sh.n_even || n * c.UO < sh.n_odd) continue;
            if (n * c.GE < sh.int_gen || n * (c.UE - c.UB) < sh.n_bnd || n * c.GE2 < sh.bnd_gen)
                continue;
            if (n * c.GO < sh.odd_gen || n * c.XO < sh.odd_x) continue;
            if (sh.max_slots + 33 > 0x7fff) continue;
            lds = split_lds_bytes(c, sh.max_slots);
            if (need_interaction) lds += 3 * 256 * (c.dtype == FTWA_F64 ? 8 : 4);  // D, h copies
            else if (need_hop) lds += 256 * 6 * (c.dtype == FTWA_F64 ? 8 : 4);  // ratio table
            else if (need_potential) lds += 256 * (c.dtype == FTWA_F64 ? 8 : 4);  // the profile
        } else {
            if (P + 33 > 0x7fff) continue;
            if ((int64_t)c.NTU * c.UE < n_even || (int64_t)c.NTU * c.UO < n_odd) continue;
            if ((int64_t)c.NTU * c.GE < tab.n_gen_even || (int64_t)c.NTU * c.GO < tab.n_gen_odd)
                continue;
            lds = lds_bytes(c, N, P);
            // spin split: the potential's profile, the general interaction's
            // D and two site-ordered copies of the partner's diagonal, or the
            // first kHopLds places of the complex-hopping stage table; shared
            // blocks: D of every unit and spin or the profile (one value per
            // site at the element stride), or the whole ratio table
            const size_t tb = c.dtype == FTWA_F64 ? 8 : 4;
            const size_t cbb = 2 * tb;
            if (need_interaction) {
                lds += c.S == 1 ? 3 * 256 * tb : ((size_t)c.UNITS * 2 * N * cbb + 15) / 16 * 16;
                // shared blocks: a copy of u and the units' h = d + 1/2 in
                // site order beside D where they fit (read there by the
                // per-stage chains instead of from L2 and the blocks)
                const size_t ub = (size_t)umat_rows(N) * N * tb +  // multiples of 16
                                  (size_t)c.UNITS * 2 * umat_rows(N) * tb;
                if (c.S == 2 && lds + ub <= kMaxLds) {
                    lds += ub;
                    u_lds = true;
                }
            }
            else if (need_hop)
                lds += c.S == 1 ? (size_t)kHopLds * 6 * tb : ((size_t)N * 3 * cbb + 15) / 16 * 16;
            else if (need_potential)
                lds += c.S == 1 ? 256 * tb : ((size_t)N * cbb + 15) / 16 * 16;
        }
        if (lds > kMaxLds) continue;
        plan->config = k;
        plan->spins_per_unit = c.S;
        plan->threads = c.NTU * c.UNITS;
        plan->units = c.UNITS;
        plan->even_slots = (int64_t)c.NTU * c.UE;
        plan->odd_slots = (int64_t)c.NTU * c.UO;
        plan->lds = lds;
        plan->bnd_entry = (int64_t)c.NTU * c.UB;
        plan->u_lds = u_lds;
        return true;
    }
    return false;
}

int resident_config_count() { return (int)(sizeof(kConfigs) / sizeof(kConfigs[0])); }

int resident_spins(int config) { return kConfigs[config].S; }
int resident_parts(int config) { return kConfigs[config].G; }
bool resident_has_potential(int config) { return kConfigs[config].fn_pot != nullptr; }
bool resident_has_hop(int config) { return kConfigs[config].fn_hop != nullptr; }
bool resident_has_interaction(int config) { return kConfigs[config].fn_gint != nullptr; }

int64_t resident_item_traj(int config) {
    const Config& c = kConfigs[config];
    return c.S == 1 ? 1 : c.UNITS;
}

namespace {
int device_cus() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    return cus;
}
}  // namespace

ftwa_status resident_prepare(int config, size_t lds) {
    (void)lds;  // the limit is raised to the whole LDS once; launches use less
    FTWA_HIP_TRY(hipFuncSetAttribute(kConfigs[config].fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    if (kConfigs[config].fn_t1)
        FTWA_HIP_TRY(hipFuncSetAttribute(kConfigs[config].fn_t1,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    if (kConfigs[config].fn_pot)
        FTWA_HIP_TRY(hipFuncSetAttribute(kConfigs[config].fn_pot,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    for (const void* f : {kConfigs[config].fn_pot_t1, kConfigs[config].fn_hop,
                          kConfigs[config].fn_hop_t1, kConfigs[config].fn_gint,
                          kConfigs[config].fn_gint_t1})
        if (f)
            FTWA_HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)kMaxLds));
    return FTWA_OK;
}

// Pairs of spin-split workgroups that are resident together: one workgroup
// per CU (LDS bound), pairs in groups of 8 (one per XCD).
int64_t resident_max_pairs() {
    const int64_t pairs = (int64_t)device_cus() / 2 / 8 * 8;
    return pairs < 8 ? 8 : pairs;
}

// Groups of 2G split workgroups resident together: whole groups per XCD.
int64_t split_max_groups(int G) {
    const int64_t per_xcd = (int64_t)device_cus() / 8 / (2 * G);
    return 8 * (per_xcd < 1 ? 1 : per_xcd);
}

// Trajectories (items) a spin-split launch runs at once, and its grid.
int64_t spin_split_slots(const Config& c) {
    return c.G > 1 ? split_max_groups(c.G) : resident_max_pairs();
}

int64_t resident_concurrency(int config, size_t lds) {
    const Config& c = kConfigs[config];
    if (c.S == 1) return spin_split_slots(c);
    // the occupancy query honours the dynamic-LDS limit of the kernel
    if (resident_prepare(config, kMaxLds) != FTWA_OK) return (int64_t)device_cus() * c.UNITS;
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c.fn, c.NTU * c.UNITS, lds) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    return (int64_t)per_cu * device_cus() * c.UNITS;
}

int64_t resident_grid(int config, size_t lds, int64_t n_items) {
    const Config& c = kConfigs[config];
    if (c.S == 1) {
        const int64_t units = std::min((n_items + 7) / 8 * 8, spin_split_slots(c));
        return 2 * (int64_t)c.G * units;
    }
    const int64_t cap = resident_concurrency(config, lds) / c.UNITS;
    return std::max<int64_t>(1, std::min(n_items, cap));
}

// Spin-split scratch of one launch: the mailbox words (split kernel: the
// published words of every group).
size_t mailbox_words(const Config& c, int Nmax, int64_t grid) {
    if (c.G > 1) return (size_t)(grid / (2 * c.G)) * (size_t)split_words(c);
    return (size_t)(grid / 2) * 2 * 2 * Nmax;
}

size_t resident_mailbox_bytes(int config, int Nmax, int64_t n_items) {
    const Config& c = kConfigs[config];
    if (c.S != 1) return 0;
    return mailbox_words(c, Nmax, resident_grid(config, 0, n_items)) * sizeof(uint64_t);
}


namespace {
// The ratio table of the complex-hopping variant: out[r][dpos[i]][n] = w[r][i][n]
// rounded once to T for n < deg(i), zero for a missing neighbour (whose
// caller-side value may be anything), r over the 2 n_steps + 1 half steps.
template <typename T>
__global__ __launch_bounds__(256) void hop_table_kernel(const double2* __restrict__ w,
                                                        const int32_t* __restrict__ nb,
                                                        const int32_t* __restrict__ dpos, int N,
                                                        int64_t n_rows, cplx_t<T>* __restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_rows * N * 3) return;
    const int64_t r = x / (3 * N);
    const int i = (int)(x / 3 - r * N), n = (int)(x % 3);
    cplx_t<T> v;
    v.x = 0;
    v.y = 0;
    if (n < nb[i * 4 + 3]) {
        const double2 a = w[x];
        v.x = (T)a.x;
        v.y = (T)a.y;
    }
    out[(r * N + (dpos ? dpos[i] : i)) * 3 + n] = v;
}
}  // namespace

ftwa_status hop_table(const double* hop_w, const int32_t* nb, const int32_t* dpos, int N,
                      int64_t n_steps, ftwa_dtype dtype, void* out, hipStream_t stream) {
    const int64_t n_rows = 2 * n_steps + 1, n = n_rows * N * 3;
    const dim3 grid((unsigned)((n + 255) / 256));
    const double2* w = reinterpret_cast<const double2*>(hop_w);
    if (dtype == FTWA_F64)
        hipLaunchKernelGGL(hop_table_kernel<double>, grid, dim3(256), 0, stream, w, nb, dpos, N,
                           n_rows, static_cast<cplx_t<double>*>(out));
    else
        hipLaunchKernelGGL(hop_table_kernel<float>, grid, dim3(256), 0, stream, w, nb, dpos, N,
                           n_rows, static_cast<cplx_t<float>*>(out));
    FTWA_LAUNCH_CHECK("hop_table_kernel");
    return FTWA_OK;
}

namespace {
// u of the general-interaction variant rounded once to T, blocked by four
// along k: out[((k / 4) N + i) 4 + k % 4] = u_ki, rows k >= N zero.
template <typename T>
__global__ __launch_bounds__(256) void umat_table_kernel(const double* __restrict__ u, int N,
                                                         int64_t n, T* __restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t kb = x / (4 * (int64_t)N);
    const int64_t rem = x - kb * 4 * N;
    const int64_t i = rem / 4;
    const int64_t k = 4 * kb + (rem & 3);
    out[x] = k < N ? (T)u[k * N + i] : (T)0;
}
}  // namespace

ftwa_status umat_table(const double* u_mat, int N, ftwa_dtype dtype, void* out,
                       hipStream_t stream) {
    const int64_t n = (int64_t)umat_rows(N) * N;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (dtype == FTWA_F64)
        hipLaunchKernelGGL(umat_table_kernel<double>, grid, dim3(256), 0, stream, u_mat, N, n,
                           static_cast<double*>(out));
    else
        hipLaunchKernelGGL(umat_table_kernel<float>, grid, dim3(256), 0, stream, u_mat, N, n,
                           static_cast<float*>(out));
    FTWA_LAUNCH_CHECK("umat_table_kernel");
    return FTWA_OK;
}

ftwa_status resident_launch(const ResidentLaunch& L, hipStream_t stream) {
    const Config& c = kConfigs[L.config];
    if (L.n_items <= 0) return FTWA_OK;
    ResidentArgs A;
    A.table = L.table;
    A.n_entries = L.n_entries;
    A.n_items = L.n_items;
    A.dt = L.dt;
    A.n_steps = L.n_steps;
    A.record_every = L.record_every;
    A.mailbox = static_cast<uint64_t*>(L.mailbox);
    A.Nmax = L.Nmax;
    A.tail_off = (uint32_t)(L.lds - lds_tail(c));
    A.error = L.error;
    A.spin_limit = L.spin_limit ? L.spin_limit : (c.G > 1 ? kSplitSpinLimit : kSpinLimit);
    void* args[] = {&A};
    // fault injection for tests of the timeout path: only the up-spin
    // workgroups of eight pairs run, so that each of them gives up its first
    // wait for the absent partner and exits
    const int64_t grid = (L.drop_partners && c.S == 1 && c.G == 1) ? 8 : L.grid;
    const bool t1 = L.unit_hop && !L.dumps;
    const void* fn = L.interaction ? (t1 && c.fn_gint_t1 ? c.fn_gint_t1 : c.fn_gint)
                     : L.hopping   ? (t1 && c.fn_hop_t1 ? c.fn_hop_t1 : c.fn_hop)
                     : L.potential ? (t1 && c.fn_pot_t1 ? c.fn_pot_t1 : c.fn_pot)
                                   : (t1 && c.fn_t1 ? c.fn_t1 : c.fn);
    if (!fn)
        return fail(FTWA_ENOTSUP, L.interaction ? "this configuration has no general-interaction variant"
                                  : L.hopping   ? "this configuration has no complex-hopping variant"
                                                : "this configuration has no external-potential variant");
    if (c.S == 1) {
        // every word starts at stage 0, which no wait accepts (a fill kernel,
        // no memset node)
        ftwa_status st = zero_words(static_cast<unsigned*>(L.mailbox),
                                    (int64_t)mailbox_words(c, L.Nmax, grid) * 2, stream);
        if (st != FTWA_OK) return st;
        // both workgroups of a pair must be resident at the same time: the
        // grid never exceeds one workgroup per CU; a cooperative launch checks
        // it (not available under graph capture, where the bounded waits
        // report a partner that never came)
        if (L.cooperative)
            FTWA_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3((unsigned)grid),
                                                    dim3(c.NTU * c.UNITS), args,
                                                    (unsigned)L.lds, stream));
        else
            FTWA_HIP_TRY(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(c.NTU * c.UNITS), args,
                                         (unsigned)L.lds, stream));
    } else {
        FTWA_HIP_TRY(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(c.NTU * c.UNITS), args,
                                     (unsigned)L.lds, stream));
    }
    return FTWA_OK;
}

}  // namespace ftwa
