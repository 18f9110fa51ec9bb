// Wilson pass D or D^H in FP32 for lattices with X = Y = 16, one column per
// thread: the shape for many right-hand sides at once (the batched CG
// iterations of the mixed-precision solve).
//
// A block of 256 threads owns one xy-plane of one column and walks t through
// a segment of time slices.  Lane p = x + 16 y; wave w holds rows y = 4w..4w+3,
// so each 16-lane row of a wave is one x-row of the plane.  Per slice:
//   x hops: every lane projects its own spinor for both x hops and forms the
//     backward-hop product with its own link, U_x(s)^H P psi(s); the
//     neighbours' halves are then read from lanes x +- 1 of the same row by
//     DPP rotations (row_ror), which wrap exactly as the periodic x boundary
//     does.  No memory traffic, and only the lane's own link is loaded.
//   y hops: the same two halves for y go through LDS (the forward projection
//     and the backward product, 96 bytes per site), so the y neighbours' links
//     are never loaded either.
//   z hops: the neighbouring planes' spinors and the backward link are read
//     from global memory (other blocks load them at about the same time).
//   t hops: the +t neighbour is the lane's next slice; the -t hop of the next
//     slice, U_t(s)^H P psi(s), is formed while this slice is current and
//     carried in registers.
// One column per thread keeps a lane's state (accumulator, carried half
// spinor, one hop's operands) within 128 VGPRs, so four waves share a SIMD.
// Work items (column group, plane, segment) are ordered in one of three ways
// (tx_item): planes fastest, column groups fastest, or quads of planes with
// the column groups of a quad consecutive.
//
// Empty asm statements with a memory clobber fence the sections of a slice:
// they keep the compiler from hoisting every load of the slice to its top,
// which would need far more than 128 registers per lane.
//
// NC = 1 or 2 columns per thread: with two, every link load serves both
// columns (the links are the largest part of the bytes a pass moves through
// the vector memory path), at two waves per SIMD instead of four.
//
// Epilogues as the other stencil shapes (TM_PLAIN, TM_NORM, TM_CG), with one
// partial per (column, plane, segment) at index col * (Z nseg) + seg Z + z.
// When e.st is given, a column that is not active in it stores nothing (its
// partials are not read by the CG kernels).
#pragma once

#include "wilson_dev.h"

namespace sc {

#define SC_TX_FENCE() asm volatile("" ::: "memory")

// ---- the kernel's index arithmetic, shared with the host-side range check
// (wilson_tx_check in k_stencil.hip walks every access of a launch with these
// functions and compares it with its descriptor's record size)
constexpr int kTxPlane = 256;             // sites of an xy-plane (X = Y = 16)
constexpr unsigned kTxSpinorBytes = 96u;  // per site of a spinor column: 12 complex64
constexpr unsigned kTxLinkBytes = 288u;   // per site of the links: 4 x 9 complex64

// work item L -> (column group, z-plane, t-segment), in one of three orders:
//   0: the planes of a segment consecutive (z fastest, then segment, then
//      column group): z neighbours shared in L2, links read once per group;
//   1: the column groups of a plane consecutive (then z, then segment): links
//      shared in L2 by all groups, z neighbours read again by each plane;
//   2: quads of Q = 4 consecutive planes (2 or 1 when Z is not a multiple of
//      4): the Q planes of one column group consecutive, then the next group on
//      the same quad, then the next quad, then the next segment.  The z
//      neighbours inside a quad and the quad's links are shared in L2; only
//      the two planes bordering the quad come from outside it.
struct TxItem {
    int cg, z, seg;
};
__host__ __device__ inline int tx_quad(int Z) { return Z % 4 == 0 ? 4 : (Z % 2 == 0 ? 2 : 1); }
__host__ __device__ inline TxItem tx_item(int L, int ncg, int Z, int nseg, int order) {
    TxItem w;
    if (order == 1) {
        w.cg = L % ncg;
        const int r = L / ncg;
        w.z = r % Z;
        w.seg = r / Z;
    } else if (order == 2) {
        const int Q = tx_quad(Z);
        const int per_seg = Z * ncg;
        w.seg = L / per_seg;
        const int r = L % per_seg;
        const int quad = r / (Q * ncg), r2 = r % (Q * ncg);
        w.cg = r2 / Q;
        w.z = quad * Q + r2 % Q;
    } else {
        w.z = L % Z;
        const int r = L / Z;
        w.seg = r % nseg;
        w.cg = r / nseg;
    }
    return w;
}
// column c of group cg: a column past k (a partial last group) repeats the last one
__host__ __device__ inline int tx_col(int cg, int c, int nc, int k) {
    const int j = cg * nc + c;
    return j < k ? j : k - 1;
}
__host__ __device__ inline int tx_site(int p, int z, int t, int Z) { return p + kTxPlane * (z + Z * t); }
// offset from a site of plane z to the same (x, y, t) on plane z + 1 (dir > 0) or z - 1, periodic
__host__ __device__ inline int tx_zstep(int z, int Z, int dir) {
    if (dir > 0) return z == Z - 1 ? -(Z - 1) * kTxPlane : kTxPlane;
    return z == 0 ? (Z - 1) * kTxPlane : -kTxPlane;
}
__host__ __device__ inline int tx_tprev(int t, int T) { return t == 0 ? T - 1 : t - 1; }
// the site one slice up from site s of slice t, periodic
__host__ __device__ inline int tx_tnext_site(int s, int t, int T, int Z) {
    return t == T - 1 ? s - (T - 1) * kTxPlane * Z : s + kTxPlane * Z;
}
__host__ __device__ inline unsigned tx_boff(unsigned site) { return site * 8u; }               // per-lane part
__host__ __device__ inline unsigned tx_soff(int comp, unsigned V) { return (unsigned)comp * V * 8u; }  // wave-uniform

// Memory access through buffer resources: one descriptor per array (a
// spinor column, the links, the output column), the component's byte offset
// (comp * V * 8, wave-uniform) in a scalar register and the site's byte
// offset (site * 8) in one vector register shared by every component, so a
// site's 12 spinor or 9 link loads need no per-component address registers.
// Each descriptor's record count is its array's exact size in bytes, so every
// access of the kernel is in range (the host allows this shape only when the
// link array, the largest, is below 2^31 bytes, so no 32-bit offset wraps).
// The fourth descriptor word is the gfx9 format word for untyped dword access.
struct TxBuf {
    __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ TxBuf tx_buf(const float* base, unsigned bytes) {
    return {__builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000)};
}
__device__ __forceinline__ cplx<float> tx_ld(const TxBuf& b, unsigned boff, unsigned soff) {
    const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)boff, (int)soff, 0));
    return {v.x, v.y};
}
__device__ __forceinline__ void tx_st(const TxBuf& b, unsigned boff, unsigned soff, cplx<float> c) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned,
                                                             float2{c.re, c.im}),
                                          b.r, (int)boff, (int)soff, 0);
}
__device__ __forceinline__ void tx_spinor(const TxBuf& f, unsigned V, unsigned site, cplx<float> psi[4][3]) {
    const unsigned boff = tx_boff(site);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) psi[s][c] = tx_ld(f, boff, tx_soff(s * 3 + c, V));
}
// A value the optimizer cannot see through: a link loaded a second time with
// it is a second load, not the first load's registers kept live across the
// sections in between (which would cost 18 registers per lane).
__device__ __forceinline__ unsigned tx_opaque(unsigned x) {
    asm volatile("" : "+v"(x));
    return x;
}
// REC (links in SU(3)): rows 0 and 1 are read, row 2 rebuilt from them
template <bool REC>
__device__ __forceinline__ void tx_link(const TxBuf& U, unsigned V, int mu, unsigned site, cplx<float> u[3][3]) {
    const unsigned boff = tx_boff(site);
#pragma unroll
    for (int a = 0; a < (REC ? 2 : 3); ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u[a][b] = tx_ld(U, boff, tx_soff((mu * 3 + a) * 3 + b, V));
    if constexpr (REC) su3_row2(u);
}

template <bool DAG, int EPI, int NC, bool REC>
__global__ __launch_bounds__(kBlock, NC == 1 ? 4 : 3) void k_wilson_tx(float* __restrict__ out, int64_t ldo,
                                                                     const float* __restrict__ in, int64_t ldi,
                                                                     const float* __restrict__ U, Geom g, float kappa,
                                                                     float tsign, int k, int nseg, int tlen,
                                                                     int per_xcd, int order, TmEpi e) {
    using C = cplx<float>;
    // per lane and column: P psi for the -y neighbour (colours 0..2), U^H P psi for the +y one
    __shared__ float4 ys[NC][6][kBlock];
    __shared__ double nsh[kWaves];
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    const int ncg = (k + NC - 1) / NC;  // column groups
    if (L >= ncg * g.Z * nseg) return;  // uniform over the block
    const TxItem wi = tx_item(L, ncg, g.Z, nseg, order);
    const int cg = wi.cg, z = wi.z, seg = wi.seg;
    // the group's columns; a column past k (a partial last group) repeats the
    // last one and stores nothing, as does a column not active in e.st
    int col[NC];
    bool upd[NC];
    bool any = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        col[c] = tx_col(cg, c, NC, k);
        upd[c] = cg * NC + c < k && (!e.st || e.st[col[c]].active);
        any |= upd[c];
    }
    if (!any) return;  // uniform over the block
    constexpr int SF = DAG ? 1 : -1;  // projector sign of the forward hop
    constexpr int SB = -SF;
    const int t0 = seg * tlen;
    const int t1 = min(g.T, t0 + tlen);
    const int p = threadIdx.x;
    const int pyp = (p + 16) & (kBlock - 1), pym = (p - 16) & (kBlock - 1);
    static_assert(kBlock == kTxPlane, "a block is one xy-plane");
    const unsigned uV = (unsigned)g.V;
    const int zoff_p = tx_zstep(z, g.Z, 1);
    const int zoff_m = tx_zstep(z, g.Z, -1);
    const unsigned colbytes = kTxSpinorBytes * uV;
    const TxBuf Ub = tx_buf(U, kTxLinkBytes * uV);
    TxBuf src[NC], dst[NC];
    float alpha[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        src[c] = tx_buf(in + (int64_t)col[c] * ldi, colbytes);
        // a column that stores nothing gets a zero-size record (its stores are
        // dropped by the hardware's range check; a branch would split the slice)
        const unsigned nb = upd[c] ? colbytes : 0u;
        dst[c] = EPI == TM_CG ? tx_buf((const float*)e.r + (int64_t)col[c] * e.ldr, nb)
                              : tx_buf(out + (int64_t)col[c] * ldo, nb);
        alpha[c] = 0.0f;
    }
    if constexpr (EPI == TM_CG) {
        const int G = g.Z * nseg;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double pq = sum_partials(e.pq + (int64_t)col[c] * G, G, nsh);
            alpha[c] = upd[c] ? (float)(e.st[col[c]].rho / pq) : 0.0f;
        }
    }
    const float rk = -1.0f / kappa;  // acc starts at -psi / kappa, so D psi = -kappa acc
    double nacc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) nacc[c] = 0.0;

    // the -t hop into slice t0, from slice t0 - 1
    C cr0[NC][3], cr1[NC][3];
    {
        const int tm = tx_tprev(t0, g.T);
        const unsigned sm = (unsigned)tx_site(p, z, tm, g.Z);
        const float bf = t0 == 0 ? tsign : 1.0f;
        C u[3][3];
        tx_link<REC>(Ub, uV, 3, sm, u);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            C psi[4][3], h0[3], h1[3];
            tx_spinor(src[c], uV, sm, psi);
            project<3, SB>(psi, h0, h1);
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                h0[cc] = {h0[cc].re * bf, h0[cc].im * bf};
                h1[cc] = {h1[cc].re * bf, h1[cc].im * bf};
            }
            su3_mul<true>(u, h0, cr0[c]);
            su3_mul<true>(u, h1, cr1[c]);
        }
    }
    C cur[NC][4][3];
#pragma unroll
    for (int c = 0; c < NC; ++c) tx_spinor(src[c], uV, (unsigned)tx_site(p, z, t0, g.Z), cur[c]);

#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
        const unsigned s = (unsigned)tx_site(p, z, t, g.Z);
        C acc[NC][4][3];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) acc[c][a][cc] = {cur[c][a][cc].re * rk, cur[c][a][cc].im * rk};
            hop_acc<3, SB>(acc[c], cr0[c], cr1[c]);  // the carried -t hop
        }
        // y, source side: the halves the +-y neighbours need, into LDS
        {
            C u[3][3];
            tx_link<REC>(Ub, uV, 1, s, u);
            __syncthreads();  // the previous slice's reads of ys are done
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C h0[3], h1[3], c0[3], c1[3];
                project<1, SB>(cur[c], h0, h1);
                su3_mul<true>(u, h0, c0);
                su3_mul<true>(u, h1, c1);
                project<1, SF>(cur[c], h0, h1);
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    ys[c][cc][p] = float4{h0[cc].re, h0[cc].im, h1[cc].re, h1[cc].im};
                    ys[c][3 + cc][p] = float4{c0[cc].re, c0[cc].im, c1[cc].re, c1[cc].im};
                }
            }
        }
        SC_TX_FENCE();
        // x: both hops through the lanes of this row
        {
            C u[3][3];
            tx_link<REC>(Ub, uV, 0, s, u);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C h0[3], h1[3], g0[3], g1[3], c0[3], c1[3];
                project<0, SF>(cur[c], h0, h1);
                project<0, SB>(cur[c], g0, g1);
                su3_mul<true>(u, g0, c0);
                su3_mul<true>(u, g1, c1);
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    h0[cc] = {dpp_from_xp(h0[cc].re), dpp_from_xp(h0[cc].im)};
                    h1[cc] = {dpp_from_xp(h1[cc].re), dpp_from_xp(h1[cc].im)};
                    c0[cc] = {dpp_from_xm(c0[cc].re), dpp_from_xm(c0[cc].im)};
                    c1[cc] = {dpp_from_xm(c1[cc].re), dpp_from_xm(c1[cc].im)};
                }
                hop_acc<0, SB>(acc[c], c0, c1);
                su3_mul<false>(u, h0, c0);
                su3_mul<false>(u, h1, c1);
                hop_acc<0, SF>(acc[c], c0, c1);
            }
        }
        SC_TX_FENCE();
        // t: the -t hop of the next slice, formed from this one (the last use of cur)
        {
            C u[3][3];
            tx_link<REC>(Ub, uV, 3, s, u);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C h0[3], h1[3];
                project<3, SB>(cur[c], h0, h1);
                su3_mul<true>(u, h0, cr0[c]);
                su3_mul<true>(u, h1, cr1[c]);
            }
        }
        SC_TX_FENCE();
        // z: the neighbouring planes from global memory
        {
            C u[3][3];
            tx_link<REC>(Ub, uV, 2, s, u);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C psi[4][3], h0[3], h1[3], c0[3], c1[3];
                tx_spinor(src[c], uV, (unsigned)((int)s + zoff_p), psi);
                project<2, SF>(psi, h0, h1);
                su3_mul<false>(u, h0, c0);
                su3_mul<false>(u, h1, c1);
                hop_acc<2, SF>(acc[c], c0, c1);
            }
        }
        SC_TX_FENCE();
        {
            C u[3][3];
            const unsigned sm = (unsigned)((int)s + zoff_m);
            tx_link<REC>(Ub, uV, 2, sm, u);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C psi[4][3], h0[3], h1[3], c0[3], c1[3];
                tx_spinor(src[c], uV, sm, psi);
                project<2, SB>(psi, h0, h1);
                su3_mul<true>(u, h0, c0);
                su3_mul<true>(u, h1, c1);
                hop_acc<2, SB>(acc[c], c0, c1);
            }
        }
        SC_TX_FENCE();
        // y, destination side
        {
            C u[3][3];
            __syncthreads();  // every lane's halves are in ys
            tx_link<REC>(Ub, uV, 1, tx_opaque(s), u);  // U_y(s) again
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C h0[3], h1[3], c0[3], c1[3];
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    const float4 a = ys[c][cc][pyp];
                    const float4 bb = ys[c][3 + cc][pym];
                    h0[cc] = {a.x, a.y};
                    h1[cc] = {a.z, a.w};
                    c0[cc] = {bb.x, bb.y};
                    c1[cc] = {bb.z, bb.w};
                }
                hop_acc<1, SB>(acc[c], c0, c1);
                su3_mul<false>(u, h0, c0);
                su3_mul<false>(u, h1, c1);
                hop_acc<1, SF>(acc[c], c0, c1);
            }
        }
        SC_TX_FENCE();
        // +t with the next slice, which becomes current, and the epilogue, one
        // column after the other: a column's r (TM_CG) is loaded together with
        // its next slice, so the epilogue's loads are waited for together with
        // the +t hop's instead of after it, and the registers of one column's r
        // are those its finished accumulator frees
        const bool tlast = t == g.T - 1;
        const unsigned sn = (unsigned)tx_tnext_site((int)s, t, g.T, g.Z);
        // the boundary sign as a multiply, not a branch: a branch here splits
        // the slice into basic blocks and the allocation across them spills
        const float bf = tlast ? tsign : 1.0f;
        {
            C u[3][3];
            tx_link<REC>(Ub, uV, 3, tx_opaque(s), u);  // U_t(s) again
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                C q[4][3];
                if constexpr (EPI == TM_CG) {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) q[a][cc] = tx_ld(dst[c], tx_boff(s), tx_soff(a * 3 + cc, uV));
                }
                tx_spinor(src[c], uV, sn, cur[c]);  // cur is dead since the t section: the next slice
                C h0[3], h1[3], c0[3], c1[3];
                project<3, SF>(cur[c], h0, h1);
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    h0[cc] = {h0[cc].re * bf, h0[cc].im * bf};
                    h1[cc] = {h1[cc].re * bf, h1[cc].im * bf};
                }
                su3_mul<false>(u, h0, c0);
                su3_mul<false>(u, h1, c1);
                hop_acc<3, SF>(acc[c], c0, c1);
                // out = psi - kappa H psi = -kappa acc, or r -= alpha out
                float sq = 0.0f;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        C r = {-kappa * acc[c][a][cc].re, -kappa * acc[c][a][cc].im};
                        if constexpr (EPI == TM_CG) r = {q[a][cc].re - alpha[c] * r.re, q[a][cc].im - alpha[c] * r.im};
                        tx_st(dst[c], tx_boff(s), tx_soff(a * 3 + cc, uV), r);
                        sq = __builtin_fmaf(r.re, r.re, sq);
                        sq = __builtin_fmaf(r.im, r.im, sq);
                    }
                // |.|^2 of the site in FP32 (12 components), summed over sites in FP64
                if constexpr (EPI != TM_PLAIN) nacc[c] += (double)sq;
                SC_TX_FENCE();  // the next column's loads stay after this column's epilogue
            }
        }
    }
    if constexpr (EPI != TM_PLAIN) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double tot = block_sum(nacc[c], nsh);
            if (p == 0 && upd[c]) e.part[(int64_t)col[c] * (g.Z * nseg) + seg * g.Z + z] = tot;
        }
    }
}

#undef SC_TX_FENCE

}  // namespace sc
