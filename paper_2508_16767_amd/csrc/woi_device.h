// woi_device.h -- device-resident layout of a compiled Walk-on-Interfaces problem.
//
// One contiguous device blob: a DevProblem header followed by three payload arrays
// (doubles, floats, bytes).  Every table exists in FP64 (for the FP64 path) and in
// FP32 (for the mixed-precision path) so that neither path converts on the fly.
// Offsets are element offsets into the payload array of the matching type.
#pragma once
#include <stdint.h>

#include "woi.h"

namespace woi {

enum : int { REL_SAME = 1, REL_DESC = 2, REL_OTHER = 3 };

// Device-only data kind: DIRPOLY data in dimension 2 or 3 stored as a dense triangular
// coefficient table in nested-Horner order (nt = total degree n), followed by the center.
constexpr int DK_DIRPOLY_HORNER = 16;

// Geometry payload of one region (offsets g64 / g32, same layout in both types):
//   SPHERE     : c[m], R
//   ELLIPSOID  : c[m], A[m*m], L[m*m] (= A^{-1/2}), 1/lambda_max(A)
//   POLYLINE2D : vertices v[2*(nv+1)] (v[nv] = v[0]), segment lengths len[nv],
//                cumulative arclength cum[nv+1] (FP64; the FP32 table holds the pairs
//                (cum[j], 1/len[j]), j <= nv), outward unit normals nrm[2*nv].
// Mesh BVH (float payload, shared by both precisions): nodes in depth-first order, 8 floats
//   each: box min (3), box max (3) -- widened outward to stay conservative under FP32
//   rounding --, the index of the node that follows the subtree, and for a leaf
//   8 * (first entry in the leaf triangle list) + (triangle count <= 4), -1 for an inner node
//   (floats holding exact integers); the list holds original triangle indices.
// Polyline search tables (float payload, shared by both precisions):
//   for every level l >= 1 and aligned block b (vertices [b 2^l, min((b+1) 2^l, nv)]),
//   bnd[(N2 >> l) + b] bounds the distance of the block's vertices from its chord (heap
//   layout, N2 = nv rounded up to a power of two, entry 0 unused); the segments (level 0)
//   follow as bnd[N2 + j] = hband_f, so block (j, l) sits at (N2 + j) >> l at every level; the
//   walk starts at level top.  The FP32 vertex copy is padded with v[nv] up to N2 + 1
//   entries (a block [j, j + 2^l] past nv then ends on v[nv], the end of its chord).  Guide table (int payload): gd[k] = largest j with
//   cum[j] <= k L / nv.
struct DevRegion {
    int kind, dkind, nt, nv;
    int g64, g32;              // shape parameters / polyline vertices
    int len64, len32;          // polyline segment lengths
    int cum64, cum32;          // polyline cumulative lengths
    int nrm64, nrm32;          // polyline segment normals
    int bnd;                   // float offset of the block bounds (N2 + nv entries)
    int n2, top;               // nv rounded up to a power of two, first walk level
    int guide;                 // int offset of the guide table (nv entries)
    int d64, d32, dexp;        // data coefficients, DIRPOLY exponents (byte offset; 8 bytes per term)
    int b64, b32, nbrk, class0;// VR (2D): sign breakpoints of beta along arclength
    int lds_v, lds_b;          // byte offsets of the LDS copies (FP32 vertices, FP16 bounds), -1 if none
    int lds_c, lds_g;          // byte offsets of the LDS copies of the FP32 arclength CDF ((cum, 1/len)
                               // pairs) and of the guide table, -1 if they stay in global memory
    int bvh, nbvh, bvhidx;     // mesh: float offset of the BVH nodes, node count, int offset of the leaf triangle lists
    double alpha, sgn, s, area, meas[2], total;
    double gscale;             // polyline: nv / total length (guide-table index scale)
    float alpha_f, sgn_f, s_f, area_f, meas_f[2], total_f, gscale_f;
    float hband_f;             // polyline: |signed distance| below which FP32 walks decide a crossing in FP64
};

// Largest LDS staging area per workgroup: two 512-thread workgroups per CU share its
// 160 KB of LDS on gfx950 (256 bytes left for a kernel's own static LDS).
constexpr int LDS_BUDGET_MAX = 80 * 1024 - 256;

struct DevProblem {
    int dim, N, vr_ok, lds_bytes;             // lds_bytes: LDS needed to stage every polyline (0: none)
    double alpha_l1, unit_area, phi_c;        // |S^{m-1}|, Phi prefactor (m >= 3)
    float alpha_l1_f, unit_area_f, phi_c_f;
    float inv_unit_area_f;                    // 1 / |S^{m-1}| in FP32 (the gradient terms' factor)
    float sign_band_f;                        // FP32 walks: |(y_i - y_{i-1}) . n(y_i)| at or below it is
                                              // inside the dot product's rounding band (sign from FP64)
    double cdf[WOI_MAX_REGIONS];              // schedule CDF over |alpha| / ||alpha||_1
    // the CDF test on the 32-bit schedule word w itself: u(w) = (w + 1/2) 2^-32 < cdf[h] exactly
    // when w < sthr[h] (sthr[h] = ceil(cdf[h] 2^32 - 1/2), at least 0, at most 2^32)
    uint64_t sthr[WOI_MAX_REGIONS];
    unsigned char rel[WOI_MAX_REGIONS][WOI_MAX_REGIONS];
    // start of the inverse-CDF search for u in [k/64, (k+1)/64): the search's result at
    // u = k/64, so no region below it can be the result for a larger u
    unsigned char sguide[64];
    DevRegion reg[WOI_MAX_REGIONS];
    uint64_t off64, off32, offb, offi;        // byte offsets of the payload arrays
    uint64_t bytes;
};

}  // namespace woi
