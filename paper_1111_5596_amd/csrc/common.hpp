// Lattice geometry, lattice-object types and the device storage layout,
// shared by the host runtime and the kernels.
//
// Device layout: checkerboard site order, 64-site tiles.
//   cb(x, y, z, t) = p * V/2 + (x/2) + (Lx/2) * (y + Ly * (z + Lz * t)),
//   p = (x + y + z + t) mod 2,
// so the even sites come first, each parity half is ordered like the
// lexicographic order with x halved, and a time slice is a contiguous range
// of Vs/2 sites in each half.  Sites are grouped in tiles of 64 consecutive
// checkerboard sites (one wavefront); a tile stores, for each of its rows, the
// 64 sites' values of one component, one row after the other:
//   row r*ncomp + k  component k of record r (nrec records of ncomp complex)
//   F64   double2 elements  (1024-byte rows)
//   F32   float2 elements   ( 512-byte rows)
//   F16S  half2 elements    ( 256-byte rows), then nrec rows of FP32 record
//         scales
// Lanes of a wavefront read consecutive elements of a row (coalesced), and all
// the components of a site block sit in one contiguous tile, so a wavefront
// touches one memory page per neighbouring tile instead of one per component
// plane (the paper's kernels used uncoalesced per-site records, section 6).
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/qdpmi.h"

#if defined(__HIPCC__)
#define QDP_HD __host__ __device__
#else
#define QDP_HD
#endif

namespace qdpmi {

struct TypeShape {
    int32_t nrec;            // records per site
    int32_t ncomp;           // complex components per record
    int32_t s1, s2, c1, c2;  // spin row/col and colour row/col extents
};

QDP_HD inline TypeShape type_shape(int32_t type) {
    switch (type) {
        case QDP_REAL: return {1, 1, 1, 1, 1, 1};
        case QDP_COMPLEX: return {1, 1, 1, 1, 1, 1};
        case QDP_COLOR_VECTOR: return {1, 3, 1, 1, 3, 1};
        case QDP_COLOR_MATRIX: return {1, 9, 1, 1, 3, 3};
        case QDP_FERMION: return {1, 12, 4, 1, 3, 1};
        case QDP_SPIN_MATRIX: return {1, 16, 4, 4, 1, 1};
        case QDP_PROPAGATOR: return {1, 144, 4, 4, 3, 3};
        case QDP_GAUGE: return {4, 9, 1, 1, 3, 3};
        default: return {0, 0, 0, 0, 0, 0};
    }
}

QDP_HD inline bool valid_type(int32_t t) { return t >= QDP_REAL && t <= QDP_GAUGE; }
QDP_HD inline bool valid_prec(int32_t p) { return p >= QDP_F64 && p <= QDP_F16S; }

// F16S scale of an all-zero record: the smallest normal FP32 power of two
// (any scale decodes zeros; this one never outweighs a non-zero record when
// the smearing brings the records of a site's neighbours to a common scale).
constexpr float kF16sZeroScale = 0x1p-126f;

// Bytes per complex component in a plane (16, 8, 4: a power of two, so the
// offsets below take shifts and masks, not divisions; kernels evaluate them
// with the precision and record shape known only at run time).
QDP_HD constexpr int32_t prec_log2_bytes(int32_t prec) { return prec == QDP_F64 ? 4 : (prec == QDP_F32 ? 3 : 2); }
QDP_HD constexpr int64_t prec_complex_bytes(int32_t prec) { return int64_t(1) << prec_log2_bytes(prec); }

struct Geometry {
    int32_t L[4];   // Lx, Ly, Lz, Lt
    int32_t Lxh;    // Lx / 2
    int32_t pad;
    int64_t V;      // sites
    int64_t Vh;     // V / 2
    int64_t Vsh;    // sites per time slice per parity = Lx Ly Lz / 2
    int64_t plane;  // allocated sites: V rounded up to a whole number of 64-site tiles
};

inline Geometry make_geometry(const int32_t d[4]) {
    Geometry g;
    for (int i = 0; i < 4; ++i) g.L[i] = d[i];
    g.Lxh = d[0] / 2;
    g.pad = 0;
    g.V = (int64_t)d[0] * d[1] * d[2] * d[3];
    g.Vh = g.V / 2;
    g.Vsh = (int64_t)g.Lxh * d[1] * d[2];
    g.plane = (g.V + 63) / 64 * 64;
    return g;
}

// Bytes of one 64-site tile of a field.
QDP_HD constexpr int64_t tile_bytes(int32_t nrec, int32_t ncomp, int32_t prec) {
    return 64 * ((int64_t)nrec * ncomp * prec_complex_bytes(prec) + (prec == QDP_F16S ? 4 * (int64_t)nrec : 0));
}

// Device bytes of a field.
inline int64_t field_bytes(const Geometry& g, int32_t type, int32_t prec) {
    const TypeShape s = type_shape(type);
    return g.plane / 64 * tile_bytes(s.nrec, s.ncomp, prec);
}

// Byte offset of row 0 of site `site` (elements of `esize` bytes) in a field
// whose tiles are `tb` bytes.
QDP_HD constexpr int64_t tile_site_offset(int64_t tb, int64_t esize, int64_t site) {
    return (site >> 6) * tb + (site & 63) * esize;
}

// Inside a tile the components are stored in rows of 16-byte chunks: row q
// holds, for each of the 64 sites in turn, the q-th run of 16 / element-size
// consecutive components of the site (4 F16S, 2 F32 or 1 F64 complex
// numbers), so a lane fetches a chunk with one 16-byte load and a wavefront's
// load covers 1024 contiguous bytes.  Fields whose per-site component count
// is not a multiple of the chunk size (colour matrices, vectors and scalars
// in F16S/F32) keep one row per component instead.
QDP_HD constexpr int32_t chunk_elems(int32_t prec) { return 1 << (4 - prec_log2_bytes(prec)); }
QDP_HD constexpr bool chunked_layout(int32_t nrec, int32_t ncomp, int32_t prec) {
    return ((nrec * ncomp) & (chunk_elems(prec) - 1)) == 0;
}

// Byte offset of component k of record rec at `site`: element e = rec ncomp
// + k sits in chunk row e / CE at position e mod CE (chunked layout, CE =
// chunk_elems), else in row e.
QDP_HD constexpr int64_t comp_offset(int32_t nrec, int32_t ncomp, int32_t prec, int32_t rec, int32_t comp,
                                     int64_t site) {
    const int32_t les = prec_log2_bytes(prec), lce = 4 - les;
    const int64_t tb = tile_bytes(nrec, ncomp, prec);
    const int32_t e = rec * ncomp + comp;
    if (chunked_layout(nrec, ncomp, prec))
        return tile_site_offset(tb, 16, site) + ((int64_t)(e >> lce) << 10) + ((e & ((1 << lce) - 1)) << les);
    return tile_site_offset(tb, int64_t(1) << les, site) + ((int64_t)e << (6 + les));
}

// Byte offset of the F16S scale of record rec at `site`.
QDP_HD constexpr int64_t scale_offset(int32_t nrec, int32_t ncomp, int32_t rec, int64_t site) {
    return tile_site_offset(tile_bytes(nrec, ncomp, QDP_F16S), 4, site) + ((int64_t)nrec * ncomp + rec) * 64 * 4;
}

// The shifts and masks above against the plain division form of the layout,
// for every record shape, precision and component at sites in the first,
// second and a later tile.
constexpr bool layout_offsets_match_division_form() {
    const int32_t shapes[][2] = {{1, 1}, {1, 3}, {1, 9}, {1, 12}, {1, 16}, {1, 144}, {4, 9}};
    const int64_t sites[] = {0, 65, 1000};
    for (const auto& sh : shapes)
        for (int32_t prec = QDP_F64; prec <= QDP_F16S; ++prec) {
            const int64_t es = prec == QDP_F64 ? 16 : (prec == QDP_F32 ? 8 : 4), ce = 16 / es;
            const int64_t n = (int64_t)sh[0] * sh[1];
            const int64_t tb = 64 * (n * es + (prec == QDP_F16S ? 4 * sh[0] : 0));
            for (int32_t rec = 0; rec < sh[0]; ++rec)
                for (int32_t k = 0; k < sh[1]; ++k)
                    for (const int64_t site : sites) {
                        const int64_t e = (int64_t)rec * sh[1] + k;
                        const int64_t want = n % ce == 0 ? (site / 64) * tb + (site % 64) * 16 + (e / ce) * 1024 + (e % ce) * es
                                                         : (site / 64) * tb + (site % 64) * es + e * 64 * es;
                        if (comp_offset(sh[0], sh[1], prec, rec, k, site) != want) return false;
                    }
        }
    return true;
}
static_assert(layout_offsets_match_division_form(), "tile layout offsets");

// Checkerboard index of lexicographic coordinates.
QDP_HD inline int64_t cb_index(const Geometry& g, int32_t x, int32_t y, int32_t z, int32_t t) {
    const int32_t p = (x + y + z + t) & 1;
    return p * g.Vh + (x >> 1) + (int64_t)g.Lxh * (y + (int64_t)g.L[1] * (z + (int64_t)g.L[2] * t));
}

// 32-bit unsigned arithmetic: a lattice holds at most 2^31 sites.
QDP_HD inline void cb_coords(const Geometry& g, int64_t s, int32_t c[4]) {
    const uint32_t Vh = (uint32_t)g.Vh, Lxh = (uint32_t)g.Lxh, Ly = (uint32_t)g.L[1], Lz = (uint32_t)g.L[2];
    const uint32_t p = (uint32_t)s >= Vh ? 1u : 0u;
    const uint32_t i = (uint32_t)s - p * Vh;
    const uint32_t r1 = i / Lxh, r2 = r1 / Ly, r3 = r2 / Lz;
    c[1] = (int32_t)(r1 - r2 * Ly);
    c[2] = (int32_t)(r2 - r3 * Lz);
    c[3] = (int32_t)r3;
    c[0] = (int32_t)(2 * (i - r1 * Lxh) + ((p + (uint32_t)c[1] + (uint32_t)c[2] + r3) & 1u));
}

}  // namespace qdpmi
