// Lattice geometry, lattice-object types and the device storage layout,
// shared by the host runtime and the kernels.
//
// Device layout (structure of arrays, checkerboard site order):
//   cb(x, y, z, t) = p * V/2 + (x/2) + (Lx/2) * (y + Ly * (z + Lz * t)),
//   p = (x + y + z + t) mod 2,
// so the even sites come first, each parity half is ordered like the
// lexicographic order with x halved, and a time slice is a contiguous range
// of Vs/2 sites in each half.  A field is nrec records per site (4 colour
// matrices for a gauge field, 1 otherwise) of ncomp complex components;
// component k of record r is one plane of `plane` sites:
//   F64   double2 planes                      16 B per complex
//   F32   float2 planes                        8 B per complex
//   F16S  half2 planes, then nrec float scale planes (one scale per record)
// The paper's GPU kernels used uncoalesced per-site layouts (section 6);
// with this layout consecutive lanes of a wavefront read consecutive 8-byte
// (4-byte) words.
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

// Bytes per complex component in a plane.
QDP_HD inline int64_t prec_complex_bytes(int32_t prec) {
    return prec == QDP_F64 ? 16 : (prec == QDP_F32 ? 8 : 4);
}

struct Geometry {
    int32_t L[4];   // Lx, Ly, Lz, Lt
    int32_t Lxh;    // Lx / 2
    int32_t pad;
    int64_t V;      // sites
    int64_t Vh;     // V / 2
    int64_t Vsh;    // sites per time slice per parity = Lx Ly Lz / 2
    int64_t plane;  // plane stride in sites (V rounded up to 64)
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

// Device bytes of a field.
inline int64_t field_bytes(const Geometry& g, int32_t type, int32_t prec) {
    const TypeShape s = type_shape(type);
    int64_t b = (int64_t)s.nrec * s.ncomp * g.plane * prec_complex_bytes(prec);
    if (prec == QDP_F16S) b += (int64_t)s.nrec * g.plane * 4;
    return b;
}

// Offset in bytes of component plane (rec, comp).
QDP_HD inline int64_t plane_offset(int64_t plane, int32_t ncomp, int32_t prec, int32_t rec,
                                   int32_t comp) {
    return ((int64_t)rec * ncomp + comp) * plane * prec_complex_bytes(prec);
}

// Offset in bytes of the F16S scale plane of record rec.
QDP_HD inline int64_t scale_offset(int64_t plane, int32_t nrec, int32_t ncomp, int32_t rec) {
    return (int64_t)nrec * ncomp * plane * 4 + (int64_t)rec * plane * 4;
}

// Checkerboard index of lexicographic coordinates.
QDP_HD inline int64_t cb_index(const Geometry& g, int32_t x, int32_t y, int32_t z, int32_t t) {
    const int32_t p = (x + y + z + t) & 1;
    return p * g.Vh + (x >> 1) + (int64_t)g.Lxh * (y + (int64_t)g.L[1] * (z + (int64_t)g.L[2] * t));
}

QDP_HD inline void cb_coords(const Geometry& g, int64_t s, int32_t c[4]) {
    const int32_t p = s >= g.Vh ? 1 : 0;
    int64_t i = s - p * g.Vh;
    const int32_t h = (int32_t)(i % g.Lxh);
    i /= g.Lxh;
    c[1] = (int32_t)(i % g.L[1]);
    i /= g.L[1];
    c[2] = (int32_t)(i % g.L[2]);
    c[3] = (int32_t)(i / g.L[2]);
    c[0] = 2 * h + ((p + c[1] + c[2] + c[3]) & 1);
}

}  // namespace qdpmi
