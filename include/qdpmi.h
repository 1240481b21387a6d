/*
 * qdpmi: site-parallel lattice-field expressions, Jacobi smearing and meson
 * contractions on one AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The calls follow the problem statement of F. Winter, "Accelerating
 * QDP++/Chroma on GPUs" (Lattice 2011): expressions are evaluated site by
 * site over lattice objects (section 4.2 and Figure 3), lattice objects live
 * in device memory managed by a software cache over a pool reserved at start
 * up that spills least-recently-used objects (section 4.1 and Figure 2), and
 * the accelerated Chroma stages are source/sink smearing and the hadron
 * spectrum (section 5 and Figure 4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every call returns QDP_OK (0) or a negative qdp_status; no call
 *   throws.  qdp_last_error() returns a message for the last failure on the
 *   context.  A failing call leaves no partial writes in its destination
 *   fields unless stated otherwise.
 * - Ownership: the library owns fields and lattices (opaque handles freed
 *   with qdp_field_free / qdp_finalize).  Arrays passed in (nodes, handles,
 *   host buffers) are borrowed for the duration of the call only.  When the
 *   caller supplies pool memory (qdp_init_opts.pool_ptr) it must outlive the
 *   context.  Pinned host memory for spills is allocated and owned by the
 *   library.
 * - Streams: all device work is ordered on the context's stream.  Calls that
 *   return host data (qdp_field_read, qdp_sum_multi, qdp_hadron_contract,
 *   qdp_cache_stats) synchronise the stream; the others are asynchronous.
 *   One context per host thread.
 * - Lattices: extents (Lx, Ly, Lz, Lt) must all be even (sites are stored in
 *   checkerboard order) and at least 2.  Direction mu = 0, 1, 2 are x, y, z,
 *   mu = 3 is time; the time direction is the only supported j_decay.
 * - Canonical host layout (qdp_field_write / qdp_field_read): lexicographic
 *   sites s = x + Lx*(y + Ly*(z + Lz*t)), x fastest; complex numbers as
 *   interleaved (re, im) doubles; per-site index order
 *     REAL           [site]                      1 double per site
 *     COMPLEX        [site]                      2 doubles
 *     COLOR_VECTOR   [site][colour 3]
 *     COLOR_MATRIX   [site][row 3][col 3]
 *     FERMION        [site][spin 4][colour 3]
 *     SPIN_MATRIX    [site][row 4][col 4]
 *     PROPAGATOR     [site][spin row][spin col][colour row][colour col]
 *     GAUGE          [mu 4][site][row 3][col 3]  (four colour matrices)
 *   A propagator for smearing and contraction is 12 FERMION columns, column
 *   j = 3*spin_source + colour_source.
 * - Precisions: QDP_F64, QDP_F32, and QDP_F16S: IEEE half storage of every
 *   component with one FP32 scale per site record (one fermion column at a
 *   site, or one colour matrix of a site), scale = 2^e with e the binary
 *   exponent of the record's largest |component| (2^-126, the smallest normal
 *   FP32 power of two, for an all-zero record),
 *   stored value = round-to-nearest-even(v / scale).  Arithmetic on F16S
 *   fields is FP32.
 */
#ifndef QDPMI_H
#define QDPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qdp_ctx qdp_ctx;
typedef uint64_t qdp_field;   /* 0 is never a valid handle */
typedef uint64_t qdp_lattice; /* 0 is never a valid handle */
typedef int32_t qdp_status;

enum {
    QDP_OK = 0,
    QDP_ERR_ARG = -1,         /* bad argument (null pointer, size, range) */
    QDP_ERR_TYPE = -2,        /* lattice type mismatch / invalid expression */
    QDP_ERR_LATTICE = -3,     /* fields on different lattices / bad extents */
    QDP_ERR_NOMEM = -4,       /* pool and spill area cannot hold the fields */
    QDP_ERR_ALIAS = -5,       /* destination aliases a shifted operand */
    QDP_ERR_UNSUPPORTED = -6, /* valid request the library does not implement */
    QDP_ERR_HIP = -7,         /* HIP runtime error */
    QDP_ERR_STATE = -8        /* bad handle or context state */
};

enum qdp_type {
    QDP_REAL = 0,
    QDP_COMPLEX = 1,
    QDP_COLOR_VECTOR = 2,
    QDP_COLOR_MATRIX = 3,
    QDP_FERMION = 4,     /* spin 4 x colour 3 */
    QDP_SPIN_MATRIX = 5, /* 4 x 4 */
    QDP_PROPAGATOR = 6,  /* (4 x 4 spin) x (3 x 3 colour) */
    QDP_GAUGE = 7        /* four colour matrices U_mu, mu = 0..3 */
};

enum qdp_prec { QDP_F64 = 0, QDP_F32 = 1, QDP_F16S = 2 };

/* Site subsets for qdp_eval / qdp_shift.  Parity is (x + y + z + t) mod 2;
 * QDP_TIMESLICE selects the sites with time coordinate t. */
enum qdp_subset_kind { QDP_ALL = 0, QDP_EVEN = 1, QDP_ODD = 2, QDP_TIMESLICE = 3 };
typedef struct {
    int32_t kind;
    int32_t t;
} qdp_subset;

/* Sets for qdp_sum_multi: one subset, the two parities (even, odd), or the
 * Lt time slices in order. */
enum qdp_set_kind { QDP_SET_ALL = 0, QDP_SET_PARITY = 1, QDP_SET_TIMESLICE = 2 };

enum qdp_assign { QDP_ASSIGN = 0, QDP_ADD_ASSIGN = 1, QDP_SUB_ASSIGN = 2, QDP_MUL_ASSIGN = 3 };

enum qdp_smear_mode {
    QDP_SMEAR_FULL = 0,    /* every site updated in one launch per iteration
                              (tiles of the two parities interleaved) */
    QDP_SMEAR_EVEN_ODD = 1 /* two subset launches per iteration, even sites and
                              odd sites, both reading the previous iterate;
                              they depend on the previous iteration only, not
                              on each other, so they may overlap in time */
};

/* Flags for qdp_init_opts.flags. */
enum {
    QDP_INIT_NO_AUTOTUNE = 1u << 0,    /* use the default launch shapes */
    QDP_INIT_NO_GRAPH = 1u << 1,       /* launch smearing iterations one by one */
    QDP_INIT_FLAT_ADDRESSING = 1u << 2 /* 64-bit flat addresses in every kernel
                                          (the form fields of 4 GiB or more
                                          take; buffer addressing otherwise),
                                          so that form can be run at any size */
};

typedef struct {
    int32_t device;          /* HIP device ordinal */
    void* pool_ptr;          /* device memory for the pool, or NULL: the
                                library allocates pool_bytes itself */
    size_t pool_bytes;       /* pool size in bytes (> 0) */
    size_t host_spill_bytes; /* pinned host capacity for spilled fields
                                (0: no spilling, allocation fails instead) */
    void* hip_stream;        /* hipStream_t to order work on (NULL: null
                                stream) */
    uint32_t flags;          /* QDP_INIT_* */
} qdp_init_opts;

/* ---------------------------------------------------------------------- */
/* Context, lattices, fields                                               */
/* ---------------------------------------------------------------------- */

/* Create a context on opts->device.  Errors: QDP_ERR_ARG (null/zero sizes),
 * QDP_ERR_HIP (device or pool allocation failed).  *out is set only on
 * success. */
qdp_status qdp_init(const qdp_init_opts* opts, qdp_ctx** out);

/* Synchronise, free every field, lattice, graph and pinned buffer, and the
 * pool if the library allocated it.  The context pointer is invalid after. */
qdp_status qdp_finalize(qdp_ctx* ctx);

/* Register a lattice with extents dims = {Lx, Ly, Lz, Lt}, all even >= 2.
 * Errors: QDP_ERR_LATTICE. */
qdp_status qdp_lattice_create(qdp_ctx* ctx, const int32_t dims[4], qdp_lattice* out);

/* Allocate a device-resident field of the given qdp_type and qdp_prec.  The
 * contents are undefined until written.  May spill least-recently-used
 * fields to pinned host memory to make room (section 4.1).  Errors:
 * QDP_ERR_ARG, QDP_ERR_STATE (bad lattice), QDP_ERR_NOMEM. */
qdp_status qdp_field_alloc(qdp_ctx* ctx, qdp_lattice lat, int32_t type, int32_t prec,
                           qdp_field* out);

/* Release a field (its device block and any host copy).  Stream-ordered:
 * work already enqueued that reads the field still sees its data. */
qdp_status qdp_field_free(qdp_ctx* ctx, qdp_field f);

/* Number of doubles of the field in canonical host layout. */
qdp_status qdp_field_host_doubles(qdp_ctx* ctx, qdp_field f, size_t* n_doubles);

/* Copy a canonical host array (n_doubles must equal qdp_field_host_doubles)
 * into the field, converting to its precision and device layout.  REAL
 * fields take 1 double per site.  Errors: QDP_ERR_ARG on size mismatch. */
qdp_status qdp_field_write(qdp_ctx* ctx, qdp_field f, const double* host, size_t n_doubles);

/* Copy the field to a canonical host array (synchronises). */
qdp_status qdp_field_read(qdp_ctx* ctx, qdp_field f, double* host, size_t n_doubles);

/* Copy time slices t_begin .. t_end-1 of a field to a canonical host array
 * of the sub-lattice Lx x Ly x Lz x (t_end - t_begin) (same per-site layout
 * as qdp_field_read; for GAUGE the four directions of the sub-lattice one
 * after another).  Only the device tiles holding those slices are copied.
 * n_doubles must equal the sub-lattice's canonical size.  Synchronises.
 * Errors: QDP_ERR_ARG (range or size). */
qdp_status qdp_field_read_timeslices(qdp_ctx* ctx, qdp_field f, int32_t t_begin, int32_t t_end,
                                     double* host, size_t n_doubles);

/* Describe a field: type, precision, lattice, device bytes, residency
 * (1 = on device, 0 = spilled to host). */
typedef struct {
    int32_t type, prec;
    qdp_lattice lattice;
    uint64_t bytes;
    int32_t on_device;
    int32_t reserved;
} qdp_field_info_t;
qdp_status qdp_field_info(qdp_ctx* ctx, qdp_field f, qdp_field_info_t* out);

/* ---------------------------------------------------------------------- */
/* Expressions (section 4.2: one expression dest = expr over lattice       */
/* objects, evaluated site-parallel)                                       */
/* ---------------------------------------------------------------------- */

/* Postfix program.  Leaves push, operators pop (binary operators pop the
 * right operand first).  QDP++ semantics: a product multiplies spin parts
 * and colour parts as matrices; a scalar spin (colour) part acts as the
 * identity there. */
enum qdp_op {
    QDP_OP_FIELD = 0,         /* push field `field` (any non-GAUGE type) */
    QDP_OP_GAUGE = 1,         /* push colour matrix U_{i0} of GAUGE field */
    QDP_OP_REAL_CONST = 2,    /* push REAL constant re */
    QDP_OP_COMPLEX_CONST = 3, /* push COMPLEX constant (re, im) */
    QDP_OP_SHIFT = 4,         /* a(x + i1 * mu_hat), mu = i0, i1 = +1 / -1 */
    QDP_OP_NEG = 5,
    QDP_OP_CONJ = 6,          /* elementwise complex conjugate */
    QDP_OP_ADJ = 7,           /* conjugate transpose (square types) */
    QDP_OP_ADD = 8,
    QDP_OP_SUB = 9,
    QDP_OP_MUL = 10,
    QDP_OP_GAMMA_LEFT = 11,   /* Gamma_{i0} * a, a has a spin row index */
    QDP_OP_GAMMA_RIGHT = 12,  /* a * Gamma_{i0}, a has a spin column index */
    QDP_OP_TRACE = 13,        /* full trace -> COMPLEX (REAL for REAL) */
    QDP_OP_TRACE_COLOR = 14,  /* COLOR_MATRIX -> COMPLEX, PROPAGATOR -> SPIN_MATRIX */
    QDP_OP_TRACE_SPIN = 15,   /* SPIN_MATRIX -> COMPLEX, PROPAGATOR -> COLOR_MATRIX */
    QDP_OP_REAL = 16,         /* REAL/COMPLEX -> REAL */
    QDP_OP_IMAG = 17,
    QDP_OP_LOCAL_NORM2 = 18,  /* sum |a_k|^2 over the site's components -> REAL */
    QDP_OP_LOCAL_INNER = 19   /* sum conj(a_k) b_k -> COMPLEX */
};
/* Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 (b_k = bit k of n) in the DeGrand-Rossi
 * basis; Gamma_15 = gamma_5 = diag(1, 1, -1, -1). */

typedef struct {
    int32_t op;
    int32_t i0;
    int32_t i1;
    int32_t reserved;
    qdp_field field;
    double re;
    double im;
} qdp_node;

typedef struct {
    const qdp_node* nodes;
    int32_t n;
} qdp_expr;

/* dest op= expr on the sites of `subset`; other sites are untouched.
 * assign is a qdp_assign; MUL_ASSIGN means dest = dest * expr.  The result
 * type must equal dest's type (REAL may be assigned to COMPLEX).  Shifts are
 * pushed down to the leaves; the tree is matched against fused kernels
 * (linear stencils of colour-matrix x fermion/colour-vector terms) and
 * otherwise evaluated node by node with pool temporaries.  Errors:
 * QDP_ERR_TYPE, QDP_ERR_LATTICE, QDP_ERR_ALIAS (dest is a leaf read at a
 * shifted site), QDP_ERR_NOMEM. */
qdp_status qdp_eval(qdp_ctx* ctx, const qdp_expr* expr, qdp_field dest, qdp_subset subset,
                    int32_t assign);

/* dest(x) = src(x + sign * mu_hat) on the sites of subset (sign = +1 / -1).
 * Errors: as qdp_eval; dest == src gives QDP_ERR_ALIAS. */
qdp_status qdp_shift(qdp_ctx* ctx, qdp_field dest, qdp_field src, int32_t mu, int32_t sign,
                     qdp_subset subset);

/* Sum every component of expr over each subset of a set (qdp_set_kind):
 * out[(sub * ncomp + k) * 2 + {0, 1}] = (re, im) of the sum of component k,
 * ncomp = number of complex components of the expression's type.  The
 * expression is evaluated in FP64 and the sums are FP64 with a fixed
 * reduction order (bitwise repeatable).  n_doubles must be at least
 * nsub * ncomp * 2.  Synchronises. */
qdp_status qdp_sum_multi(qdp_ctx* ctx, const qdp_expr* expr, int32_t set, double* out,
                         size_t n_doubles);

/* ---------------------------------------------------------------------- */
/* Jacobi smearing (source and sink smearing, SRC and SNK of section 5)    */
/* ---------------------------------------------------------------------- */

/* psi <- (1 + kappa H)^n_iter psi on each column, in place, with
 *   (H psi)(x) = sum_{i != j_decay} U_i(x) psi(x + i) + U_i(x - i)^dagger psi(x - i)
 * acting on colour, identity on spin, no normalisation.  gauge is a GAUGE
 * field; cols are 1..12 FERMION fields of the same lattice and a precision
 * equal to the gauge's.  mode is a qdp_smear_mode (EVEN_ODD gives the same
 * result bitwise).  All columns are updated by one launch per pass, the
 * iterations are replayed from a cached HIP graph.  Errors: QDP_ERR_TYPE,
 * QDP_ERR_LATTICE, QDP_ERR_ARG (ncols, n_iter < 0), QDP_ERR_UNSUPPORTED
 * (j_decay != 3, mixed precisions), QDP_ERR_NOMEM. */
qdp_status qdp_smear_jacobi(qdp_ctx* ctx, qdp_field gauge, const qdp_field* cols, int32_t ncols,
                            double kappa, int32_t n_iter, int32_t j_decay, int32_t mode);

/* Out-of-place variant: dst[c] <- (1 + kappa H)^n_iter src[c]; src is not
 * modified (dst may equal src, which is the in-place call). */
qdp_status qdp_smear_jacobi_to(qdp_ctx* ctx, qdp_field gauge, const qdp_field* src,
                               const qdp_field* dst, int32_t ncols, double kappa, int32_t n_iter,
                               int32_t j_decay, int32_t mode);

/* Many independent lattices of any sizes smeared together: one persistent
 * launch per iteration covers every job (full-lattice passes).  Each job's
 * dst may equal its src.  Same per-site arithmetic as qdp_smear_jacobi, so
 * results are bitwise equal to smearing the jobs one by one. */
typedef struct {
    qdp_field gauge;
    const qdp_field* src;
    const qdp_field* dst;
    int32_t ncols;
    int32_t reserved;
} qdp_smear_job;
qdp_status qdp_smear_jacobi_batch(qdp_ctx* ctx, const qdp_smear_job* jobs, int32_t njobs,
                                  double kappa, int32_t n_iter);

/* ---------------------------------------------------------------------- */
/* Meson contractions (mesonic hadron spectrum, HAD of section 5)          */
/* ---------------------------------------------------------------------- */

/* C_n(t) = sum_{x: x_3 = t} Tr[ g5 S2(x)^dagger g5 Gamma_n S1(x) Gamma_n ]
 * for every n with bit n set in gamma_mask, zero momentum.  S1, S2: 12
 * FERMION columns each (S[(alpha a),(beta b)] = component (alpha, a) of
 * column 3*beta + b), same lattice; S2 may equal S1.  Per-site products and
 * all sums are FP64.  out has 16 * Lt * 2 doubles: out[(n * Lt + t') * 2 + k]
 * with t' = (t - t0) mod Lt; entries of n not in the mask are 0.
 * Synchronises.  Errors: QDP_ERR_TYPE, QDP_ERR_LATTICE,
 * QDP_ERR_UNSUPPORTED (j_decay != 3). */
qdp_status qdp_hadron_contract(qdp_ctx* ctx, const qdp_field* S1, const qdp_field* S2,
                               uint32_t gamma_mask, int32_t t0, int32_t j_decay, double* out);

/* qdp_hadron_contract without any allocation, for callers that cannot
 * allocate device or pinned memory during the call (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc).  Same
 * contraction, same kernels and bitwise the same values as
 * qdp_hadron_contract, but:
 * - out_dev is DEVICE memory (8-byte aligned) of 16 * Lt * 2 doubles in the
 *   layout of qdp_hadron_contract's out, written in order on the context
 *   stream; the call does not synchronise (read out_dev after qdp_sync or
 *   after work ordered behind the stream);
 * - the per-block partial sums go to a fixed 4 MiB device array of the
 *   library (one per GPU, held until the process ends) instead of a pool
 *   temporary: 256 * Lt * min(ceil(8192 / Lt), ceil(Lx Ly Lz / 64)) bytes,
 *   within the 4 MiB for every Lt <= 16384; larger needs give
 *   QDP_ERR_UNSUPPORTED;
 * - every column must be resident on the device (a spilled column gives
 *   QDP_ERR_STATE; the call never refills it).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams or other contexts) race.  Each call writes every
 * partial sum it reads, so none needs clearing.  Errors: as
 * qdp_hadron_contract; QDP_ERR_ARG (null or misaligned out_dev),
 * QDP_ERR_STATE (spilled column), QDP_ERR_UNSUPPORTED (scratch size). */
qdp_status qdp_hadron_contract_noalloc(qdp_ctx* ctx, const qdp_field* S1, const qdp_field* S2,
                                       uint32_t gamma_mask, int32_t t0, int32_t j_decay, double* out_dev);

/* Momentum-projected meson correlators (the hadron spectrum's plane-wave
 * projections, HAD of section 5):
 *   C_n(p, t) = sum_{x: x_3 = t} exp(-i p.x) Tr[ g5 S2^dagger g5 Gamma_n S1 Gamma_n ](x)
 * with p_i = 2 pi k_i / L_i and x = (x, y, z) the site's absolute spatial
 * coordinates.  moms: host array of nmom >= 1 integer triples (k_0, k_1,
 * k_2), any sign (taken modulo L_i).  The traces are formed as in
 * qdp_hadron_contract; the plane wave multiplies each site's FP64 traces
 * before the FP64 slice sums.  out: nmom * 16 * Lt * 2 doubles,
 * out[((q * 16 + n) * Lt + t') * 2 + k], momentum slowest; n outside the
 * mask gives 0.  Cost: one read of S1 and S2 per four momenta.
 * Synchronises.  Errors: as qdp_hadron_contract; QDP_ERR_ARG (nmom < 1,
 * null moms). */
qdp_status qdp_hadron_contract_mom(qdp_ctx* ctx, const qdp_field* S1, const qdp_field* S2,
                                   uint32_t gamma_mask, const int32_t* moms, int32_t nmom, int32_t t0,
                                   int32_t j_decay, double* out);

/* ---------------------------------------------------------------------- */
/* Baryon contractions (the baryon part of the hadron spectrum, HAD of     */
/* section 5)                                                              */
/* ---------------------------------------------------------------------- */

enum qdp_baryon_kind { QDP_BARYON_PROTON = 0, QDP_BARYON_DELTA_PP = 1 };

/* Baryon two-point functions with parity projection,
 *   C(t) = sum_{x: x_3 = t} sum_{g g'} P_{g'g} < chi_g(x) chibar_g'(0) >,
 *   P = (1 + parity gamma_4) / 2,  C = gamma_2 gamma_4 (DeGrand-Rossi),
 *   chibar = chi^dagger gamma_4, evaluated by Wick's theorem with no
 *   overall fermion sign:
 * - QDP_BARYON_PROTON: chi = eps_abc (u_a^T C g5 d_b) u_c with Su = <u ubar>
 *   and Sd = <d dbar> (Sd may equal Su): a direct and an exchange term;
 * - QDP_BARYON_DELTA_PP: chi^mu = eps_abc (u_a^T C gamma_mu u_b) u_c, summed
 *   over mu = 1, 2, 3 (no spin-3/2 projection), three u quarks: the
 *   determinant of the six pairings; Sd is not read (may be NULL).
 * Su, Sd: 12 FERMION columns each, the layout of qdp_hadron_contract.
 * Values are decoded to FP64; products and sums are FP64.  out: Lt * 2
 * doubles, out[t' * 2 + k] with t' = (t - t0) mod Lt.  Synchronises.
 * Errors: QDP_ERR_ARG (parity not +-1), QDP_ERR_UNSUPPORTED (kind,
 * j_decay != 3, mixed precisions), QDP_ERR_TYPE, QDP_ERR_LATTICE. */
qdp_status qdp_baryon_contract(qdp_ctx* ctx, const qdp_field* Su, const qdp_field* Sd, int32_t kind,
                               int32_t parity, int32_t t0, int32_t j_decay, double* out);

/* ---------------------------------------------------------------------- */
/* Field cache (section 4.1 and Figure 2)                                  */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint64_t hits;          /* operand uses that found the field on device */
    uint64_t misses;        /* operand uses that had to fill it from host */
    uint64_t spills;        /* device -> host evictions */
    uint64_t fills;         /* host -> device restores */
    uint64_t bytes_spilled;
    uint64_t bytes_filled;
    uint64_t pool_capacity; /* bytes */
    uint64_t pool_limit;    /* current usable bytes (qdp_set_pool_limit) */
    uint64_t pool_used;
    uint64_t pool_high_water;
    uint64_t host_used;     /* pinned spill bytes in use */
    uint64_t n_fields;
    uint64_t n_external;     /* live qdp_pool_malloc blocks */
    uint64_t external_bytes; /* their total size */
} qdp_cache_stats_t;

/* Fill *out (synchronises). */
qdp_status qdp_cache_stats(qdp_ctx* ctx, qdp_cache_stats_t* out);

/* Move one field to pinned host memory now (it is brought back on its next
 * use).  Errors: QDP_ERR_NOMEM (spill area full). */
qdp_status qdp_cache_evict(qdp_ctx* ctx, qdp_field f);

/* Evict every device-resident field. */
qdp_status qdp_cache_evict_all(qdp_ctx* ctx);

/* Restrict the pool to its first `bytes` bytes (<= capacity).  Fields above
 * the new limit are moved below it or spilled.  Errors: QDP_ERR_NOMEM. */
qdp_status qdp_set_pool_limit(qdp_ctx* ctx, size_t bytes);

/* Fail the n-th device pool allocation from now (n >= 1) with
 * QDP_ERR_NOMEM, once; 0 disarms.  For tests of the failure paths. */
qdp_status qdp_fault_alloc_after(qdp_ctx* ctx, int64_t n);

/* ---------------------------------------------------------------------- */
/* External allocations from the pool (QUDA-integration subsection and     */
/* Figure 2: a solver library's device allocations are redirected to the   */
/* pool manager, spilling LRU fields first when the pool is full, so that  */
/* the library and the fields share one pool)                              */
/* ---------------------------------------------------------------------- */

/* Allocate `bytes` (> 0) bytes of device memory from the pool: *out gets a
 * 256-byte aligned device pointer, contents undefined.  The block stays at
 * that address until qdp_pool_free (it is never spilled or moved, and
 * qdp_set_pool_limit below its end fails with QDP_ERR_STATE).  Making room
 * may spill least-recently-used unpinned fields to pinned host memory (the
 * copies are enqueued on the context stream).  The memory may still be read
 * or written by work queued on the context stream (a spill copy, a freed
 * field's last kernel): work on the context stream is ordered after it; a
 * caller touching the block from another stream calls qdp_sync first.
 * Errors: QDP_ERR_ARG (bytes 0, null out), QDP_ERR_NOMEM (no room even with
 * every field spilled; no allocation is made, *out untouched). */
qdp_status qdp_pool_malloc(qdp_ctx* ctx, size_t bytes, void** out);

/* Return a block of qdp_pool_malloc to the pool.  The block may be reused by
 * the next allocation, so work on other streams that touches it must have
 * finished (work on the context stream is ordered).  Errors: QDP_ERR_ARG (p
 * is not a live block of qdp_pool_malloc). */
qdp_status qdp_pool_free(qdp_ctx* ctx, void* p);

/* Wait for all work enqueued on the context's stream. */
qdp_status qdp_sync(qdp_ctx* ctx);

/* Message of the last failing call on ctx (never NULL; "" if none). */
const char* qdp_last_error(qdp_ctx* ctx);

/* ---------------------------------------------------------------------- */
/* Synthetic inputs on the device (benchmark and test workloads)           */
/* ---------------------------------------------------------------------- */

/* Counter-based generator Philox4x32-10 (Salmon et al., SC'11); complex
 * normal number e of stream sid under seed = Box-Muller of the block with
 * counter (e mod 2^32, e div 2^32, sid, 0), key (seed mod 2^32,
 * seed div 2^32), uniforms (k + 0.5) 2^-53 from 53-bit words.
 *   kind QDP_RANDOM_SU3: GAUGE field; element e = (mu V + s) 9 + 3 a + b of
 *     stream 1, Gram-Schmidt (two passes) on the columns, divided by the
 *     principal cube root of the determinant;
 *   kind QDP_RANDOM_GAUSSIAN: FERMION column `column`; element
 *     e = (column V + s) 12 + 3 spin + colour of stream 2, times `scale`.
 * s is the lexicographic site index.  Errors: QDP_ERR_TYPE. */
enum { QDP_RANDOM_SU3 = 0, QDP_RANDOM_GAUSSIAN = 1 };
qdp_status qdp_fill_random(qdp_ctx* ctx, qdp_field f, int32_t kind, uint64_t seed, int32_t column,
                           double scale);

/* Point source: zero the FERMION field, then set component (spin, colour) of
 * lexicographic site `site` to 1. */
qdp_status qdp_fill_point(qdp_ctx* ctx, qdp_field f, int64_t site, int32_t spin, int32_t colour);

/* ---------------------------------------------------------------------- */
/* Launch tuning                                                           */
/* ---------------------------------------------------------------------- */

/* Launch shape of the smearing kernel: sites per block = 64 * site_waves,
 * column groups = col_groups (each thread updates ceil(ncols / col_groups)
 * columns of one site), xcd = 1 maps consecutive blocks to one XCD, xcd =
 * 2 keeps each z-stack group of blocks on one XCD with the eight XCDs on
 * adjacent groups (z-stacked shapes; the multi-lattice kernel treats it as
 * 1),
 * waves_per_simd selects the kernel variant compiled for that occupancy
 * (0, 2 or 3; 0 = compiler default; FP64 always uses 0), flat = 1 uses
 * 64-bit flat addresses instead of buffer addressing (forced on when a field
 * is 4 GiB or larger), zstack = 1 gives the site_waves wavefronts of a
 * block 64-site tiles one (x, y) plane apart (the tiles of z-neighbouring
 * sites, so that the neighbour records they share are read by one CU;
 * single-lattice launches with site_waves > 1) instead of
 * consecutive tiles (zstack = 2: on whole-lattice updates with one column
 * group and an even site_waves, half of a block's waves take even tiles and
 * half the odd tiles with the same indices, z-stacked; elsewhere as 1; in
 * qdp_smear_jacobi_batch, zstack = 1 launches one block per work item
 * instead of the persistent grid that walks the item list),
 * lds = S (1 or 2; 0 = off) runs whole-lattice F16S updates
 * (QDP_SMEAR_FULL) with the kernel that stages each block's x/y neighbour
 * window in LDS, blocks of 2 S wavefronts updating 64 S checkerboard
 * indices of both parities (site_waves, col_groups and waves_per_simd do
 * not apply to it; zstack = 1 or 2 orders its blocks by two (three where two
 * do not fit) or four y bands of the (x, y) planes, one band over all planes
 * after the other, where Ly splits evenly and a band of a plane is a whole
 * number of blocks, else the plain order; other launches, flat addressing
 * and lattices with Lx > 64 ignore lds).
 * Every shape computes bitwise-identical results.
 * qdp_smear_set_shape forces a shape (site_waves = 0 returns to
 * autotuning); qdp_smear_get_shape reports the shape the last smearing call
 * used. */
typedef struct {
    int32_t site_waves;
    int32_t col_groups;
    int32_t xcd;
    int32_t waves_per_simd;
    int32_t flat;
    int32_t zstack;
    int32_t lds;
} qdp_launch_shape;
qdp_status qdp_smear_set_shape(qdp_ctx* ctx, const qdp_launch_shape* shape);
qdp_status qdp_smear_get_shape(qdp_ctx* ctx, qdp_launch_shape* out);

/* Device pointer and byte size of a field's storage (for profiling and
 * bandwidth accounting; the layout is internal). */
qdp_status qdp_field_device_ptr(qdp_ctx* ctx, qdp_field f, void** ptr, uint64_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* QDPMI_H */
