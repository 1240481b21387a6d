// Library-internal context, field and lattice records, and the helpers the
// translation units share.  Host code only.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "cache.hpp"
#include "common.hpp"

namespace qdpmi {

struct Lattice {
    Geometry geo;
};

struct Field {
    uint64_t id = 0;
    uint64_t lattice = 0;
    int32_t type = 0, prec = 0;
    int64_t bytes = 0;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

struct SmearTuneKey {
    int32_t L[4];
    int32_t ncols, prec, mode, batch;
    bool operator<(const SmearTuneKey& o) const;
};

struct Ctx;

// Mover over the context's pool and pinned spill area.
struct HipMover : Mover {
    Ctx* ctx = nullptr;
    bool host_area_ready() override;
    bool d2h(size_t dev_off, size_t host_off, size_t bytes) override;
    bool h2d(size_t host_off, size_t dev_off, size_t bytes) override;
    bool d2d(size_t src_off, size_t dst_off, size_t bytes) override;
};

struct Ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    int32_t num_cus = 256;

    char* pool_base = nullptr;
    size_t pool_bytes = 0;
    bool own_pool = false;
    char* host_base = nullptr;
    size_t host_bytes = 0;

    HipMover mover;
    FieldCache cache;
    std::unordered_map<uint64_t, Field> fields;
    std::unordered_map<uint64_t, Lattice> lattices;
    uint64_t next_id = 1;
    // qdp_pool_malloc blocks: device address -> cache entry id (pinned for life)
    std::unordered_map<uintptr_t, uint64_t> external;
    uint64_t external_bytes = 0;

    // small pinned buffer for results copied back to the host
    double* host_result = nullptr;
    size_t host_result_bytes = 0;

    // device address of this device's copy of the allocation-free
    // contraction's scratch array (looked up at qdp_init)
    void* noalloc_scratch = nullptr;

    // smearing: launch-shape tuning and graph cache
    std::map<SmearTuneKey, qdp_launch_shape> tuned;
    std::map<std::string, qdp_launch_shape> tuned_batch;  // keyed by precision, every lattice and column count
    qdp_launch_shape forced{0, 0, 0, 0, 0, 0, 0};
    qdp_launch_shape last_shape{0, 0, 0, 0, 0, 0, 0};
    std::map<std::string, GraphEntry> graphs;
    uint64_t graph_tick = 0;

    // gamma tables for the contraction kernels (host copy, built at init)
    struct GammaTables {
        int32_t group_perm[4][4];     // sigma -> permutation of spin indices
        int32_t group_members[4][4];  // sigma -> the 4 values of n
        double p_phase[16][4][2];     // s_a Gamma_n[a, sigma a]
        double q_phase[16][4][2];     // s_b Gamma_n[sigma b, b]
    } gamma;

    std::string last_error;
};

// Error helpers ----------------------------------------------------------

qdp_status set_error(Ctx* ctx, qdp_status code, const char* fmt, ...);
qdp_status hip_error(Ctx* ctx, hipError_t err, const char* what);

#define QDP_HIP(ctx, call)                                   \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return hip_error(ctx, _e, #call); \
    } while (0)

#define QDP_CHECK(call)                  \
    do {                                 \
        qdp_status _s = (call);          \
        if (_s != QDP_OK) return _s;     \
    } while (0)

// Handle lookups --------------------------------------------------------

Field* find_field(Ctx* ctx, uint64_t id);
Lattice* find_lattice(Ctx* ctx, uint64_t id);

// Pin a field on the device for one operation and return its storage.
// need_contents = false when the operation overwrites every byte.
qdp_status acquire_field(Ctx* ctx, uint64_t id, bool need_contents, char** ptr);
void release_field(Ctx* ctx, uint64_t id);

// Scoped pinning of several fields.
class PinSet {
public:
    explicit PinSet(Ctx* ctx) : ctx_(ctx) {}
    ~PinSet() {
        for (uint64_t id : ids_) release_field(ctx_, id);
    }
    qdp_status add(uint64_t id, bool need_contents, char** ptr) {
        qdp_status s = acquire_field(ctx_, id, need_contents, ptr);
        if (s == QDP_OK) ids_.push_back(id);
        return s;
    }

private:
    Ctx* ctx_;
    std::vector<uint64_t> ids_;
};

// Temporary device buffer from the pool, released at scope end
// (stream-ordered reuse is safe because all work is on one stream).
class PoolTemp {
public:
    PoolTemp() = default;
    ~PoolTemp();
    qdp_status alloc(Ctx* ctx, int64_t bytes);
    char* ptr() const { return ptr_; }

private:
    Ctx* ctx_ = nullptr;
    uint64_t id_ = 0;
    char* ptr_ = nullptr;
};

// Create / destroy a field record (also used for internal temporaries).
qdp_status field_create(Ctx* ctx, uint64_t lattice, int32_t type, int32_t prec, uint64_t* out);
qdp_status field_destroy(Ctx* ctx, uint64_t id);

// Pinned host buffer of at least `bytes` for results.
qdp_status host_result_buffer(Ctx* ctx, size_t bytes, double** out);

// Kernel launch error check.
qdp_status check_launch(Ctx* ctx, const char* what);

// Entry points implemented in the kernel translation units --------------

qdp_status smear_jacobi_impl(Ctx* ctx, uint64_t gauge, const uint64_t* src, const uint64_t* dst,
                             int32_t ncols, double kappa, int32_t n_iter, int32_t j_decay,
                             int32_t mode);
qdp_status smear_batch_impl(Ctx* ctx, const qdp_smear_job* jobs, int32_t njobs, double kappa,
                            int32_t n_iter);
qdp_status hadron_contract_impl(Ctx* ctx, const uint64_t* S1, const uint64_t* S2, uint32_t mask,
                                int32_t t0, int32_t j_decay, const int32_t* moms, int32_t nmom, double* out);
qdp_status hadron_contract_noalloc_impl(Ctx* ctx, const uint64_t* S1, const uint64_t* S2, uint32_t mask,
                                        int32_t t0, int32_t j_decay, double* out_dev);
qdp_status noalloc_scratch_init(Ctx* ctx);
qdp_status baryon_contract_impl(Ctx* ctx, const uint64_t* Su, const uint64_t* Sd, int32_t kind, int32_t parity,
                                int32_t t0, int32_t j_decay, double* out);
qdp_status eval_impl(Ctx* ctx, const qdp_expr* expr, uint64_t dest, qdp_subset subset,
                     int32_t assign);
qdp_status sum_multi_impl(Ctx* ctx, const qdp_expr* expr, int32_t set, double* out,
                          size_t n_doubles);
qdp_status fill_random_impl(Ctx* ctx, uint64_t f, int32_t kind, uint64_t seed, int32_t column,
                            double scale);
qdp_status fill_point_impl(Ctx* ctx, uint64_t f, int64_t site, int32_t spin, int32_t colour);
void build_gamma_tables(Ctx* ctx);
void release_graphs(Ctx* ctx);

}  // namespace qdpmi

struct qdp_ctx : qdpmi::Ctx {};
