// C ABI and host-side search driver.  Every arithmetic step of the method runs in the kernels of
// exact.hip and walk.hip; this file validates arguments, owns device buffers, launches kernels on
// the caller's stream and sequences the search (Sec. 3: depth loop, chunk loop, function
// versions, budgets from the Appendix's runtime law).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/tcw.h"
#include "common.h"
#include "internal.h"

namespace tcw {
// Depth-order network, weight gradient (mlp.hip): dW = H^T G (H: K x M, G: K x N, both bf16
// row-major; dW: M x N fp32) with the batch K split over workgroups when that fills the GPU better;
// `part` (mlp_dw_part_floats(M, N, K) floats, or null) holds the partial tiles, added in a fixed order.
size_t mlp_dw_part_floats(int M, int N, int K);
hipError_t mlp_gemm_dw(const void* H, const void* G, int M, int N, int K, float* dW, float* part, size_t part_floats,
                       hipStream_t s);
}  // namespace tcw

struct TunedCfg {
    int64_t walks = 0;
    int iters = 0;
    int log2_table = 0;
    double rate = 0;
};

namespace tcw {
// n = 4: rotated key vectors (SpaceDev::rkeys, rkeys2), shared by the spaces of one search seed.
struct RotKeys {
    uint64_t* t1 = nullptr;  // 1 MiB
    uint64_t* t2 = nullptr;  // 256 MiB, or null when the allocation failed
    ~RotKeys() {
        if (t1) (void)hipFree(t1);
        if (t2) (void)hipFree(t2);
    }
};
}  // namespace tcw

constexpr size_t ROT_KEYS_KEEP = 32;  // seeds whose n = 4 rotated keys (257 MiB each) a context keeps

struct tcw_ctx {
    std::map<uint64_t, TunedCfg> tuned;  // autotuner results by (n, k, delta)
    // n = 4 rotated keys by search seed, kept for later spaces of the same seed: freeing device
    // memory waits for the device, so a table lives until the context ends or until more than
    // ROT_KEYS_KEEP seeds are cached and it is the least recently used one no space holds
    struct RotEntry {
        std::shared_ptr<tcw::RotKeys> rk;
        uint64_t last = 0;
    };
    std::map<uint64_t, RotEntry> rot_keys;
    uint64_t rot_clock = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int* flag = nullptr;          // device scratch flag
    void* claw_scratch = nullptr;
    size_t claw_scratch_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct tcw_target {
    tcw_ctx* ctx = nullptr;
    int n = 0;
    tcw::ExactDev U;
};

namespace {

using tcw::ExactDev;
using tcw::SpaceDev;

int fail(tcw_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(tcw_ctx* c, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? TCW_ENOMEM : TCW_EDEVICE, m);
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

// Device buffers local to one call, freed when the call returns on any path (an early HIP_TRY
// return included).
class DevScope {
   public:
    DevScope() = default;
    DevScope(const DevScope&) = delete;
    DevScope& operator=(const DevScope&) = delete;
    ~DevScope() {
        for (void* q : bufs_) (void)hipFree(q);
    }
    template <typename T>
    hipError_t alloc(T** p, size_t bytes) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return e;
        bufs_.push_back(q);
        *p = static_cast<T*>(q);
        return hipSuccess;
    }

   private:
    std::vector<void*> bufs_;
};

uint32_t xi_of(int n) { return (1u << (2 * n)) - 1; }

// xi^h, or 0 if it does not fit in 32 bits
uint64_t n_half_of(int n, int h) {
    uint64_t v = 1;
    for (int i = 0; i < h; ++i) {
        v *= xi_of(n);
        if (v >= (1ull << 32)) return 0;
    }
    return v;
}

int clear_flag(tcw_ctx* c) {
    HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    return TCW_OK;
}

int read_flag(tcw_ctx* c, int* out) {
    HIP_TRY(c, hipMemcpyAsync(out, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

// A prepared search space: S_c on the device (exact and int8-packed), keys, salts.
struct Space {
    tcw_ctx* ctx = nullptr;
    int n = 0, k = 0, chunk = 0, delta = 0;
    uint64_t seed = 0;
    uint32_t version = 0;
    ExactDev S;
    int32_t e_s = 0;
    uint32_t* phi = nullptr;
    uint64_t* keys = nullptr;
    std::shared_ptr<tcw::RotKeys> rk;  // n = 4: rotated keys (SpaceDev::rkeys, rkeys2)
    SpaceDev dev{};

    ~Space() {
        tcw::exact_free(S);
        if (phi) (void)hipFree(phi);
        if (keys) (void)hipFree(keys);
    }

    void set_version(uint32_t v) {
        version = v;
        const uint64_t ctxi = ((uint64_t)v << 16) | ((uint64_t)k << 8) | (uint64_t)chunk;
        dev.salt_h = tcw::sm64(tcw::sm64(seed, 2), ctxi);
        dev.salt_d = tcw::sm64(tcw::sm64(seed, 3), ctxi);
        dev.salt_s = tcw::sm64(tcw::sm64(seed, 4), ctxi);
    }
};

int check_space(tcw_ctx* c, int n, const tcw_space* sp) {
    if (!sp) return fail(c, TCW_EINVAL, "space is NULL");
    if (sp->k < 1 || sp->k > TCW_MAX_T) return fail(c, TCW_EINVAL, "k must be in 1..64");
    if (sp->k % 2 == 1) {
        if (sp->chunk < 1 || (uint32_t)sp->chunk > xi_of(n)) return fail(c, TCW_EINVAL, "odd k needs chunk in 1..xi");
    } else if (sp->chunk != 0) {
        return fail(c, TCW_EINVAL, "even k needs chunk 0");
    }
    if (sp->delta < 0 || sp->delta > 32) return fail(c, TCW_EINVAL, "delta must be in 0..32");
    if (n_half_of(n, sp->k / 2) == 0) return fail(c, TCW_EINVAL, "xi^h must be below 2^32");
    if (sp->k > 255) return fail(c, TCW_EINVAL, "k too large");
    return TCW_OK;
}

int prepare_space(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, Space& out) {
    int rc = check_space(c, t->n, sp);
    if (rc) return rc;
    const int n = t->n;
    const int R = 1 << (2 * n);
    out.ctx = c;
    out.n = n;
    out.k = sp->k;
    out.chunk = sp->chunk;
    out.delta = sp->delta;
    out.seed = sp->seed;
    HIP_TRY(c, tcw::exact_alloc(out.S, n));
    HIP_TRY(c, hipMalloc(&out.phi, (size_t)R * R / 2 * sizeof(uint32_t) + 16));
    HIP_TRY(c, hipMalloc(&out.keys, (size_t)R * sizeof(uint64_t)));
    if ((rc = clear_flag(c))) return rc;
    // S_c = U R(c)^T for odd k, U for even k
    DevScope scope;
    uint16_t* seq = nullptr;
    uint8_t* tr = nullptr;
    int nseq = 0;
    if (sp->k % 2 == 1) {
        HIP_TRY(c, scope.alloc(&seq, sizeof(uint16_t)));
        HIP_TRY(c, scope.alloc(&tr, 1));
        const uint16_t cc = (uint16_t)sp->chunk;
        const uint8_t one = 1;
        HIP_TRY(c, hipMemcpyAsync(seq, &cc, sizeof(cc), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(tr, &one, 1, hipMemcpyHostToDevice, c->stream));
        nseq = 1;
    }
    hipError_t e = tcw::exact_apply(out.S, t->U, seq, tr, nseq, c->flag, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "chunk matrix");
    HIP_TRY(c, tcw::exact_pack_phi(out.S, out.phi, c->flag, c->stream));
    HIP_TRY(c, tcw::keys_fill(n, sp->seed, out.keys, c->stream));
    if (n == 4) {
        // the keys depend on the seed only: one set of rotated keys per seed, cached in the context
        auto it = c->rot_keys.find(sp->seed);
        if (it == c->rot_keys.end()) {
            while (c->rot_keys.size() >= ROT_KEYS_KEEP) {
                auto victim = c->rot_keys.end();
                for (auto e = c->rot_keys.begin(); e != c->rot_keys.end(); ++e) {
                    const bool unused = e->second.rk.use_count() == 1;
                    if (unused && (victim == c->rot_keys.end() || e->second.last < victim->second.last)) victim = e;
                }
                if (victim == c->rot_keys.end()) break;  // every cached table is in use
                c->rot_keys.erase(victim);
            }
            auto rk = std::make_shared<tcw::RotKeys>();
            HIP_TRY(c, hipMalloc(&rk->t1, (size_t)2 * 256 * 256 * sizeof(uint64_t)));
            HIP_TRY(c, tcw::rot_keys_fill(out.keys, rk->t1, c->stream));
            if (hipMalloc(&rk->t2, (size_t)2 * 256 * 256 * 256 * sizeof(uint64_t)) == hipSuccess) {
                HIP_TRY(c, tcw::rot_keys2_fill(rk->t1, rk->t2, c->stream));
            } else {
                rk->t2 = nullptr;  // without the 256 MiB table the step applies one more rotation
                (void)hipGetLastError();
            }
            it = c->rot_keys.emplace(sp->seed, tcw_ctx::RotEntry{rk, 0}).first;
        }
        it->second.last = ++c->rot_clock;
        out.rk = it->second.rk;
    }
    HIP_TRY(c, hipMemcpyAsync(&out.e_s, out.S.e, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    int flag = 0;
    if ((rc = read_flag(c, &flag))) return rc;
    if (flag & 4) return fail(c, TCW_EOVERFLOW, "exact value out of range while forming S_c");
    if (flag & 2) return fail(c, TCW_EOVERFLOW, "S_c entry outside int8 range (exponent too large)");
    const int h = sp->k / 2;
    out.dev.n_half = (uint32_t)n_half_of(n, h);
    out.dev.h = h;
    out.dev.delta = sp->delta;
    out.dev.rot_e = (int32_t)((30ll * out.e_s) % 61);
    out.dev.phi = out.phi;
    out.dev.keys = out.keys;
    out.dev.rkeys = out.rk ? out.rk->t1 : nullptr;
    out.dev.rkeys2 = out.rk ? out.rk->t2 : nullptr;
    out.set_version(sp->version);
    return TCW_OK;
}

int default_log2_table(int n) { return n <= 2 ? 12 : (n == 3 ? 20 : 26); }

// theta of a walk space when the caller leaves it open.  The time to a golden collision falls as
// theta rises for as long as memory holds the distinguished points (Sec. 5.1), so take the largest
// theta = 2^-delta, delta >= 1, whose 2 N theta distinguished points per function version fill at
// most a quarter of the table: 8 N <= 2^(log2_table + delta).
int auto_delta(uint64_t npts, int log2_table) {
    int d = 1;
    while (d < 30 && (npts << 3) > (1ull << (log2_table + d))) ++d;
    return d;
}
int default_iters(int n) { return n <= 2 ? 64 : (n == 3 ? 32 : 8); }

}  // namespace

// ---------------------------------------------------------------------------------------------
struct tcw_walk {
    tcw_ctx* ctx = nullptr;
    Space space;
    tcw::WalkDev wd{};
    bool ended = false;

    ~tcw_walk() {
        if (wd.states) (void)hipFree(wd.states);
        if (wd.table) (void)hipFree(wd.table);
        if (wd.stats) (void)hipFree(wd.stats);
        if (wd.claws) (void)hipFree(wd.claws);
        if (wd.claw_count) (void)hipFree(wd.claw_count);
    }
};

namespace {

int walk_restart(tcw_walk* w) {
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, tcw::launch_table_clear(w->wd.table, w->wd.log2_table, c->stream));
    HIP_TRY(c, hipMemsetAsync(w->wd.stats, 0, tcw::ST_COUNT * sizeof(unsigned long long), c->stream));
    HIP_TRY(c, hipMemsetAsync(w->wd.claw_count, 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(c, tcw::launch_walk_init(w->space.dev, w->wd, c->stream));
    return TCW_OK;
}

}  // namespace

extern "C" {

int tcw_create(tcw_ctx** out, int device, void* stream) {
    if (!out) return TCW_EINVAL;
    *out = nullptr;
    tcw_ctx* c = new (std::nothrow) tcw_ctx();
    if (!c) return TCW_ENOMEM;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete c;
        return TCW_EDEVICE;
    }
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->flag, sizeof(int)) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return TCW_EDEVICE;
    }
    *out = c;
    return TCW_OK;
}

int tcw_destroy(tcw_ctx* c) {
    if (!c) return TCW_EINVAL;
    if (c->flag) (void)hipFree(c->flag);
    if (c->claw_scratch) (void)hipFree(c->claw_scratch);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return TCW_OK;
}

const char* tcw_last_error(const tcw_ctx* c) { return c ? c->err.c_str() : "no context"; }

int tcw_set_stream(tcw_ctx* c, void* stream) {
    if (!c) return TCW_EINVAL;
    c->stream = (hipStream_t)stream;
    return TCW_OK;
}

int tcw_target_n(const tcw_target* t) { return t ? t->n : 0; }

int tcw_target_from_words(tcw_ctx* c, int n, const uint16_t* paulis, int k, const uint16_t* clifford, int m,
                          tcw_target** out) {
    if (!c || !out) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (k < 0 || m < 0 || (k > 0 && !paulis) || (m > 0 && !clifford)) return fail(c, TCW_EINVAL, "bad word arrays");
    const uint32_t xi = xi_of(n);
    // right-multiplication sequence: C_1 C_1 C_2 C_2 ... C_m C_m P_k ... P_1
    std::vector<uint16_t> seq;
    seq.reserve(2 * m + k);
    for (int j = 0; j < m; ++j) {
        if (clifford[j] < 1 || clifford[j] > xi) return fail(c, TCW_EINVAL, "Clifford Pauli out of range");
        seq.push_back(clifford[j]);
        seq.push_back(clifford[j]);
    }
    for (int j = k - 1; j >= 0; --j) {
        if (paulis[j] < 1 || paulis[j] > xi) return fail(c, TCW_EINVAL, "Pauli out of range");
        seq.push_back(paulis[j]);
    }
    tcw_target* t = new (std::nothrow) tcw_target();
    if (!t) return TCW_ENOMEM;
    t->ctx = c;
    t->n = n;
    hipError_t e = tcw::exact_alloc(t->U, n);
    uint16_t* seq_dev = nullptr;
    if (e == hipSuccess && !seq.empty()) e = hipMalloc(&seq_dev, seq.size() * sizeof(uint16_t));
    if (e == hipSuccess && !seq.empty())
        e = hipMemcpyAsync(seq_dev, seq.data(), seq.size() * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = tcw::exact_build(t->U, seq_dev, nullptr, (int)seq.size(), c->flag, c->stream);
    if (seq_dev) (void)hipFree(seq_dev);
    if (e != hipSuccess) {
        tcw::exact_free(t->U);
        delete t;
        return hip_fail(c, e, "target build");
    }
    int flag = 0;
    int rc = read_flag(c, &flag);
    if (rc == TCW_OK && flag) rc = fail(c, TCW_EOVERFLOW, "exact value out of range while building the target");
    if (rc) {
        tcw::exact_free(t->U);
        delete t;
        return rc;
    }
    *out = t;
    return TCW_OK;
}

int tcw_target_from_channel(tcw_ctx* c, int n, const int32_t* a, const int32_t* b, int32_t e0, tcw_target** out) {
    if (!c || !out || !a || !b) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (e0 < 0 || e0 > 60) return fail(c, TCW_EINVAL, "exponent must be in 0..60");
    const size_t rr = (size_t)1 << (4 * n);
    tcw_target* t = new (std::nothrow) tcw_target();
    if (!t) return TCW_ENOMEM;
    t->ctx = c;
    t->n = n;
    int32_t *da = nullptr, *db = nullptr;
    hipError_t e = tcw::exact_alloc(t->U, n);
    if (e == hipSuccess) e = hipMalloc(&da, rr * 4);
    if (e == hipSuccess) e = hipMalloc(&db, rr * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(da, a, rr * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(db, b, rr * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = tcw::exact_from_i32(t->U, da, db, e0, c->flag, c->stream);
    if (e == hipSuccess) e = tcw::exact_check_orthogonal(t->U, c->flag, c->stream);
    int flag = 0;
    int rc = TCW_OK;
    if (e == hipSuccess) {
        rc = read_flag(c, &flag);
    } else {
        rc = hip_fail(c, e, "target upload");
    }
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (rc == TCW_OK && (flag & 4)) rc = fail(c, TCW_EOVERFLOW, "entries too large");
    if (rc == TCW_OK && (flag & 1)) rc = fail(c, TCW_EINVAL, "matrix is not orthogonal (X X^T != 2^e I)");
    if (rc) {
        tcw::exact_free(t->U);
        delete t;
        return rc;
    }
    *out = t;
    return TCW_OK;
}

int tcw_target_from_unitary(tcw_ctx* c, int n, const int64_t* v, int32_t e, tcw_target** out) {
    if (!c || !out || !v) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (e < 0 || n + e > 29) return fail(c, TCW_EINVAL, "need 0 <= e and n + e <= 29");
    const size_t d = (size_t)1 << n, rr = (size_t)1 << (4 * n);
    for (size_t x = 0; x < d * d * 4; ++x)
        if (v[x] > (1 << 20) || v[x] < -(1 << 20)) return fail(c, TCW_EINVAL, "coefficients must lie in [-2^20, 2^20]");
    tcw_target* t = new (std::nothrow) tcw_target();
    if (!t) return TCW_ENOMEM;
    t->ctx = c;
    t->n = n;
    int64_t* dv = nullptr;
    int32_t *da = nullptr, *db = nullptr;
    hipError_t err = tcw::exact_alloc(t->U, n);
    if (err == hipSuccess) err = hipMalloc(&dv, d * d * 4 * sizeof(int64_t));
    if (err == hipSuccess) err = hipMalloc(&da, rr * 4);
    if (err == hipSuccess) err = hipMalloc(&db, rr * 4);
    if (err == hipSuccess) err = hipMemcpyAsync(dv, v, d * d * 4 * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
    if (err == hipSuccess) err = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (err == hipSuccess) err = tcw::exact_from_unitary(t->U, dv, e, da, db, c->flag, c->stream);
    int flag = 0;
    int rc = TCW_OK;
    // the orthogonality check only runs on values that passed the unitary and range checks
    if (err == hipSuccess) rc = read_flag(c, &flag);
    else rc = hip_fail(c, err, "unitary upload");
    if (rc == TCW_OK && flag == 0) {
        err = tcw::exact_check_orthogonal(t->U, c->flag, c->stream);
        if (err == hipSuccess) rc = read_flag(c, &flag);
        else rc = hip_fail(c, err, "orthogonality check");
    }
    if (dv) (void)hipFree(dv);
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (rc == TCW_OK && (flag & 8)) rc = fail(c, TCW_EINVAL, "U is not unitary (V V^dag != 2^e I)");
    if (rc == TCW_OK && (flag & 1)) rc = fail(c, TCW_EINVAL, "channel rep is not real orthogonal");
    if (rc == TCW_OK && (flag & 4)) rc = fail(c, TCW_EOVERFLOW, "channel rep entry out of range");
    if (rc) {
        tcw::exact_free(t->U);
        delete t;
        return rc;
    }
    *out = t;
    return TCW_OK;
}

int tcw_target_free(tcw_target* t) {
    if (!t) return TCW_EINVAL;
    tcw::exact_free(t->U);
    delete t;
    return TCW_OK;
}

int tcw_target_channel(tcw_ctx* c, const tcw_target* t, int32_t* a, int32_t* b, int32_t* e) {
    if (!c || !t || !a || !b || !e) return TCW_EINVAL;
    const size_t rr = (size_t)1 << (4 * t->n);
    int32_t *da = nullptr, *db = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&da, rr * 4));
    HIP_TRY(c, scope.alloc(&db, rr * 4));
    int rc = clear_flag(c);
    if (!rc) {
        hipError_t err = tcw::exact_to_i32(t->U, da, db, c->flag, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(a, da, rr * 4, hipMemcpyDeviceToHost, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(b, db, rr * 4, hipMemcpyDeviceToHost, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(e, t->U.e, 4, hipMemcpyDeviceToHost, c->stream);
        if (err != hipSuccess) rc = hip_fail(c, err, "target copy");
    }
    int flag = 0;
    if (!rc) rc = read_flag(c, &flag);
    if (!rc && flag) rc = fail(c, TCW_EOVERFLOW, "entry does not fit int32");
    return rc;
}

int tcw_step(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* in, uint64_t* out, uint64_t* hash,
             int64_t count) {
    if (!c || !t || count < 0 || (count > 0 && (!in || !out))) return TCW_EINVAL;
    if (count == 0) return check_space(c, t->n, sp);
    Space s;
    int rc = prepare_space(c, t, sp, s);
    if (rc) return rc;
    HIP_TRY(c, tcw::launch_step(t->n, s.dev, in, out, hash, count, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_trails(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* starts, int64_t count,
               uint32_t cap, uint64_t* dp, uint32_t* len) {
    if (!c || !t || count < 0 || cap == 0 || (count > 0 && (!starts || !dp || !len))) return TCW_EINVAL;
    if (count == 0) return check_space(c, t->n, sp);
    Space s;
    int rc = prepare_space(c, t, sp, s);
    if (rc) return rc;
    HIP_TRY(c, tcw::launch_trails(t->n, s.dev, starts, count, cap, dp, len, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_start_points(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, int64_t w0, uint32_t j, int64_t count,
                     uint64_t* out) {
    if (!c || !t || count < 0 || (count > 0 && !out) || w0 < 0 || w0 + count > (1ll << 32)) return TCW_EINVAL;
    int rc = check_space(c, t->n, sp);
    if (rc || count == 0) return rc;
    Space s;
    s.k = sp->k;
    s.chunk = sp->chunk;
    s.seed = sp->seed;
    s.dev.n_half = (uint32_t)n_half_of(t->n, sp->k / 2);
    s.set_version(sp->version);
    HIP_TRY(c, tcw::launch_starts(s.dev, w0, j, count, out, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_canon_hash(tcw_ctx* c, int n, const tcw_space* sp, const int32_t* a, const int32_t* b, const int32_t* e,
                   int64_t count, uint64_t* h_out) {
    if (!c || !sp || count < 0 || (count > 0 && (!a || !b || !e || !h_out))) return TCW_EINVAL;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (count == 0) return TCW_OK;
    const int R = 1 << (2 * n);
    if (count > (int64_t)1 << 31) return fail(c, TCW_EINVAL, "count above 2^31");  // keeps the byte count exact
    uint32_t* phi = nullptr;
    uint64_t* keys = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&phi, (size_t)count * R * R / 2 * sizeof(uint32_t)));
    HIP_TRY(c, scope.alloc(&keys, (size_t)R * sizeof(uint64_t)));
    int rc = clear_flag(c);
    Space s;
    s.k = sp->k;
    s.chunk = sp->chunk;
    s.seed = sp->seed;
    s.dev.keys = keys;
    s.dev.delta = sp->delta;
    s.set_version(sp->version);
    hipError_t err = hipSuccess;
    if (!rc) err = tcw::pack_phi_i32(n, a, b, count, phi, c->flag, c->stream);
    if (!rc && err == hipSuccess) err = tcw::keys_fill(n, sp->seed, keys, c->stream);
    int flag = 0;
    if (!rc && err == hipSuccess) rc = read_flag(c, &flag);
    if (!rc && err == hipSuccess && flag) rc = fail(c, TCW_EOVERFLOW, "matrix entry outside int8 range");
    if (!rc && err == hipSuccess) err = tcw::launch_canon_hash(n, s.dev, phi, e, count, h_out, c->stream);
    if (!rc && err == hipSuccess) err = hipStreamSynchronize(c->stream);
    if (!rc && err != hipSuccess) rc = hip_fail(c, err, "canon hash");
    return rc;
}

int tcw_claw_check(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* u0, const uint64_t* u1,
                   int64_t count, int32_t* ok, int32_t* perm, int8_t* sign) {
    if (!c || !t || count < 0 || (count > 0 && (!u0 || !u1 || !ok || !perm || !sign))) return TCW_EINVAL;
    if (count == 0) return check_space(c, t->n, sp);
    Space s;
    int rc = prepare_space(c, t, sp, s);
    if (rc) return rc;
    const size_t need = tcw::exact_claw_scratch_bytes(t->n);
    if (c->claw_scratch_bytes < need) {
        if (c->claw_scratch) (void)hipFree(c->claw_scratch);
        c->claw_scratch = nullptr;
        c->claw_scratch_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->claw_scratch, need));
        c->claw_scratch_bytes = need;
    }
    HIP_TRY(c, tcw::exact_claw_check(s.S, sp->k, u0, u1, count, c->claw_scratch, c->claw_scratch_bytes, ok, perm,
                                     sign, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

// ---- walk sessions ----
int tcw_walk_begin(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, int64_t walks, int log2_table, uint32_t cap,
                   int enumerate, tcw_walk** out) {
    if (!c || !t || !out) return TCW_EINVAL;
    *out = nullptr;
    if (walks < 1 || walks > (1ll << 31)) return fail(c, TCW_EINVAL, "walks must be in 1..2^31");
    if (log2_table < 4 || log2_table > 32) return fail(c, TCW_EINVAL, "log2_table must be in 4..32");
    if (cap == 0) return fail(c, TCW_EINVAL, "cap must be positive");
    tcw_walk* w = new (std::nothrow) tcw_walk();
    if (!w) return TCW_ENOMEM;
    w->ctx = c;
    int rc = prepare_space(c, t, sp, w->space);
    if (rc) {
        delete w;
        return rc;
    }
    tcw::WalkDev& wd = w->wd;
    wd.walks = walks;
    wd.log2_table = log2_table;
    wd.cap = cap;
    wd.enumerate = enumerate ? 1 : 0;
    wd.n_points = 2ull * w->space.dev.n_half;
    wd.claw_cap = 4096;
    hipError_t e = hipMalloc(&wd.states, (size_t)walks * sizeof(tcw::WalkState));
    if (e == hipSuccess) e = hipMalloc(&wd.table, ((size_t)1 << log2_table) * 16);
    if (e == hipSuccess) e = hipMalloc(&wd.stats, tcw::ST_COUNT * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&wd.claws, (size_t)wd.claw_cap * 16);
    if (e == hipSuccess) e = hipMalloc(&wd.claw_count, sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete w;
        return hip_fail(c, e, "walk session allocation");
    }
    rc = walk_restart(w);
    if (rc) {
        delete w;
        return rc;
    }
    *out = w;
    return TCW_OK;
}

int tcw_walk_run(tcw_walk* w, int iters) {
    if (!w || iters < 1) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    if (w->ended) return fail(c, TCW_ESTATE, "walk session ended");
    HIP_TRY(c, hipMemsetAsync(&w->wd.stats[tcw::ST_ACTIVE], 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    HIP_TRY(c, tcw::launch_walk(w->space.n, w->space.dev, w->wd, iters, tcw::walk_grid_blocks(w->space.n, c->device),
                                c->stream));
    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    return TCW_OK;
}

int tcw_walk_stats_get(tcw_walk* w, tcw_walk_stats* out) {
    if (!w || !out) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    unsigned long long v[tcw::ST_COUNT];
    HIP_TRY(c, hipMemcpyAsync(v, w->wd.stats, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out->steps = (int64_t)v[tcw::ST_STEPS];
    out->dps = (int64_t)v[tcw::ST_DPS];
    out->inserts = (int64_t)v[tcw::ST_INSERTS];
    out->abandoned = (int64_t)v[tcw::ST_ABANDONED];
    out->robin_hood = (int64_t)v[tcw::ST_ROBIN];
    out->same_side = (int64_t)v[tcw::ST_SAME];
    out->reduction = (int64_t)v[tcw::ST_REDUCTION];
    out->claws = (int64_t)v[tcw::ST_CLAWS];
    out->table_full = (int64_t)v[tcw::ST_FULL];
    out->spin_timeouts = (int64_t)v[tcw::ST_SPIN];
    out->active_walks = (int64_t)v[tcw::ST_ACTIVE];
    return TCW_OK;
}

int tcw_walk_claws(tcw_walk* w, uint64_t* u0, uint64_t* u1, int64_t max_pairs, int64_t* total) {
    if (!w || !total || max_pairs < 0 || (max_pairs > 0 && (!u0 || !u1))) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    unsigned long long cnt = 0;
    HIP_TRY(c, hipMemcpyAsync(&cnt, w->wd.claw_count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *total = (int64_t)cnt;
    int64_t avail = (int64_t)(cnt < w->wd.claw_cap ? cnt : w->wd.claw_cap);
    int64_t m = avail < max_pairs ? avail : max_pairs;
    if (m > 0) {
        std::vector<uint64_t> buf(2 * m);
        HIP_TRY(c, hipMemcpyAsync(buf.data(), w->wd.claws, 16 * m, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < m; ++i) {
            u0[i] = buf[2 * i];
            u1[i] = buf[2 * i + 1];
        }
    }
    return TCW_OK;
}

int tcw_walk_reset(tcw_walk* w, uint32_t version) {
    if (!w) return TCW_EINVAL;
    w->space.set_version(version);
    return walk_restart(w);
}

int tcw_walk_last_ms(tcw_walk* w, float* ms) {
    if (!w || !ms) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipEventSynchronize(c->ev1));
    HIP_TRY(c, hipEventElapsedTime(ms, c->ev0, c->ev1));
    return TCW_OK;
}

int tcw_walk_read_states(tcw_walk* w, int64_t first, int64_t count, void* host_out) {
    if (!w || !host_out || first < 0 || count < 0 || first + count > w->wd.walks) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(host_out, w->wd.states + first, (size_t)count * sizeof(tcw::WalkState),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_write_states(tcw_walk* w, int64_t first, int64_t count, const void* host_in) {
    if (!w || !host_in || first < 0 || count < 0 || first + count > w->wd.walks) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(w->wd.states + first, host_in, (size_t)count * sizeof(tcw::WalkState),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_read_table(tcw_walk* w, void* host_out) {
    if (!w || !host_out) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(host_out, w->wd.table, ((size_t)1 << w->wd.log2_table) * 16, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_write_table(tcw_walk* w, const void* host_in) {
    if (!w || !host_in) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(w->wd.table, host_in, ((size_t)1 << w->wd.log2_table) * 16, hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_end(tcw_walk* w) {
    if (!w) return TCW_EINVAL;
    (void)hipStreamSynchronize(w->ctx->stream);
    delete w;
    return TCW_OK;
}

// ---- search driver ----
void tcw_default_params(tcw_walk_params* p, int n) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->k_max = 7;
    p->delta = -1;
    p->walks = n <= 2 ? 64 : (n == 3 ? (1 << 16) : (1 << 20));
    p->log2_table = default_log2_table(n);
    p->seed = 1;
    p->version = 0;
    p->trail_cap_factor = 20;
    p->budget_beta = 16;
    p->version_factor = 2;
    p->enum_max = 1 << 16;
    p->iters_per_launch = 0;
    p->depth_order_kind = TCW_ORDER_PLAIN;
    p->chunk_first = 0;
    p->chunk_last = 0;
    p->max_seconds = 0.0;
    p->chunk_parallel = 1;
}

}  // extern "C"

namespace {

void decode_desc(uint64_t pt, int n, int h, std::vector<uint16_t>& out) {
    uint32_t x = (uint32_t)pt;
    const uint32_t xi = xi_of(n);
    for (int t = 0; t < h; ++t) {
        out.push_back((uint16_t)(x % xi + 1));
        x /= xi;
    }
}

void add_stats(tcw_walk_stats& a, const tcw_walk_stats& b) {
    a.steps += b.steps;
    a.dps += b.dps;
    a.inserts += b.inserts;
    a.abandoned += b.abandoned;
    a.robin_hood += b.robin_hood;
    a.same_side += b.same_side;
    a.reduction += b.reduction;
    a.claws += b.claws;
    a.table_full += b.table_full;
    a.spin_timeouts += b.spin_timeouts;
}

// Exact check of claw candidate pairs (host arrays) of a space: the first that passes fills res.
int check_pairs(tcw_ctx* c, const Space& sp, const uint64_t* u0, const uint64_t* u1, int64_t m, tcw_result* res,
                int* found) {
    *found = 0;
    if (m <= 0) return TCW_OK;
    const int n = sp.n;
    const int R = 1 << (2 * n);
    uint64_t *d0 = nullptr, *d1 = nullptr;
    int32_t *dok = nullptr, *dperm = nullptr;
    int8_t* dsign = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&d0, m * 8));
    HIP_TRY(c, scope.alloc(&d1, m * 8));
    HIP_TRY(c, scope.alloc(&dok, m * 4));
    HIP_TRY(c, scope.alloc(&dperm, m * R * 4));
    HIP_TRY(c, scope.alloc(&dsign, m * R));
    HIP_TRY(c, hipMemcpyAsync(d0, u0, m * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d1, u1, m * 8, hipMemcpyHostToDevice, c->stream));
    const size_t need = tcw::exact_claw_scratch_bytes(n);
    if (c->claw_scratch_bytes < need) {
        if (c->claw_scratch) (void)hipFree(c->claw_scratch);
        c->claw_scratch = nullptr;
        c->claw_scratch_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->claw_scratch, need));
        c->claw_scratch_bytes = need;
    }
    HIP_TRY(c, tcw::exact_claw_check(sp.S, sp.k, d0, d1, m, c->claw_scratch, c->claw_scratch_bytes, dok, dperm, dsign,
                                     c->stream));
    std::vector<int32_t> ok(m), perm(m * R);
    std::vector<int8_t> sign(m * R);
    HIP_TRY(c, hipMemcpyAsync(ok.data(), dok, m * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(perm.data(), dperm, m * R * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sign.data(), dsign, m * R, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < m; ++i) {
        if (!ok[i]) {
            res->false_claws++;
            continue;
        }
        uint64_t pv = u0[i], pw = u1[i];
        if ((pv >> 32) & 1) std::swap(pv, pw);
        const int h = sp.k / 2;
        std::vector<uint16_t> dv, dw, desc;
        decode_desc(pv, n, h, dv);
        decode_desc(pw, n, h, dw);
        desc = dv;
        for (int t = h - 1; t >= 0; --t) desc.push_back(dw[t]);
        if (sp.k % 2) desc.push_back((uint16_t)sp.chunk);
        res->status = 1;
        res->t = sp.k;
        res->chunk = sp.chunk;
        for (size_t j = 0; j < desc.size() && j < TCW_MAX_T; ++j) res->paulis[j] = desc[j];
        for (int q = 0; q < R; ++q) {
            res->clifford_perm[q] = perm[i * R + q];
            res->clifford_sign[q] = sign[i * R + q];
        }
        *found = 1;
        break;
    }
    return TCW_OK;
}

// New claw candidates of a walk session; `seen` counts those already checked.
int check_claws(tcw_ctx* c, tcw_walk* w, int64_t& seen, tcw_result* res, int* found) {
    *found = 0;
    int64_t total = 0;
    std::vector<uint64_t> u0(4096), u1(4096);
    int rc = tcw_walk_claws(w, u0.data(), u1.data(), 4096, &total);
    if (rc) return rc;
    const int64_t avail = total < 4096 ? total : 4096;
    if (avail <= seen) return TCW_OK;
    rc = check_pairs(c, w->space, u0.data() + seen, u1.data() + seen, avail - seen, res, found);
    seen = avail;
    return rc;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int depth_order_of(tcw_ctx* c, const tcw_walk_params* p, std::vector<int>& order) {
    order.clear();
    if (p->k_max < 0 || p->k_max > TCW_MAX_T) return fail(c, TCW_EINVAL, "k_max out of range");
    if (p->depth_order_kind == TCW_ORDER_GIVEN) {
        if (p->depth_order_len < 0 || p->depth_order_len > 16) return fail(c, TCW_EINVAL, "bad depth order");
        for (int i = 0; i < p->depth_order_len; ++i) {
            const int k = p->depth_order[i];
            if (k < 0 || k > p->k_max) return fail(c, TCW_EINVAL, "depth order entry out of range");
            bool dup = false;
            for (int o : order) dup |= (o == k);
            if (!dup) order.push_back(k);
        }
    }
    // the plain increasing order is the fallback for depths the given order left out
    for (int k = 0; k <= p->k_max; ++k) {
        bool have = false;
        for (int o : order) have |= (o == k);
        if (!have) order.push_back(k);
    }
    return TCW_OK;
}

// Depth 0: is U_hat itself a signed permutation (a Clifford)?
int search_k0(tcw_ctx* c, const tcw_target* t, tcw_result* res, int* found) {
    const int R = 1 << (2 * t->n);
    *found = 0;
    int32_t *dok = nullptr, *dperm = nullptr;
    int8_t* dsign = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&dok, 4));
    HIP_TRY(c, scope.alloc(&dperm, R * 4));
    HIP_TRY(c, scope.alloc(&dsign, R));
    HIP_TRY(c, tcw::exact_signed_perm(t->U, dok, dperm, dsign, c->stream));
    int32_t ok = 0;
    std::vector<int32_t> perm(R);
    std::vector<int8_t> sign(R);
    HIP_TRY(c, hipMemcpyAsync(&ok, dok, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(perm.data(), dperm, R * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sign.data(), dsign, R, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    res->spaces++;
    if (ok) {
        res->status = 1;
        res->t = 0;
        for (int q = 0; q < R; ++q) {
            res->clifford_perm[q] = perm[q];
            res->clifford_sign[q] = sign[q];
        }
        *found = 1;
    }
    return TCW_OK;
}

// A small space: every point once, keyed by the full matrix hash.
int search_enum(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, int k, int chunk, int iters,
                tcw_result* res, int* found, double t0) {
    *found = 0;
    const uint64_t npts = 2 * n_half_of(t->n, k / 2);
    tcw_space sp{k, chunk, p->seed, p->version, 0};
    res->spaces++;
    res->versions++;
    int64_t walks = (int64_t)npts < p->walks ? (int64_t)npts : p->walks;
    if (walks < 64) walks = (int64_t)npts < 64 ? (int64_t)npts : 64;
    int lg = 4;
    while ((1ull << lg) < 4 * npts && lg < 30) ++lg;
    tcw_walk* w = nullptr;
    int rc = tcw_walk_begin(c, t, &sp, walks, lg, 2, 1, &w);
    if (rc) return rc;
    int64_t seen = 0;
    // each point costs one evaluation; a bounded number of launches covers them all
    const int64_t max_launches = (int64_t)(npts / (uint64_t)walks + 2) / iters + 4;
    for (int64_t launch = 0;; ++launch) {
        rc = tcw_walk_run(w, iters);
        res->launches++;
        tcw_walk_stats st{};
        if (!rc) rc = tcw_walk_stats_get(w, &st);
        if (!rc) rc = check_claws(c, w, seen, res, found);
        if (rc) {
            tcw_walk_end(w);
            return rc;
        }
        if (*found || st.active_walks == 0 || launch >= max_launches ||
            (p->max_seconds > 0 && now_s() - t0 > p->max_seconds)) {
            add_stats(res->stats, st);
            break;
        }
    }
    tcw_walk_end(w);
    return TCW_OK;
}

// Steps per function version: max(factor * N, 2 walks / theta), but no more than the table holds
// at half load (slots / 2 distinguished points, i.e. slots / (2 theta) steps).
// Ranges of the search parameters, checked before any of them enters a shift or a launch.  In a
// batch, walks and log2_table <= 0 take the autotuner's choice.
int check_params(tcw_ctx* c, const tcw_walk_params* p, int n, bool batch) {
    if (p->delta > 32) return fail(c, TCW_EINVAL, "delta must be at most 32 (negative: automatic)");
    if ((!batch && p->walks < 1) || p->walks > (1ll << 31)) return fail(c, TCW_EINVAL, "walks must be in 1..2^31");
    if ((!batch || p->log2_table > 0) && (p->log2_table < 4 || p->log2_table > 32))
        return fail(c, TCW_EINVAL, "log2_table must be in 4..32");
    if (p->trail_cap_factor < 1 || p->budget_beta < 1 || p->version_factor < 1)
        return fail(c, TCW_EINVAL, "trail_cap_factor, budget_beta and version_factor must be positive");
    if (p->enum_max < 0) return fail(c, TCW_EINVAL, "enum_max must be non-negative");
    const int32_t xi = (int32_t)xi_of(n);
    if (p->chunk_first < 0 || p->chunk_first > xi || p->chunk_last < 0 || p->chunk_last > xi)
        return fail(c, TCW_EINVAL, "chunk_first and chunk_last must lie in 1..xi (0: default)");
    if (!(p->max_seconds >= 0)) return fail(c, TCW_EINVAL, "max_seconds must be non-negative");
    return TCW_OK;
}

uint64_t version_steps(const tcw_walk_params* p, uint64_t npts, int delta, int64_t walks, int log2_table) {
    uint64_t per_version = (uint64_t)p->version_factor * npts;
    const uint64_t floor_v = 2ull * (uint64_t)walks << delta;
    if (per_version < floor_v) per_version = floor_v;
    const uint64_t table_v = (1ull << (log2_table - 1)) << delta;
    return per_version < table_v ? per_version : table_v;
}

// the tables of one group of concurrently searched chunks stay within 2^35 bytes (32 GiB)
constexpr int CHUNK_TABLE_POOL_LOG2 = 35;

struct BatchTarget;
int search_chunks_concurrent(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, int k, int c_first,
                             int c_last, int delta, tcw_result* res, int* found, double t0);

}  // namespace

extern "C" int tcw_search(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, tcw_result* res) {
    if (!c || !t || !p || !res) return TCW_EINVAL;
    std::memset(res, 0, sizeof(*res));
    const double t0 = now_s();
    const int n = t->n;
    res->n = n;
    int rc = check_params(c, p, n, false);
    if (rc) return rc;
    std::vector<int> order;
    rc = depth_order_of(c, p, order);
    if (rc) return rc;
    const uint32_t xi = xi_of(n);
    const int iters = p->iters_per_launch > 0 ? p->iters_per_launch : default_iters(n);
    for (int k : order) {
        if (p->max_seconds > 0 && now_s() - t0 > p->max_seconds) break;
        int found = 0;
        if (k == 0) {
            if ((rc = search_k0(c, t, res, &found))) return rc;
            if (found) {
                res->seconds = now_s() - t0;
                return TCW_OK;
            }
            continue;
        }
        const int h = k / 2;
        const uint64_t nh = n_half_of(n, h);
        if (nh == 0) continue;  // space beyond 32-bit points: not searchable here
        const uint64_t npts = 2 * nh;
        int cf = 0, cl = 0;
        if (k % 2) {
            cf = p->chunk_first > 0 ? p->chunk_first : 1;
            cl = p->chunk_last > 0 ? p->chunk_last : (int)xi;
            if (cl > (int)xi) cl = (int)xi;
        }
        const bool enumerate = (int64_t)npts <= p->enum_max;
        const int delta = p->delta >= 0 ? p->delta : auto_delta(npts, p->log2_table);
        // odd depths with chunk_parallel != 1 run their chunks as concurrent batch members; for
        // enumerated chunks only while their tables (4 npts slots of 16 B each) fit the chunk pool
        const uint64_t n_chunks = (uint64_t)(cl - cf + 1);
        const bool concurrent =
            k % 2 && p->chunk_parallel != 1 &&
            (!enumerate || n_chunks * 64 * npts <= (1ull << CHUNK_TABLE_POOL_LOG2));
        if (concurrent) {
            // chunks in groups of G searched concurrently, one batch member each
            const int G = p->chunk_parallel <= 0 ? cl - cf + 1 : p->chunk_parallel;
            for (int first = cf; first <= cl && !found; first += G) {
                if (p->max_seconds > 0 && now_s() - t0 > p->max_seconds) break;
                // each member resolves an open delta against its own (smaller) table
                rc = search_chunks_concurrent(c, t, p, k, first, std::min(cl, first + G - 1), p->delta, res, &found,
                                              t0);
                if (rc) return rc;
            }
        }
        for (int chunk = cf; chunk <= cl && !found && !concurrent; ++chunk) {
            if (p->max_seconds > 0 && now_s() - t0 > p->max_seconds) break;
            if (enumerate) {
                if ((rc = search_enum(c, t, p, k, chunk, iters, res, &found, t0))) return rc;
                continue;
            }
            tcw_space sp{k, chunk, p->seed, p->version, delta};
            res->spaces++;
            const uint64_t budget = (uint64_t)p->budget_beta * npts << delta;
            const uint64_t per_version = version_steps(p, npts, delta, p->walks, p->log2_table);
            const uint32_t cap = (uint32_t)p->trail_cap_factor << delta;
            // a launch must not overrun a function version
            int iters_v = iters;
            const uint64_t fit = per_version / (uint64_t)p->walks;
            if ((uint64_t)iters_v > fit) iters_v = fit > 0 ? (int)fit : 1;
            tcw_walk* w = nullptr;
            rc = tcw_walk_begin(c, t, &sp, p->walks, p->log2_table, cap, 0, &w);
            if (rc) return rc;
            uint64_t used = 0, used_v = 0;
            uint32_t version = p->version;
            int64_t seen = 0;
            res->versions++;
            tcw_walk_stats st{};
            while (used < budget) {
                rc = tcw_walk_run(w, iters_v);
                res->launches++;
                if (!rc) rc = tcw_walk_stats_get(w, &st);
                if (!rc) rc = check_claws(c, w, seen, res, &found);
                if (rc) {
                    tcw_walk_end(w);
                    return rc;
                }
                used = used - used_v + (uint64_t)st.steps;
                used_v = (uint64_t)st.steps;
                if (found) break;
                if (p->max_seconds > 0 && now_s() - t0 > p->max_seconds) break;
                if (used_v >= per_version && used < budget) {
                    add_stats(res->stats, st);
                    std::memset(&st, 0, sizeof(st));
                    used_v = 0;
                    seen = 0;
                    ++version;
                    res->versions++;
                    rc = tcw_walk_reset(w, version);
                    if (rc) {
                        tcw_walk_end(w);
                        return rc;
                    }
                }
            }
            add_stats(res->stats, st);
            tcw_walk_end(w);
        }
        if (found) {
            res->seconds = now_s() - t0;
            return TCW_OK;
        }
    }
    res->status = 0;
    res->seconds = now_s() - t0;
    return TCW_OK;
}

// ---------------------------------------------------------------------------------------------
// Autotuner and batched search (many targets of mixed n and k)
namespace {

int64_t floor_pow2(uint64_t v) {
    int64_t p = 1;
    while ((uint64_t)(p * 2) <= v) p *= 2;
    return p;
}

int autotune(tcw_ctx* c, const tcw_target* t, int k, int chunk, int delta, uint64_t seed, TunedCfg* out) {
    const int n = t->n;
    const uint64_t key = ((uint64_t)n << 40) | ((uint64_t)k << 20) | (uint64_t)delta;
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        *out = it->second;
        return TCW_OK;
    }
    const uint64_t npts = 2 * n_half_of(n, k / 2);
    if (npts == 0) return fail(c, TCW_EINVAL, "space too large");
    // walks beyond N/4 only add warm-up (m / theta steps before the first distinguished points)
    const int64_t wmax = std::min<int64_t>(1 << 20, std::max<int64_t>(64, floor_pow2(npts / 4)));
    std::vector<int64_t> cands;
    for (int64_t w = 64; w < wmax; w *= 4) cands.push_back(w);
    cands.push_back(wmax);
    tcw_space sp{k, chunk, seed, 0xFFFFu, delta};
    std::vector<double> rates;
    for (int64_t w : cands) {
        tcw_walk* ws = nullptr;
        int rc = tcw_walk_begin(c, t, &sp, w, 16, (uint32_t)20 << delta, 0, &ws);
        if (rc) return rc;
        const int iters = (int)std::max<int64_t>(1, std::min<int64_t>(64, (1 << 21) / w));
        float ms = 0, tot = 0;
        rc = tcw_walk_run(ws, iters);
        if (!rc) rc = tcw_walk_last_ms(ws, &ms);
        for (int r = 0; r < 2 && !rc; ++r) {
            rc = tcw_walk_run(ws, iters);
            if (!rc) rc = tcw_walk_last_ms(ws, &ms);
            tot += ms;
        }
        tcw_walk_end(ws);
        if (rc) return rc;
        rates.push_back((double)w * iters * 2 / (tot * 1e-3));
    }
    double best = 0;
    for (double r : rates) best = std::max(best, r);
    size_t pick = cands.size() - 1;
    for (size_t i = 0; i < cands.size(); ++i)
        if (rates[i] >= 0.85 * best) {
            pick = i;
            break;
        }
    TunedCfg cfg;
    cfg.walks = cands[pick];
    cfg.rate = rates[pick];
    // launches of about 4 ms between host checks
    cfg.iters = (int)std::max(1.0, std::min(64.0, cfg.rate * 4e-3 / (double)cfg.walks));
    // the table holds every distinguished point of a version: max(2 N theta, 2 m) of them, 4x headroom
    const double dps = std::max(2.0 * (double)npts / (double)(1ull << delta), 2.0 * (double)cfg.walks);
    int lg = 10;
    while ((double)(1ull << lg) < 4 * dps && lg < 26) ++lg;
    cfg.log2_table = lg;
    c->tuned[key] = cfg;
    *out = cfg;
    return TCW_OK;
}

constexpr uint32_t BATCH_CLAW_CAP = 1024;

struct BatchTarget {
    const tcw_target* t = nullptr;
    tcw_walk_params p{};
    tcw_result* res = nullptr;
    std::vector<int> order;
    size_t oi = 0;
    int k = -1, chunk = 0, cl = 0;
    bool walking = false, done = false;
    std::unique_ptr<Space> space;
    tcw::WalkDev wd{};
    int64_t walks = 0;
    int iters = 0, log2 = 0, blocks = 0;
    uint64_t budget = 0, per_version = 0, used = 0, used_v = 0;
    uint32_t version = 0;
    int64_t seen = 0;
    size_t states_cap = 0;
    int table_cap = 0;
};

struct BatchBuffers {
    unsigned long long* stats = nullptr;   // count x ST_COUNT
    unsigned long long* claw_count = nullptr;
    uint64_t* claws = nullptr;             // count x BATCH_CLAW_CAP x 2
    tcw::SpaceDev* sps = nullptr;          // count
    tcw::WalkDev* wds = nullptr;           // count
    int32_t* blk_target[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int32_t* tgt_first = nullptr;          // count
    int32_t* tgt_blocks = nullptr;         // count
    ~BatchBuffers() {
        for (void* q : {(void*)stats, (void*)claw_count, (void*)claws, (void*)sps, (void*)wds, (void*)tgt_first,
                        (void*)tgt_blocks})
            if (q) (void)hipFree(q);
        for (auto* q : blk_target)
            if (q) (void)hipFree(q);
    }
};

void free_walk_buffers(BatchTarget& b) {
    if (b.wd.states) (void)hipFree(b.wd.states);
    if (b.wd.table) (void)hipFree(b.wd.table);
    b.wd.states = nullptr;
    b.wd.table = nullptr;
    b.states_cap = 0;
    b.table_cap = 0;
}

// (Re)start the walks of a target's current space on stream s: table cleared, counters zeroed.
int batch_restart(tcw_ctx* c, BatchTarget& b, int slot, BatchBuffers& bb, hipStream_t s) {
    HIP_TRY(c, tcw::launch_table_clear(b.wd.table, b.wd.log2_table, s));
    HIP_TRY(c, hipMemsetAsync(bb.stats + (size_t)slot * tcw::ST_COUNT, 0, tcw::ST_COUNT * 8, s));
    HIP_TRY(c, hipMemsetAsync(bb.claw_count + slot, 0, 8, s));
    HIP_TRY(c, tcw::launch_walk_init(b.space->dev, b.wd, s));
    return TCW_OK;
}

// Move a target to its next space: depth 0 is checked on the spot; the next space of a positive
// depth, enumerated when small and walked otherwise, leaves the target `walking`.
int batch_advance(tcw_ctx* c, BatchTarget& b, int slot, BatchBuffers& bb, hipStream_t s, double t0) {
    const int n = b.t->n;
    const uint32_t xi = xi_of(n);
    while (!b.done) {
        if (b.p.max_seconds > 0 && now_s() - t0 > b.p.max_seconds) {
            b.done = true;
            break;
        }
        // next (k, chunk)
        if (b.k >= 0 && b.k % 2 == 1 && b.chunk < b.cl) {
            b.chunk++;
        } else {
            if (b.oi >= b.order.size()) {
                b.done = true;
                break;
            }
            b.k = b.order[b.oi++];
            b.chunk = 0;
            b.cl = 0;
            if (b.k % 2) {
                b.chunk = b.p.chunk_first > 0 ? b.p.chunk_first : 1;
                b.cl = b.p.chunk_last > 0 ? std::min<int>(b.p.chunk_last, (int)xi) : (int)xi;
            }
        }
        int found = 0, rc = 0;
        if (b.k == 0) {
            if ((rc = search_k0(c, b.t, b.res, &found))) return rc;
            if (found) b.done = true;
            continue;
        }
        const uint64_t nh = n_half_of(n, b.k / 2);
        if (nh == 0) {
            b.chunk = b.cl;
            continue;
        }
        const uint64_t npts = 2 * nh;
        // A small space is enumerated: every point evaluated once, keyed in the table by its full
        // matrix hash, as one more member of the batch; it is done after npts steps.  Larger
        // spaces are walked.
        const bool enumerate = (int64_t)npts <= b.p.enum_max;
        int delta = 0;
        if (enumerate) {
            const int64_t wmax = std::max<int64_t>(64, b.p.walks);
            b.walks = (int64_t)npts < wmax ? (int64_t)npts : wmax;
            int lg = 4;
            while ((1ull << lg) < 4 * npts && lg < 30) ++lg;
            b.log2 = lg;
            b.iters = default_iters(n);
        } else {
            delta = b.p.delta >= 0 ? b.p.delta
                                   : auto_delta(npts, b.p.log2_table > 0 ? b.p.log2_table : default_log2_table(n));
            TunedCfg cfg;
            if (b.p.walks <= 0 || b.p.log2_table <= 0 || b.p.iters_per_launch <= 0) {
                if ((rc = autotune(c, b.t, b.k, b.chunk, delta, b.p.seed, &cfg))) return rc;
            }
            b.walks = b.p.walks > 0 ? b.p.walks : cfg.walks;
            b.log2 = b.p.log2_table > 0 ? b.p.log2_table : cfg.log2_table;
            b.iters = b.p.iters_per_launch > 0 ? b.p.iters_per_launch : cfg.iters;
        }
        b.space.reset(new Space());
        tcw_space sp{b.k, b.chunk, b.p.seed, b.p.version, delta};
        if ((rc = prepare_space(c, b.t, &sp, *b.space))) return rc;
        b.res->spaces++;
        b.res->versions++;
        b.version = b.p.version;
        if (enumerate) {
            b.budget = npts;
            b.per_version = ~0ull;  // no function versions: the enumeration is exhaustive
        } else {
            b.budget = (uint64_t)b.p.budget_beta * npts << delta;
            b.per_version = version_steps(&b.p, npts, delta, b.walks, b.log2);
            const uint64_t fit = b.per_version / (uint64_t)b.walks;
            if ((uint64_t)b.iters > fit) b.iters = fit > 0 ? (int)fit : 1;
        }
        b.used = b.used_v = 0;
        b.seen = 0;
        // walk buffers (kept across spaces when large enough)
        const size_t sbytes = (size_t)b.walks * sizeof(tcw::WalkState);
        if (b.states_cap < sbytes) {
            if (b.wd.states) (void)hipFree(b.wd.states);
            HIP_TRY(c, hipMalloc(&b.wd.states, sbytes));
            b.states_cap = sbytes;
        }
        if (b.table_cap < b.log2) {
            if (b.wd.table) (void)hipFree(b.wd.table);
            HIP_TRY(c, hipMalloc(&b.wd.table, ((size_t)1 << b.log2) * 16));
            b.table_cap = b.log2;
        }
        b.wd.walks = b.walks;
        b.wd.log2_table = b.log2;
        b.wd.cap = enumerate ? 2u : (uint32_t)b.p.trail_cap_factor << delta;
        b.wd.enumerate = enumerate ? 1 : 0;
        b.wd.n_points = npts;
        b.wd.stats = bb.stats + (size_t)slot * tcw::ST_COUNT;
        b.wd.claws = bb.claws + (size_t)slot * BATCH_CLAW_CAP * 2;
        b.wd.claw_count = bb.claw_count + slot;
        b.wd.claw_cap = BATCH_CLAW_CAP;
        if ((rc = batch_restart(c, b, slot, bb, s))) return rc;
        b.walking = true;
        return TCW_OK;
    }
    b.walking = false;
    free_walk_buffers(b);
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_autotune(tcw_ctx* c, const tcw_target* t, int k, int chunk, int delta, uint64_t seed,
                            int64_t* walks, int* iters, int* log2_table, double* steps_per_s) {
    if (!c || !t || !walks || !iters || !log2_table || !steps_per_s) return TCW_EINVAL;
    tcw_space sp{k, chunk, seed, 0, delta};
    int rc = check_space(c, t->n, &sp);
    if (rc) return rc;
    TunedCfg cfg;
    rc = autotune(c, t, k, chunk, delta, seed, &cfg);
    if (rc) return rc;
    *walks = cfg.walks;
    *iters = cfg.iters;
    *log2_table = cfg.log2_table;
    *steps_per_s = cfg.rate;
    return TCW_OK;
}

namespace {

tcw_walk_stats stats_of(const unsigned long long* st) {
    tcw_walk_stats ws{};
    ws.steps = (int64_t)st[tcw::ST_STEPS];
    ws.dps = (int64_t)st[tcw::ST_DPS];
    ws.inserts = (int64_t)st[tcw::ST_INSERTS];
    ws.abandoned = (int64_t)st[tcw::ST_ABANDONED];
    ws.robin_hood = (int64_t)st[tcw::ST_ROBIN];
    ws.same_side = (int64_t)st[tcw::ST_SAME];
    ws.reduction = (int64_t)st[tcw::ST_REDUCTION];
    ws.claws = (int64_t)st[tcw::ST_CLAWS];
    ws.table_full = (int64_t)st[tcw::ST_FULL];
    ws.spin_timeouts = (int64_t)st[tcw::ST_SPIN];
    return ws;
}

// Runs every member search of bt (each with its own depth order, chunk range, walks and table)
// in graph-captured rounds until all are done, or, with stop_on_first, until one member holds a
// verified decomposition.  *agg: walk steps per second of walk-kernel time.
int batch_run(tcw_ctx* c, std::vector<BatchTarget>& bt, bool stop_on_first, double t0, double* agg) {
    const int count = (int)bt.size();
    BatchBuffers bb;
    HIP_TRY(c, hipMalloc(&bb.stats, (size_t)count * tcw::ST_COUNT * 8));
    HIP_TRY(c, hipMalloc(&bb.claw_count, (size_t)count * 8));
    HIP_TRY(c, hipMalloc(&bb.claws, (size_t)count * BATCH_CLAW_CAP * 16));
    HIP_TRY(c, hipMalloc(&bb.sps, (size_t)count * sizeof(tcw::SpaceDev)));
    HIP_TRY(c, hipMalloc(&bb.wds, (size_t)count * sizeof(tcw::WalkDev)));
    HIP_TRY(c, hipMalloc(&bb.tgt_first, (size_t)count * 4));
    HIP_TRY(c, hipMalloc(&bb.tgt_blocks, (size_t)count * 4));
    HIP_TRY(c, hipMemsetAsync(bb.stats, 0, (size_t)count * tcw::ST_COUNT * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(bb.claw_count, 0, (size_t)count * 8, c->stream));
    int rc = TCW_OK;
    for (int i = 0; i < count && !rc; ++i) {
        rc = batch_advance(c, bt[i], i, bb, c->stream, t0);
        if (bt[i].done) bt[i].res->seconds = now_s() - t0;
    }
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));

    // streams for the graph: one branch per qubit count (default priority)
    hipStream_t gs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    HIP_TRY(c, hipStreamCreateWithFlags(&gs[0], hipStreamNonBlocking));
    for (int n = 1; n <= 4; ++n) {
        HIP_TRY(c, hipStreamCreateWithFlags(&gs[n], hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&join[n], hipEventDisableTiming));
    }
    HIP_TRY(c, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool dirty = true;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    int64_t total_steps = 0;
    double walk_seconds = 0;
    std::vector<unsigned long long> stats((size_t)count * tcw::ST_COUNT), ccount(count);
    std::vector<tcw::SpaceDev> h_sps(count);
    std::vector<tcw::WalkDev> h_wds(count);
    std::vector<int32_t> h_first(count, 0), h_blocks(count, 0);
    int iters_n[5] = {0, 0, 0, 0, 0}, blocks_n[5] = {0, 0, 0, 0, 0};
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int n = 0; n <= 4; ++n) {
            if (gs[n]) (void)hipStreamDestroy(gs[n]);
            if (join[n]) (void)hipEventDestroy(join[n]);
        }
        if (fork) (void)hipEventDestroy(fork);
        for (auto& b : bt) free_walk_buffers(b);
    };
#define BATCH_TRY(expr)                      \
    do {                                     \
        hipError_t _e = (expr);              \
        if (_e != hipSuccess) {              \
            cleanup();                       \
            return hip_fail(c, _e, #expr);   \
        }                                    \
    } while (0)
    bool stop = false;
    for (;;) {
        bool any = false;
        for (auto& b : bt) any |= b.walking;
        if (!any) break;
        if (dirty) {
            // block ranges per target, per qubit count
            std::vector<int32_t> blk[5];
            for (int n = 1; n <= 4; ++n) {
                int active = 0;
                for (auto& b : bt) active += (b.walking && b.t->n == n);
                if (!active) {
                    blocks_n[n] = 0;
                    continue;
                }
                const int cap_blocks = std::max(1, tcw::walk_grid_blocks(n, c->device) / active);
                iters_n[n] = 1 << 30;
                for (int i = 0; i < count; ++i) {
                    BatchTarget& b = bt[i];
                    if (!b.walking || b.t->n != n) continue;
                    const int wpb = tcw::walks_per_block(n);
                    b.blocks = (int)std::min<int64_t>((b.walks + wpb - 1) / wpb, cap_blocks);
                    h_first[i] = (int32_t)blk[n].size();
                    h_blocks[i] = b.blocks;
                    for (int j = 0; j < b.blocks; ++j) blk[n].push_back(i);
                    iters_n[n] = std::min(iters_n[n], b.iters);
                }
                blocks_n[n] = (int)blk[n].size();
                if (bb.blk_target[n]) (void)hipFree(bb.blk_target[n]);
                BATCH_TRY(hipMalloc(&bb.blk_target[n], blk[n].size() * 4));
                BATCH_TRY(hipMemcpy(bb.blk_target[n], blk[n].data(), blk[n].size() * 4, hipMemcpyHostToDevice));
            }
            BATCH_TRY(hipMemcpy(bb.tgt_first, h_first.data(), count * 4, hipMemcpyHostToDevice));
            BATCH_TRY(hipMemcpy(bb.tgt_blocks, h_blocks.data(), count * 4, hipMemcpyHostToDevice));
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
            // capture: fork one branch per qubit count, join
            BATCH_TRY(hipStreamBeginCapture(gs[0], hipStreamCaptureModeThreadLocal));
            BATCH_TRY(hipEventRecord(fork, gs[0]));
            for (int n = 1; n <= 4; ++n) {
                if (!blocks_n[n]) continue;
                BATCH_TRY(hipStreamWaitEvent(gs[n], fork, 0));
                BATCH_TRY(tcw::launch_walk_batch(n, bb.sps, bb.wds, bb.blk_target[n], bb.tgt_first, bb.tgt_blocks,
                                                 blocks_n[n], iters_n[n], gs[n]));
                BATCH_TRY(hipEventRecord(join[n], gs[n]));
                BATCH_TRY(hipStreamWaitEvent(gs[0], join[n], 0));
            }
            BATCH_TRY(hipStreamEndCapture(gs[0], &graph));
            BATCH_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            dirty = false;
        }
        // descriptors for the next graph replay (salts change with versions)
        for (int i = 0; i < count; ++i) {
            if (!bt[i].walking) continue;
            h_sps[i] = bt[i].space->dev;
            h_wds[i] = bt[i].wd;
        }
        BATCH_TRY(hipMemcpyAsync(bb.sps, h_sps.data(), count * sizeof(tcw::SpaceDev), hipMemcpyHostToDevice, gs[0]));
        BATCH_TRY(hipMemcpyAsync(bb.wds, h_wds.data(), count * sizeof(tcw::WalkDev), hipMemcpyHostToDevice, gs[0]));
        const double tl = now_s();
        BATCH_TRY(hipGraphLaunch(exec, gs[0]));
        BATCH_TRY(hipMemcpyAsync(stats.data(), bb.stats, stats.size() * 8, hipMemcpyDeviceToHost, gs[0]));
        BATCH_TRY(hipMemcpyAsync(ccount.data(), bb.claw_count, count * 8, hipMemcpyDeviceToHost, gs[0]));
        BATCH_TRY(hipStreamSynchronize(gs[0]));
        walk_seconds += now_s() - tl;
        for (int i = 0; i < count; ++i) {
            BatchTarget& b = bt[i];
            if (!b.walking) continue;
            b.res->launches++;
            const unsigned long long* st = &stats[(size_t)i * tcw::ST_COUNT];
            const uint64_t steps_now = st[tcw::ST_STEPS];
            total_steps += (int64_t)(steps_now - b.used_v);
            b.used += steps_now - b.used_v;
            b.used_v = steps_now;
            int found = 0;
            const int64_t avail = (int64_t)std::min<unsigned long long>(ccount[i], BATCH_CLAW_CAP);
            if (avail > b.seen) {
                const int64_t m = avail - b.seen;
                std::vector<uint64_t> pairs(2 * m);
                BATCH_TRY(hipMemcpy(pairs.data(), b.wd.claws + 2 * b.seen, 16 * m, hipMemcpyDeviceToHost));
                std::vector<uint64_t> u0(m), u1(m);
                for (int64_t j = 0; j < m; ++j) {
                    u0[j] = pairs[2 * j];
                    u1[j] = pairs[2 * j + 1];
                }
                rc = check_pairs(c, *b.space, u0.data(), u1.data(), m, b.res, &found);
                if (rc) {
                    cleanup();
                    return rc;
                }
                b.seen = avail;
            }
            const tcw_walk_stats ws = stats_of(st);
            const bool over_time = b.p.max_seconds > 0 && now_s() - t0 > b.p.max_seconds;
            if (found || over_time || b.used >= b.budget) {
                add_stats(b.res->stats, ws);
                b.walking = false;
                dirty = true;
                if (found || over_time) {
                    b.done = true;
                    b.res->seconds = now_s() - t0;
                    free_walk_buffers(b);
                } else {
                    rc = batch_advance(c, b, i, bb, gs[0], t0);
                    if (rc) {
                        cleanup();
                        return rc;
                    }
                    if (b.done) b.res->seconds = now_s() - t0;
                }
            } else if (b.used_v >= b.per_version) {
                add_stats(b.res->stats, ws);
                b.version++;
                b.res->versions++;
                b.space->set_version(b.version);
                b.used_v = 0;
                b.seen = 0;
                rc = batch_restart(c, b, i, bb, gs[0]);
                if (rc) {
                    cleanup();
                    return rc;
                }
            }
            if (stop_on_first && b.res->status == 1) stop = true;
        }
        BATCH_TRY(hipStreamSynchronize(gs[0]));
        if (stop) {
            // one member found a verified decomposition: end the others with their counts so far
            for (int i = 0; i < count; ++i) {
                BatchTarget& b = bt[i];
                if (!b.walking) continue;
                add_stats(b.res->stats, stats_of(&stats[(size_t)i * tcw::ST_COUNT]));
                b.walking = false;
                b.done = true;
                b.res->seconds = now_s() - t0;
            }
            break;
        }
    }
#undef BATCH_TRY
    cleanup();
    for (auto& b : bt)
        if (b.res->seconds == 0) b.res->seconds = now_s() - t0;
    if (agg) *agg = walk_seconds > 0 ? (double)total_steps / walk_seconds : 0.0;
    return TCW_OK;
}

}  // namespace

namespace {

int search_chunks_concurrent(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, int k, int c_first,
                             int c_last, int delta, tcw_result* res, int* found, double t0) {
    const int n = t->n;
    const int G = c_last - c_first + 1;
    int lg_g = 0;
    while ((1 << lg_g) < G) ++lg_g;
    const int64_t walks_c = std::max<int64_t>(64, p->walks / G);
    const int log2_c = std::max(10, std::min(p->log2_table, CHUNK_TABLE_POOL_LOG2 - 4 - lg_g));
    const int iters = p->iters_per_launch > 0 ? p->iters_per_launch : default_iters(n);
    std::vector<BatchTarget> bt(G);
    std::vector<tcw_result> rs(G);
    for (int i = 0; i < G; ++i) {
        BatchTarget& b = bt[i];
        b.t = t;
        b.p = *p;
        b.p.walks = walks_c;
        b.p.log2_table = log2_c;
        b.p.iters_per_launch = iters;
        b.p.delta = delta;
        b.p.chunk_first = b.p.chunk_last = c_first + i;
        b.order.assign(1, k);
        std::memset(&rs[i], 0, sizeof(tcw_result));
        rs[i].n = n;
        b.res = &rs[i];
    }
    const int rc = batch_run(c, bt, true, t0, nullptr);
    if (rc) return rc;
    int64_t launches = 0;
    for (int i = 0; i < G; ++i) {
        const tcw_result& r = rs[i];
        add_stats(res->stats, r.stats);
        res->spaces += r.spaces;
        res->versions += r.versions;
        res->false_claws += r.false_claws;
        launches = std::max(launches, r.launches);
        if (r.status == 1 && !*found) {
            *found = 1;
            res->status = 1;
            res->t = r.t;
            res->chunk = r.chunk;
            std::memcpy(res->paulis, r.paulis, sizeof(res->paulis));
            std::memcpy(res->clifford_perm, r.clifford_perm, sizeof(res->clifford_perm));
            std::memcpy(res->clifford_sign, r.clifford_sign, sizeof(res->clifford_sign));
        }
    }
    res->launches += launches;
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_search_batch(tcw_ctx* c, const tcw_target* const* targets, int count, const tcw_walk_params* params,
                                tcw_result* results, double* aggregate_steps_per_s) {
    if (!c || !targets || !params || !results || count < 1) return TCW_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!targets[i]) return fail(c, TCW_EINVAL, "NULL target in batch");
    const double t0 = now_s();
    std::vector<BatchTarget> bt(count);
    int rc = TCW_OK;
    for (int i = 0; i < count && !rc; ++i) {
        BatchTarget& b = bt[i];
        b.t = targets[i];
        b.p = params[i];
        b.res = &results[i];
        std::memset(b.res, 0, sizeof(tcw_result));
        b.res->n = b.t->n;
        rc = check_params(c, &b.p, b.t->n, true);
        if (!rc) rc = depth_order_of(c, &b.p, b.order);
    }
    if (rc) return rc;
    return batch_run(c, bt, false, t0, aggregate_steps_per_s);
}

// ---------------------------------------------------------------------------------------------
// Depth-order network: canonical features, exact labels by meet in the middle, BF16 MFMA training.
struct tcw_mlp {
    tcw_ctx* ctx = nullptr;
    int inp = 0, hidden = 0, depth = 0, classes = 0, L = 0;
    std::vector<int> sz;
    std::vector<int64_t> w_off, b_off;
    int64_t count = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    std::vector<void*> Wb;
    int step = 0;
    int cap_b = 0;
    void* Xb = nullptr;
    std::vector<float*> Z, Gf;
    std::vector<void*> Hb, Gb;
    float *logits = nullptr, *probs = nullptr, *loss = nullptr, *xdev = nullptr;
    float* dw_part = nullptr;  // partial weight-gradient tiles of the batch split
    size_t dw_part_floats = 0;

    void free_batch() {
        for (void* q : {Xb, (void*)logits, (void*)probs, (void*)dw_part})
            if (q) (void)hipFree(q);
        dw_part = nullptr;
        dw_part_floats = 0;
        for (auto* q : Z)
            if (q) (void)hipFree(q);
        for (auto* q : Gf)
            if (q) (void)hipFree(q);
        for (auto* q : Hb)
            if (q) (void)hipFree(q);
        for (auto* q : Gb)
            if (q) (void)hipFree(q);
        Xb = nullptr;
        logits = probs = nullptr;
        Z.clear();
        Gf.clear();
        Hb.clear();
        Gb.clear();
        cap_b = 0;
    }
    ~tcw_mlp() {
        free_batch();
        for (void* q : {(void*)P, (void*)G, (void*)M, (void*)V, (void*)loss, (void*)xdev})
            if (q) (void)hipFree(q);
        for (auto* q : Wb)
            if (q) (void)hipFree(q);
    }
};

namespace {

int mlp_ensure_batch(tcw_mlp* m, int b) {
    tcw_ctx* c = m->ctx;
    if (b <= m->cap_b) return TCW_OK;
    m->free_batch();
    HIP_TRY(c, hipMalloc(&m->Xb, (size_t)b * m->inp * 2));
    m->Z.assign(m->depth, nullptr);
    m->Hb.assign(m->depth, nullptr);
    m->Gf.assign(m->L, nullptr);
    m->Gb.assign(m->L, nullptr);
    for (int l = 0; l < m->depth; ++l) {
        HIP_TRY(c, hipMalloc(&m->Z[l], (size_t)b * m->hidden * 4));
        HIP_TRY(c, hipMalloc(&m->Hb[l], (size_t)b * m->hidden * 2));
    }
    for (int l = 0; l < m->L; ++l) {
        HIP_TRY(c, hipMalloc(&m->Gf[l], (size_t)b * m->sz[l + 1] * 4));
        HIP_TRY(c, hipMalloc(&m->Gb[l], (size_t)b * m->sz[l + 1] * 2));
    }
    HIP_TRY(c, hipMalloc(&m->logits, (size_t)b * m->classes * 4));
    HIP_TRY(c, hipMalloc(&m->probs, (size_t)b * m->classes * 4));
    size_t part = 0;
    for (int l = 0; l < m->L; ++l) part = std::max(part, tcw::mlp_dw_part_floats(m->sz[l], m->sz[l + 1], b));
    if (part > 0) {
        HIP_TRY(c, hipMalloc(&m->dw_part, part * 4));
        m->dw_part_floats = part;
    }
    m->cap_b = b;
    return TCW_OK;
}

int mlp_sync_bf16(tcw_mlp* m) {
    for (int l = 0; l < m->L; ++l)
        HIP_TRY(m->ctx, tcw::mlp_to_bf16(m->P + m->w_off[l], m->Wb[l], (int64_t)m->sz[l] * m->sz[l + 1], m->ctx->stream));
    return TCW_OK;
}

// forward over a batch; with labels also the loss sum and the output-layer gradient
int mlp_forward(tcw_mlp* m, const float* x, int b, const int32_t* labels) {
    tcw_ctx* c = m->ctx;
    int rc = mlp_ensure_batch(m, b);
    if (rc) return rc;
    HIP_TRY(c, tcw::mlp_to_bf16(x, m->Xb, (int64_t)b * m->inp, c->stream));
    for (int l = 0; l < m->L; ++l) {
        const void* A = l == 0 ? m->Xb : m->Hb[l - 1];
        const int K = m->sz[l], N = m->sz[l + 1];
        if (l < m->L - 1) {
            HIP_TRY(c, tcw::mlp_gemm(1, A, m->Wb[l], b, N, K, K, N, m->Z[l], N, m->P + m->b_off[l], nullptr, m->Hb[l],
                                     c->stream));
        } else {
            HIP_TRY(c, tcw::mlp_gemm(2, A, m->Wb[l], b, N, K, K, N, m->logits, N, m->P + m->b_off[l], nullptr, nullptr,
                                     c->stream));
        }
    }
    if (labels) HIP_TRY(c, hipMemsetAsync(m->loss, 0, 4, c->stream));
    HIP_TRY(c, tcw::mlp_softmax_ce(m->logits, labels, b, m->classes, m->probs, labels ? m->Gf[m->L - 1] : nullptr,
                                   labels ? m->Gb[m->L - 1] : nullptr, labels ? m->loss : nullptr, c->stream));
    return TCW_OK;
}

int mlp_backward(tcw_mlp* m, int b) {
    tcw_ctx* c = m->ctx;
    for (int l = m->L - 1; l >= 0; --l) {
        const void* Hin = l == 0 ? m->Xb : m->Hb[l - 1];
        const int in = m->sz[l], out = m->sz[l + 1];
        // dW_l = H_in^T G_l
        HIP_TRY(c, tcw::mlp_gemm_dw(Hin, m->Gb[l], in, out, b, m->G + m->w_off[l], m->dw_part, m->dw_part_floats,
                                    c->stream));
        HIP_TRY(c, tcw::mlp_colsum(m->Gf[l], b, out, m->G + m->b_off[l], c->stream));
        if (l > 0) {
            // G_{l-1} = (G_l W_l^T) * gelu'(Z_{l-1})
            HIP_TRY(c, tcw::mlp_gemm(4, m->Gb[l], m->Wb[l], b, in, out, out, out, m->Gf[l - 1], in, nullptr, m->Z[l - 1],
                                     m->Gb[l - 1], c->stream));
        }
    }
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_mlp_create(tcw_ctx* c, int inp, int hidden, int depth, int classes, const float* init, uint64_t seed,
                              tcw_mlp** out) {
    if (!c || !out || inp < 1 || hidden < 1 || depth < 0 || depth > 16 || classes < 2) return TCW_EINVAL;
    *out = nullptr;
    tcw_mlp* m = new (std::nothrow) tcw_mlp();
    if (!m) return TCW_ENOMEM;
    m->ctx = c;
    m->inp = inp;
    m->hidden = hidden;
    m->depth = depth;
    m->classes = classes;
    m->L = depth + 1;
    m->sz.push_back(inp);
    for (int l = 0; l < depth; ++l) m->sz.push_back(hidden);
    m->sz.push_back(classes);
    int64_t off = 0;
    for (int l = 0; l < m->L; ++l) {
        m->w_off.push_back(off);
        off += (int64_t)m->sz[l] * m->sz[l + 1];
        m->b_off.push_back(off);
        off += m->sz[l + 1];
    }
    m->count = off;
    auto bail = [&](hipError_t e) {
        delete m;
        return hip_fail(c, e, "network allocation");
    };
    hipError_t e = hipMalloc(&m->P, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->G, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->M, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->V, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->loss, 4);
    if (e != hipSuccess) return bail(e);
    m->Wb.assign(m->L, nullptr);
    for (int l = 0; l < m->L && e == hipSuccess; ++l) e = hipMalloc(&m->Wb[l], (size_t)m->sz[l] * m->sz[l + 1] * 2);
    if (e == hipSuccess) e = hipMemsetAsync(m->M, 0, off * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->V, 0, off * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->P, 0, off * 4, c->stream);
    if (e != hipSuccess) return bail(e);
    if (init) {
        e = hipMemcpyAsync(m->P, init, off * 4, hipMemcpyHostToDevice, c->stream);
    } else {
        int64_t idx = 0;
        for (int l = 0; l < m->L && e == hipSuccess; ++l) {
            const int64_t cnt = (int64_t)m->sz[l] * m->sz[l + 1];
            e = tcw::mlp_init(m->P + m->w_off[l], cnt, idx, m->sz[l], seed, c->stream);
            idx += cnt;
        }
    }
    if (e != hipSuccess) return bail(e);
    int rc = mlp_sync_bf16(m);
    if (!rc) {
        hipError_t se = hipStreamSynchronize(c->stream);
        if (se != hipSuccess) rc = hip_fail(c, se, "network init");
    }
    if (rc) {
        delete m;
        return rc;
    }
    *out = m;
    return TCW_OK;
}

extern "C" int tcw_mlp_free(tcw_mlp* m) {
    if (!m) return TCW_EINVAL;
    (void)hipStreamSynchronize(m->ctx->stream);
    delete m;
    return TCW_OK;
}

extern "C" int tcw_mlp_param_count(const tcw_mlp* m, int64_t* count) {
    if (!m || !count) return TCW_EINVAL;
    *count = m->count;
    return TCW_OK;
}

extern "C" int tcw_mlp_get_params(tcw_mlp* m, float* host) {
    if (!m || !host) return TCW_EINVAL;
    HIP_TRY(m->ctx, hipMemcpyAsync(host, m->P, m->count * 4, hipMemcpyDeviceToHost, m->ctx->stream));
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_set_params(tcw_mlp* m, const float* host) {
    if (!m || !host) return TCW_EINVAL;
    HIP_TRY(m->ctx, hipMemcpyAsync(m->P, host, m->count * 4, hipMemcpyHostToDevice, m->ctx->stream));
    int rc = mlp_sync_bf16(m);
    if (rc) return rc;
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_forward(tcw_mlp* m, const float* x, int batch, float* probs) {
    if (!m || !x || !probs || batch < 1) return TCW_EINVAL;
    int rc = mlp_forward(m, x, batch, nullptr);
    if (rc) return rc;
    HIP_TRY(m->ctx, hipMemcpyAsync(probs, m->probs, (size_t)batch * m->classes * 4, hipMemcpyDeviceToDevice,
                                   m->ctx->stream));
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_gradients(tcw_mlp* m, const float* x, const int32_t* labels, int batch, float* grads_host,
                                 float* loss) {
    if (!m || !x || !labels || batch < 1) return TCW_EINVAL;
    int rc = mlp_forward(m, x, batch, labels);
    if (!rc) rc = mlp_backward(m, batch);
    if (rc) return rc;
    float ls = 0;
    HIP_TRY(m->ctx, hipMemcpyAsync(&ls, m->loss, 4, hipMemcpyDeviceToHost, m->ctx->stream));
    if (grads_host) HIP_TRY(m->ctx, hipMemcpyAsync(grads_host, m->G, m->count * 4, hipMemcpyDeviceToHost, m->ctx->stream));
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    if (loss) *loss = ls / (float)batch;
    return TCW_OK;
}

extern "C" int tcw_mlp_train_step(tcw_mlp* m, const float* x, const int32_t* labels, int batch, float lr, float* loss) {
    if (!m || !x || !labels || batch < 1 || !(lr > 0)) return TCW_EINVAL;
    int rc = mlp_forward(m, x, batch, labels);
    if (!rc) rc = mlp_backward(m, batch);
    if (rc) return rc;
    m->step++;
    HIP_TRY(m->ctx, tcw::mlp_adam(m->P, m->G, m->M, m->V, m->count, lr, 0.9f, 0.999f, 1e-8f, m->step, m->ctx->stream));
    rc = mlp_sync_bf16(m);
    if (rc) return rc;
    if (loss) {
        float ls = 0;
        HIP_TRY(m->ctx, hipMemcpyAsync(&ls, m->loss, 4, hipMemcpyDeviceToHost, m->ctx->stream));
        HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
        *loss = ls / (float)batch;
    }
    return TCW_OK;
}

extern "C" int tcw_features(tcw_ctx* c, const tcw_target* t, float* out_dev) {
    if (!c || !t || !out_dev) return TCW_EINVAL;
    if (t->n > 3) return fail(c, TCW_EINVAL, "features are defined for n <= 3");
    HIP_TRY(c, tcw::exact_features(t->U, out_dev, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_depth_order(tcw_mlp* m, const tcw_target* t, int k_max, int32_t* order_out, float* probs_out) {
    if (!m || !t || !order_out || k_max < 0) return TCW_EINVAL;
    tcw_ctx* c = m->ctx;
    const int R = 1 << (2 * t->n);
    if (R * R != m->inp) return fail(c, TCW_EINVAL, "network input size does not match the target");
    if (!m->xdev) HIP_TRY(c, hipMalloc(&m->xdev, (size_t)m->inp * 4));
    int rc = tcw_features(c, t, m->xdev);
    if (!rc) rc = mlp_forward(m, m->xdev, 1, nullptr);
    if (rc) return rc;
    std::vector<float> p(m->classes);
    HIP_TRY(c, hipMemcpyAsync(p.data(), m->probs, m->classes * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (probs_out)
        for (int i = 0; i < m->classes; ++i) probs_out[i] = p[i];
    // depths 0..k_max by descending probability (ties: smaller depth first)
    std::vector<int> ks;
    for (int k = 0; k <= k_max; ++k) ks.push_back(k);
    auto prob = [&](int k) { return k < m->classes ? p[k] : -1.0f; };
    std::stable_sort(ks.begin(), ks.end(), [&](int a, int b) { return prob(a) > prob(b); });
    for (int i = 0; i <= k_max; ++i) order_out[i] = ks[i];
    return TCW_OK;
}

namespace {

// Hash table of every left-Clifford coset reached by <= h_max rotations from the identity, keyed by
// matrix hash, value 255 - (least number of rotations); shared by the labelling and certificate calls.
struct LevelTable {
    uint64_t* table = nullptr;
    uint64_t* keys = nullptr;
    uint32_t* zero_phi = nullptr;
    int lg = 0;
    tcw::SpaceDev sp{};
    ~LevelTable() {
        for (void* q : {(void*)table, (void*)keys, (void*)zero_phi})
            if (q) (void)hipFree(q);
    }
};

int build_level_table(tcw_ctx* c, int n, int h_max, uint64_t seed, LevelTable& lt) {
    const int R = 1 << (2 * n);
    HIP_TRY(c, hipMalloc(&lt.zero_phi, (size_t)R * R / 2 * 4));
    HIP_TRY(c, hipMemsetAsync(lt.zero_phi, 0, (size_t)R * R / 2 * 4, c->stream));
    HIP_TRY(c, hipMalloc(&lt.keys, (size_t)R * 8));
    HIP_TRY(c, tcw::keys_fill(n, seed, lt.keys, c->stream));
    uint64_t entries = 0;
    for (int h = 0; h <= h_max; ++h) entries += n_half_of(n, h);
    lt.lg = 10;
    while ((1ull << lt.lg) < 4 * entries && lt.lg < 30) ++lt.lg;
    HIP_TRY(c, hipMalloc(&lt.table, ((size_t)1 << lt.lg) * 16));
    HIP_TRY(c, tcw::launch_table_clear(lt.table, lt.lg, c->stream));
    lt.sp.delta = 0;
    lt.sp.salt_h = tcw::sm64(tcw::sm64(seed, 2), 0x4C4142454Cull);
    lt.sp.keys = lt.keys;
    lt.sp.phi = lt.zero_phi;
    for (int h = 0; h <= h_max; ++h) {
        lt.sp.h = h;
        lt.sp.n_half = (uint32_t)n_half_of(n, h);
        HIP_TRY(c, tcw::mitm_levels(n, lt.sp, h, lt.table, lt.lg, c->stream));
    }
    return TCW_OK;
}

int check_mitm_args(tcw_ctx* c, int n, int h_max) {
    if (n < 1 || n > 3) return fail(c, TCW_EINVAL, "meet in the middle runs for n <= 3");
    if (h_max < 0 || n_half_of(n, h_max) == 0) return fail(c, TCW_EINVAL, "h_max too large");
    uint64_t entries = 0;
    for (int h = 0; h <= h_max; ++h) entries += n_half_of(n, h);
    if (entries > (1ull << 28)) return fail(c, TCW_EINVAL, "h_max too large for the level table");
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_label_batch(tcw_ctx* c, int n, int count, const uint16_t* words, const int32_t* offsets,
                               const int32_t* kof, int h_max, uint64_t seed, float* features_dev, int32_t* labels_dev) {
    if (!c || !words || !offsets || !kof || !features_dev || !labels_dev || count < 1) return TCW_EINVAL;
    int rc = check_mitm_args(c, n, h_max);
    if (rc) return rc;
    // the words are read on the device exactly as these arrays describe them: check them here
    if (offsets[0] != 0) return fail(c, TCW_EINVAL, "offsets[0] must be 0");
    const uint32_t xi = xi_of(n);
    for (int i = 0; i < count; ++i) {
        const int64_t len = (int64_t)offsets[i + 1] - offsets[i];
        if (len < 0 || kof[i] < 0 || kof[i] > len) return fail(c, TCW_EINVAL, "offsets must not decrease and kof[i] <= word length");
        if (2 * (len - kof[i]) + kof[i] > 256) return fail(c, TCW_EINVAL, "a word is longer than 256 rotations once expanded");
    }
    for (int64_t j = 0; j < offsets[count]; ++j)
        if (words[j] < 1 || words[j] > xi) return fail(c, TCW_EINVAL, "Pauli code out of range 1..4^n - 1");
    const int R = 1 << (2 * n);
    const int64_t nw = offsets[count];
    uint16_t* dwords = nullptr;
    int32_t *doff = nullptr, *dk = nullptr, *rot = nullptr;
    uint32_t* phi = nullptr;
    void* scratch = nullptr;
    const int chunk = 1024, blocks = 256;
    auto cleanup = [&]() {
        for (void* q : {(void*)dwords, (void*)doff, (void*)dk, (void*)rot, (void*)phi, scratch})
            if (q) (void)hipFree(q);
    };
#define LB_TRY(expr)                         \
    do {                                     \
        hipError_t _e = (expr);              \
        if (_e != hipSuccess) {              \
            cleanup();                       \
            return hip_fail(c, _e, #expr);   \
        }                                    \
    } while (0)
    LB_TRY(hipMalloc(&dwords, nw * 2 + 2));
    LB_TRY(hipMalloc(&doff, (count + 1) * 4));
    LB_TRY(hipMalloc(&dk, count * 4));
    LB_TRY(hipMemcpyAsync(dwords, words, nw * 2, hipMemcpyHostToDevice, c->stream));
    LB_TRY(hipMemcpyAsync(doff, offsets, (count + 1) * 4, hipMemcpyHostToDevice, c->stream));
    LB_TRY(hipMemcpyAsync(dk, kof, count * 4, hipMemcpyHostToDevice, c->stream));
    LB_TRY(hipMalloc(&rot, chunk * 4));
    LB_TRY(hipMalloc(&phi, (size_t)chunk * R * R / 2 * 4));
    LB_TRY(hipMalloc(&scratch, tcw::build_batch_scratch_bytes(n, blocks)));
    LevelTable lt;
    if ((rc = build_level_table(c, n, h_max, seed, lt)) || (rc = clear_flag(c))) {
        cleanup();
        return rc;
    }
    for (int first = 0; first < count; first += chunk) {
        const int cnt = std::min(chunk, count - first);
        LB_TRY(tcw::build_batch(n, dwords, doff + first, dk + first, cnt, scratch, blocks, phi, rot,
                                features_dev + (size_t)first * R * R, c->flag, c->stream));
        LB_TRY(tcw::mitm_probe(n, lt.sp, phi, rot, cnt, h_max, lt.table, lt.lg, labels_dev + first, c->stream));
    }
    int flag = 0;
    rc = read_flag(c, &flag);
    cleanup();
#undef LB_TRY
    if (rc) return rc;
    if (flag) return fail(c, TCW_EOVERFLOW, "target outside the int8 / int32 range or word too long");
    return TCW_OK;
}

extern "C" int tcw_min_tcount(tcw_ctx* c, const tcw_target* t, int h_max, uint64_t seed, int32_t* t_out) {
    if (!c || !t || !t_out) return TCW_EINVAL;
    int rc = check_mitm_args(c, t->n, h_max);
    if (rc) return rc;
    const int n = t->n;
    const int R = 1 << (2 * n);
    uint32_t* phi = nullptr;
    int32_t* dev_i32 = nullptr;  // [0] rot_e, [1] result
    auto cleanup = [&]() {
        if (phi) (void)hipFree(phi);
        if (dev_i32) (void)hipFree(dev_i32);
    };
    LevelTable lt;
    int32_t e_u = 0;
    int flag = 0;
    hipError_t err = hipMalloc(&phi, (size_t)R * R / 2 * 4 + 16);
    if (err == hipSuccess) err = hipMalloc(&dev_i32, 2 * sizeof(int32_t));
    if (err == hipSuccess) err = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (err == hipSuccess) err = tcw::exact_pack_phi(t->U, phi, c->flag, c->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(&e_u, t->U.e, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (err != hipSuccess) {
        cleanup();
        return hip_fail(c, err, "target packing");
    }
    if ((rc = read_flag(c, &flag))) {
        cleanup();
        return rc;
    }
    if (flag) {
        cleanup();
        return fail(c, TCW_EOVERFLOW, "target entry outside the int8 range (exponent too large)");
    }
    const int32_t rot_e = (int32_t)((30ll * e_u) % 61);
    err = hipMemcpyAsync(dev_i32, &rot_e, sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
    if (err != hipSuccess) {
        cleanup();
        return hip_fail(c, err, "rot_e upload");
    }
    if ((rc = build_level_table(c, n, h_max, seed, lt))) {
        cleanup();
        return rc;
    }
    err = tcw::mitm_probe(n, lt.sp, phi, dev_i32, 1, h_max, lt.table, lt.lg, dev_i32 + 1, c->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(t_out, dev_i32 + 1, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
    cleanup();
    if (err != hipSuccess) return hip_fail(c, err, "meet-in-the-middle probe");
    return TCW_OK;
}

extern "C" int tcw_mlp_train(tcw_mlp* m, const float* x, const int32_t* labels, int64_t count, int batch, int epochs,
                             float lr, float* last_epoch_loss) {
    if (!m || !x || !labels || count < 1 || batch < 1 || epochs < 1 || !(lr > 0)) return TCW_EINVAL;
    double tot = 0;
    int64_t nb = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        tot = 0;
        nb = 0;
        for (int64_t first = 0; first < count; first += batch) {
            const int b = (int)std::min<int64_t>(batch, count - first);
            float ls = 0;
            int rc = tcw_mlp_train_step(m, x + first * m->inp, labels + first, b, lr, &ls);
            if (rc) return rc;
            tot += ls * b;
            nb += b;
        }
    }
    if (last_epoch_loss) *last_epoch_loss = (float)(tot / (double)nb);
    return TCW_OK;
}
