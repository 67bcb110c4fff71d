// Macro-elements of mixed polynomial degree and boundary type in one call
// (the batch entry points of mehdg.h).
//
// The kernels are compiled per degree, so a batch keeps one context per
// degree present.  The macros are ordered by degree (stable), and every
// per-macro array of the batch is flat in that order: the macros of one
// degree are one contiguous slice, which that degree's context reads and
// writes in place (no copies).  The residual pass of every group that is
// not streamed (residual, entropy production, pointwise Jacobian
// coefficients: the same workgroup shape at every degree) is one persistent
// launch over a queue of all their macros in descending degree.  The rest of
// each degree's work runs on a stream of its own (default priority), forked
// from the caller's stream with an event and joined back with one event per
// degree, so the small groups overlap the large ones and the whole FP64 step
// can be captured in one HIP graph.
//
// Device memory.  A context holds its bordered matrices and coefficients for
// every macro it owns (about 300 MB per macro at p = 4).  When the groups
// together would exceed the batch's workspace budget, the groups with the
// largest macros are streamed: their context holds one wave of macros and
// is pointed at successive slices of the group (mesh sizes, wall flags and
// status codes in device arrays of the batch), assembling and condensing one
// wave after the other on the group's stream.  Their factors cannot all be
// kept, so recovering such a group assembles and factors each wave again
// from the same inputs (the same kernels on the same data: the same bits)
// before the back-substitution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/mehdg.h"
#include "batch_view.hpp"

struct mehdg_batch {
    struct Group {
        int32_t p = 0;
        int64_t first = 0, count = 0;    // slice of the batch order
        int64_t wave = 0;                // macros the context holds (count unless streamed)
        mehdg_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        int64_t sz[5] = {};              // mehdg_sizes(p)
        // streamed groups only: mesh, wall flags and status of the whole group,
        // and one wave of assemble outputs for the recovery
        double* d_h = nullptr;
        uint8_t* d_bc = nullptr;
        int32_t* d_status = nullptr;
        double* d_work = nullptr;
        bool streamed() const { return wave < count; }
    };
    int64_t n_macro = 0;
    std::vector<int64_t> order;          // batch position -> macro
    std::vector<Group> groups;
    hipEvent_t fork = nullptr;
    std::vector<int32_t> h_status;
    int32_t prec = MEHDG_FP64;           // of the last condensation
    bool residual_per_degree = false;    // the residual pass per degree instead of one persistent launch
    unsigned long long* d_counter = nullptr;   // work-queue position of the persistent launch
};

namespace {

// doubles per macro of a flat array of kind key at degree sizes sz
int64_t per_macro(int32_t key, const int64_t sz[5]) {
    const int64_t n = sz[0], nf = sz[1], NH = sz[4];
    switch (key) {
        case MEHDG_KEY_V: return 5 * n;
        case MEHDG_KEY_Q: return 15 * n;
        case MEHDG_KEY_VHAT: return 30 * nf;
        case MEHDG_KEY_ENTROPY: return 1;
        case MEHDG_KEY_AHAT: return NH * NH;
        case MEHDG_KEY_BHAT: return NH;
        default: return -1;
    }
}

int64_t group_offset(const mehdg_batch* b, int32_t key, size_t gi) {
    int64_t off = 0;
    for (size_t i = 0; i < gi; ++i) off += b->groups[i].count * per_macro(key, b->groups[i].sz);
    return off;
}

// group gi's slice of a flat array, from its macro w0 on
template <typename T>
T* slice(T* base, const mehdg_batch* b, int32_t key, size_t gi, int64_t w0 = 0) {
    return base ? base + group_offset(b, key, gi) + w0 * per_macro(key, b->groups[gi].sz) : nullptr;
}

// doubles of one wave of assemble outputs (R_q, R_v, R_vhat, entropy, bhat)
int64_t work_per_macro(const int64_t sz[5]) {
    return per_macro(MEHDG_KEY_Q, sz) + per_macro(MEHDG_KEY_V, sz) + per_macro(MEHDG_KEY_VHAT, sz) + 1 +
           per_macro(MEHDG_KEY_BHAT, sz);
}

// fork the group streams from st, run f(group index) on each, join back
template <typename F>
mehdg_err fork_join(mehdg_batch* b, hipStream_t st, F&& f) {
    if (hipEventRecord(b->fork, st) != hipSuccess) return MEHDG_EHIP;
    mehdg_err first = MEHDG_OK;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        auto& g = b->groups[gi];
        if (hipStreamWaitEvent(g.stream, b->fork, 0) != hipSuccess) return MEHDG_EHIP;
        const mehdg_err e = f(gi);
        if (e != MEHDG_OK && first == MEHDG_OK) first = e;
        if (hipEventRecord(g.done, g.stream) != hipSuccess || hipStreamWaitEvent(st, g.done, 0) != hipSuccess)
            return MEHDG_EHIP;
    }
    return first;
}

// run f(w0, n) over the waves of group g, the context viewing each in turn
template <typename F>
mehdg_err over_waves(mehdg_batch::Group& g, F&& f) {
    if (!g.streamed()) return f(0, g.count);
    for (int64_t w0 = 0; w0 < g.count; w0 += g.wave) {
        const int64_t n = std::min(g.wave, g.count - w0);
        mehdg_err e = mehdg_batch_ctx_view(g.ctx, n, g.d_h + 3 * w0, g.d_bc ? g.d_bc + 6 * w0 : nullptr,
                                           g.d_status + w0);
        if (e == MEHDG_OK) e = f(w0, n);
        if (e != MEHDG_OK) {
            (void)mehdg_batch_ctx_unview(g.ctx);
            return e;
        }
    }
    return MEHDG_OK;
}

// Wave sizes: whole groups while the budget allows, else the groups with the
// largest macros shrink first, each to what the budget leaves it.
void size_waves(std::vector<mehdg_batch::Group>& groups, int64_t budget) {
    std::vector<int64_t> bytes(groups.size());
    int64_t total = 0;
    for (size_t i = 0; i < groups.size(); ++i) {
        bytes[i] = mehdg_batch_ctx_bytes(groups[i].p);
        groups[i].wave = groups[i].count;
        total += groups[i].count * bytes[i];
    }
    std::vector<size_t> idx(groups.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t c) { return bytes[a] > bytes[c]; });
    for (size_t i : idx) {
        if (total <= budget) break;
        auto& g = groups[i];
        const int64_t rest = total - g.count * bytes[i];
        int64_t w = (budget - rest) / bytes[i];
        w = std::max<int64_t>(1, std::min(w, g.count));
        total = rest + w * bytes[i];
        g.wave = w;
    }
}

}  // namespace

extern "C" {

mehdg_err mehdg_batch_destroy(mehdg_batch* b) {
    if (!b) return MEHDG_EINVAL;
    for (auto& g : b->groups) {
        if (g.ctx) mehdg_destroy(g.ctx);
        if (g.done) (void)hipEventDestroy(g.done);
        if (g.stream) (void)hipStreamDestroy(g.stream);
        (void)hipFree(g.d_h);
        (void)hipFree(g.d_bc);
        (void)hipFree(g.d_status);
        (void)hipFree(g.d_work);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    (void)hipFree(b->d_counter);
    delete b;
    return MEHDG_OK;
}

mehdg_err mehdg_batch_create(const mehdg_batch_mesh* mesh, const mehdg_params* prm, mehdg_batch** out) {
    if (!out) return MEHDG_EINVAL;
    *out = nullptr;
    if (!mesh || !prm || !mesh->p || !mesh->h || mesh->n_macro <= 0 || mesh->max_workspace_bytes < 0 ||
        mesh->residual_per_degree < 0 || mesh->residual_per_degree > 1)
        return MEHDG_EINVAL;
    const int64_t M = mesh->n_macro;
    for (int64_t i = 0; i < M; ++i) {
        int64_t sz[5];
        if (mehdg_sizes(mesh->p[i], sz) != MEHDG_OK) return MEHDG_EINVAL;
    }
    mehdg_batch* b = new (std::nothrow) mehdg_batch();
    if (!b) return MEHDG_ENOMEM;
    b->n_macro = M;
    b->order.resize((size_t)M);
    for (int64_t i = 0; i < M; ++i) b->order[(size_t)i] = i;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int64_t a, int64_t c) { return mesh->p[a] < mesh->p[c]; });
    b->h_status.assign((size_t)M, 0);
    b->residual_per_degree = mesh->residual_per_degree != 0;
    for (int64_t first = 0; first < M;) {
        mehdg_batch::Group g;
        g.p = mesh->p[b->order[(size_t)first]];
        g.first = first;
        while (first + g.count < M && mesh->p[b->order[(size_t)(first + g.count)]] == g.p) ++g.count;
        (void)mehdg_sizes(g.p, g.sz);
        b->groups.push_back(g);
        first += g.count;
    }
    int64_t budget = mesh->max_workspace_bytes;
    if (budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            mehdg_batch_destroy(b);
            return MEHDG_EHIP;
        }
        budget = (int64_t)(0.6 * (double)free_b);
    }
    size_waves(b->groups, budget);
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&b->d_counter, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        mehdg_batch_destroy(b);
        return MEHDG_EHIP;
    }
    for (auto& g : b->groups) {
        // the context's own mesh: the group's first wave (a streamed group
        // points it at each wave in turn)
        std::vector<double> h((size_t)(3 * g.count));
        std::vector<uint8_t> bc(mesh->face_bc ? (size_t)(6 * g.count) : 0);
        bool walls = false;
        for (int64_t i = 0; i < g.count; ++i) {
            const int64_t m = b->order[(size_t)(g.first + i)];
            for (int k = 0; k < 3; ++k) h[(size_t)(3 * i + k)] = mesh->h[3 * m + k];
            if (mesh->face_bc)
                for (int k = 0; k < 6; ++k) {
                    bc[(size_t)(6 * i + k)] = mesh->face_bc[6 * m + k];
                    walls = walls || mesh->face_bc[6 * m + k] != 0;
                }
        }
        mehdg_err e = MEHDG_OK;
        for (size_t i = 0; i < bc.size(); ++i)
            if (bc[i] > 1) e = MEHDG_EINVAL;
        if (walls && !(prm->T_wall > 0.0)) e = MEHDG_EINVAL;
        mehdg_mesh sub{};
        sub.n_macro = g.wave;
        sub.p = g.p;
        sub.h = h.data();
        sub.face_bc = walls ? bc.data() : nullptr;
        if (e == MEHDG_OK) e = mehdg_create(&sub, prm, &g.ctx);
        if (e == MEHDG_OK && (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
                              hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess))
            e = MEHDG_EHIP;
        if (e == MEHDG_OK && g.streamed()) {
            const int64_t wk = g.wave * work_per_macro(g.sz);
            if (hipMalloc(&g.d_h, sizeof(double) * 3 * g.count) != hipSuccess ||
                hipMalloc(&g.d_status, sizeof(int32_t) * g.count) != hipSuccess ||
                hipMalloc(&g.d_work, sizeof(double) * wk) != hipSuccess ||
                (walls && hipMalloc(&g.d_bc, 6 * g.count) != hipSuccess))
                e = MEHDG_ENOMEM;
            else if (hipMemcpy(g.d_h, h.data(), sizeof(double) * 3 * g.count, hipMemcpyHostToDevice) != hipSuccess ||
                     hipMemset(g.d_status, 0, sizeof(int32_t) * g.count) != hipSuccess ||
                     (walls && hipMemcpy(g.d_bc, bc.data(), 6 * g.count, hipMemcpyHostToDevice) != hipSuccess))
                e = MEHDG_EHIP;
        }
        if (e != MEHDG_OK) {
            (void)hipGetLastError();
            mehdg_batch_destroy(b);
            return e;
        }
    }
    *out = b;
    return MEHDG_OK;
}

mehdg_err mehdg_batch_layout(const mehdg_batch* b, int32_t key, int64_t* order, int64_t* offsets) {
    if (!b || key < 0 || key >= MEHDG_NKEYS) return MEHDG_EINVAL;
    if (order)
        for (int64_t i = 0; i < b->n_macro; ++i) order[i] = b->order[(size_t)i];
    if (offsets) {
        int64_t off = 0, pos = 0;
        for (const auto& g : b->groups) {
            const int64_t per = per_macro(key, g.sz);
            for (int64_t i = 0; i < g.count; ++i, ++pos) {
                offsets[pos] = off;
                off += per;
            }
        }
        offsets[pos] = off;
    }
    return MEHDG_OK;
}

mehdg_err mehdg_batch_groups(const mehdg_batch* b, int32_t* n_groups, int32_t* degree, int64_t* first,
                             int64_t* count, int64_t* wave) {
    if (!b || !n_groups) return MEHDG_EINVAL;
    *n_groups = (int32_t)b->groups.size();
    for (size_t i = 0; i < b->groups.size(); ++i) {
        if (degree) degree[i] = b->groups[i].p;
        if (first) first[i] = b->groups[i].first;
        if (count) count[i] = b->groups[i].count;
        if (wave) wave[i] = b->groups[i].wave;
    }
    return MEHDG_OK;
}

mehdg_err mehdg_batch_assemble_condense(mehdg_batch* b, int32_t prec, const double* v, const double* vhat,
                                        const double* v_old, double* R_q, double* R_v, double* R_vhat,
                                        double* entropy, double* Ahat, double* bhat, mehdg_stream stream) {
    if (!b || !v || !vhat || !v_old || !R_q || !R_v || !R_vhat || !entropy || !bhat) return MEHDG_EINVAL;
    if (prec < MEHDG_FP64 || prec > MEHDG_BF16_IR) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    b->prec = prec;
    std::vector<mehdg_batch_slices> sl(b->groups.size());
    for (size_t gi = 0; gi < b->groups.size(); ++gi)
        sl[gi] = mehdg_batch_slices{slice(v, b, MEHDG_KEY_V, gi), slice(vhat, b, MEHDG_KEY_VHAT, gi),
                                    slice(v_old, b, MEHDG_KEY_V, gi), slice(R_q, b, MEHDG_KEY_Q, gi),
                                    slice(R_v, b, MEHDG_KEY_V, gi), slice(R_vhat, b, MEHDG_KEY_VHAT, gi),
                                    slice(entropy, b, MEHDG_KEY_ENTROPY, gi)};
    // the residual pass of the whole groups: one persistent launch on the caller's stream
    std::vector<char> joint(b->groups.size(), 0);
    if (!b->residual_per_degree) {
        std::vector<mehdg_ctx*> ctxs;
        std::vector<mehdg_batch_slices> jsl;
        for (size_t gi = 0; gi < b->groups.size(); ++gi)
            if (!b->groups[gi].streamed()) {
                ctxs.push_back(b->groups[gi].ctx);
                jsl.push_back(sl[gi]);
                joint[gi] = 1;
            }
        if (!ctxs.empty()) {
            const mehdg_err e =
                mehdg_batch_ctx_residual(ctxs.data(), jsl.data(), (int)ctxs.size(), b->d_counter, stream);
            if (e != MEHDG_OK) return e;
        }
    }
    return fork_join(b, st, [&](size_t gi) -> mehdg_err {
        auto& g = b->groups[gi];
        mehdg_stream gs = reinterpret_cast<mehdg_stream>(g.stream);
        if (joint[gi]) {
            const mehdg_err e = mehdg_batch_ctx_rows(g.ctx, &sl[gi], gs);
            if (e != MEHDG_OK) return e;
            return mehdg_condense(g.ctx, prec, slice(Ahat, b, MEHDG_KEY_AHAT, gi), slice(bhat, b, MEHDG_KEY_BHAT, gi),
                                  gs);
        }
        return over_waves(g, [&](int64_t w0, int64_t) -> mehdg_err {
            mehdg_err e = mehdg_assemble(g.ctx, slice(v, b, MEHDG_KEY_V, gi, w0), slice(vhat, b, MEHDG_KEY_VHAT, gi, w0),
                                         nullptr, slice(v_old, b, MEHDG_KEY_V, gi, w0),
                                         slice(R_q, b, MEHDG_KEY_Q, gi, w0), slice(R_v, b, MEHDG_KEY_V, gi, w0),
                                         slice(R_vhat, b, MEHDG_KEY_VHAT, gi, w0),
                                         slice(entropy, b, MEHDG_KEY_ENTROPY, gi, w0), 1, gs);
            if (e != MEHDG_OK) return e;
            return mehdg_condense(g.ctx, prec, slice(Ahat, b, MEHDG_KEY_AHAT, gi, w0),
                                  slice(bhat, b, MEHDG_KEY_BHAT, gi, w0), gs);
        });
    });
}

mehdg_err mehdg_batch_recover(mehdg_batch* b, const double* v, const double* vhat, const double* v_old,
                              const double* R_q, const double* dvhat, double* dv, double* dq, mehdg_stream stream) {
    if (!b || !R_q || !dvhat || !dv || !dq) return MEHDG_EINVAL;
    for (const auto& g : b->groups)
        if (g.streamed() && (!v || !vhat || !v_old)) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return fork_join(b, st, [&](size_t gi) -> mehdg_err {
        auto& g = b->groups[gi];
        mehdg_stream gs = reinterpret_cast<mehdg_stream>(g.stream);
        if (!g.streamed())
            return mehdg_recover(g.ctx, slice(R_q, b, MEHDG_KEY_Q, gi), slice(dvhat, b, MEHDG_KEY_VHAT, gi),
                                 slice(dv, b, MEHDG_KEY_V, gi), slice(dq, b, MEHDG_KEY_Q, gi), gs);
        // one wave of assemble outputs in the batch's work array
        double* wq = g.d_work;
        double* wv = wq + g.wave * per_macro(MEHDG_KEY_Q, g.sz);
        double* wvh = wv + g.wave * per_macro(MEHDG_KEY_V, g.sz);
        double* went = wvh + g.wave * per_macro(MEHDG_KEY_VHAT, g.sz);
        double* wb = went + g.wave;
        return over_waves(g, [&](int64_t w0, int64_t) -> mehdg_err {
            mehdg_err e = mehdg_assemble(g.ctx, slice(v, b, MEHDG_KEY_V, gi, w0), slice(vhat, b, MEHDG_KEY_VHAT, gi, w0),
                                         nullptr, slice(v_old, b, MEHDG_KEY_V, gi, w0), wq, wv, wvh, went, 1, gs);
            if (e == MEHDG_OK) e = mehdg_condense(g.ctx, b->prec, nullptr, wb, gs);
            if (e == MEHDG_OK)
                e = mehdg_recover(g.ctx, wq, slice(dvhat, b, MEHDG_KEY_VHAT, gi, w0), slice(dv, b, MEHDG_KEY_V, gi, w0),
                                  slice(dq, b, MEHDG_KEY_Q, gi, w0), gs);
            return e;
        });
    });
}

mehdg_err mehdg_batch_status(mehdg_batch* b, int32_t* status, mehdg_stream stream) {
    if (!b || !status) return MEHDG_EINVAL;
    (void)stream;
    for (const auto& g : b->groups) {
        int32_t* hs = b->h_status.data() + g.first;
        if (g.streamed()) {
            if (hipStreamSynchronize(g.stream) != hipSuccess ||
                hipMemcpy(hs, g.d_status, sizeof(int32_t) * g.count, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemset(g.d_status, 0, sizeof(int32_t) * g.count) != hipSuccess)
                return MEHDG_EHIP;
        } else {
            const mehdg_err e = mehdg_status(g.ctx, hs, reinterpret_cast<mehdg_stream>(g.stream));
            if (e == MEHDG_EINVAL || e == MEHDG_EHIP) return e;
        }
        for (int64_t i = 0; i < g.count; ++i) status[b->order[(size_t)(g.first + i)]] = hs[i];
    }
    for (int64_t m = 0; m < b->n_macro; ++m)
        if (status[m] != 0) return static_cast<mehdg_err>(status[m]);
    return MEHDG_OK;
}

}  // extern "C"
