// Macro-elements of mixed polynomial degree and boundary type in one call
// (the batch entry points of mehdg.h).
//
// The kernels are compiled per degree, so a batch keeps one context per
// degree present.  The macros are ordered by degree (stable), and every
// per-macro array of the batch is flat in that order: the macros of one
// degree are one contiguous slice, which that degree's context reads and
// writes in place (no copies).  Each degree runs on a stream of its own
// (default priority), forked from the caller's stream with an event and
// joined back with one event per degree, so the small groups overlap the
// large ones and the whole FP64 step can be captured in one HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/mehdg.h"

struct mehdg_batch {
    struct Group {
        int32_t p = 0;
        int64_t first = 0, count = 0;   // slice of the batch order
        mehdg_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        int64_t sz[5] = {};              // mehdg_sizes(p)
    };
    int64_t n_macro = 0;
    std::vector<int64_t> order;          // batch position -> macro
    std::vector<Group> groups;
    hipEvent_t fork = nullptr;
    std::vector<int32_t> h_status;
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

template <typename T>
T* slice(T* base, const mehdg_batch* b, int32_t key, size_t gi) {
    return base ? base + group_offset(b, key, gi) : nullptr;
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

}  // namespace

extern "C" {

mehdg_err mehdg_batch_destroy(mehdg_batch* b) {
    if (!b) return MEHDG_EINVAL;
    for (auto& g : b->groups) {
        if (g.ctx) mehdg_destroy(g.ctx);
        if (g.done) (void)hipEventDestroy(g.done);
        if (g.stream) (void)hipStreamDestroy(g.stream);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
    return MEHDG_OK;
}

mehdg_err mehdg_batch_create(const mehdg_batch_mesh* mesh, const mehdg_params* prm, mehdg_batch** out) {
    if (!out) return MEHDG_EINVAL;
    *out = nullptr;
    if (!mesh || !prm || !mesh->p || !mesh->h || mesh->n_macro <= 0) return MEHDG_EINVAL;
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
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
        mehdg_batch_destroy(b);
        return MEHDG_EHIP;
    }
    for (int64_t first = 0; first < M;) {
        const int32_t p = mesh->p[b->order[(size_t)first]];
        int64_t cnt = 0;
        while (first + cnt < M && mesh->p[b->order[(size_t)(first + cnt)]] == p) ++cnt;
        std::vector<double> h((size_t)(3 * cnt));
        std::vector<uint8_t> bc(mesh->face_bc ? (size_t)(6 * cnt) : 0);
        for (int64_t i = 0; i < cnt; ++i) {
            const int64_t m = b->order[(size_t)(first + i)];
            for (int k = 0; k < 3; ++k) h[(size_t)(3 * i + k)] = mesh->h[3 * m + k];
            if (mesh->face_bc)
                for (int k = 0; k < 6; ++k) bc[(size_t)(6 * i + k)] = mesh->face_bc[6 * m + k];
        }
        mehdg_mesh sub{};
        sub.n_macro = cnt;
        sub.p = p;
        sub.h = h.data();
        sub.face_bc = mesh->face_bc ? bc.data() : nullptr;
        mehdg_batch::Group g;
        g.p = p;
        g.first = first;
        g.count = cnt;
        (void)mehdg_sizes(p, g.sz);
        mehdg_err e = mehdg_create(&sub, prm, &g.ctx);
        if (e == MEHDG_OK && (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
                              hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess))
            e = MEHDG_EHIP;
        b->groups.push_back(g);
        if (e != MEHDG_OK) {
            mehdg_batch_destroy(b);
            return e;
        }
        first += cnt;
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
                             int64_t* count) {
    if (!b || !n_groups) return MEHDG_EINVAL;
    *n_groups = (int32_t)b->groups.size();
    for (size_t i = 0; i < b->groups.size(); ++i) {
        if (degree) degree[i] = b->groups[i].p;
        if (first) first[i] = b->groups[i].first;
        if (count) count[i] = b->groups[i].count;
    }
    return MEHDG_OK;
}

mehdg_err mehdg_batch_assemble_condense(mehdg_batch* b, int32_t prec, const double* v, const double* vhat,
                                        const double* v_old, double* R_q, double* R_v, double* R_vhat,
                                        double* entropy, double* Ahat, double* bhat, mehdg_stream stream) {
    if (!b || !v || !vhat || !v_old || !R_q || !R_v || !R_vhat || !entropy || !bhat) return MEHDG_EINVAL;
    if (prec < MEHDG_FP64 || prec > MEHDG_BF16_IR) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return fork_join(b, st, [&](size_t gi) -> mehdg_err {
        auto& g = b->groups[gi];
        mehdg_stream gs = reinterpret_cast<mehdg_stream>(g.stream);
        mehdg_err e = mehdg_assemble(g.ctx, slice(v, b, MEHDG_KEY_V, gi), slice(vhat, b, MEHDG_KEY_VHAT, gi),
                                     nullptr, slice(v_old, b, MEHDG_KEY_V, gi), slice(R_q, b, MEHDG_KEY_Q, gi),
                                     slice(R_v, b, MEHDG_KEY_V, gi), slice(R_vhat, b, MEHDG_KEY_VHAT, gi),
                                     slice(entropy, b, MEHDG_KEY_ENTROPY, gi), 1, gs);
        if (e != MEHDG_OK) return e;
        return mehdg_condense(g.ctx, prec, slice(Ahat, b, MEHDG_KEY_AHAT, gi), slice(bhat, b, MEHDG_KEY_BHAT, gi),
                              gs);
    });
}

mehdg_err mehdg_batch_recover(mehdg_batch* b, const double* R_q, const double* dvhat, double* dv, double* dq,
                              mehdg_stream stream) {
    if (!b || !R_q || !dvhat || !dv || !dq) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return fork_join(b, st, [&](size_t gi) -> mehdg_err {
        auto& g = b->groups[gi];
        return mehdg_recover(g.ctx, slice(R_q, b, MEHDG_KEY_Q, gi), slice(dvhat, b, MEHDG_KEY_VHAT, gi),
                             slice(dv, b, MEHDG_KEY_V, gi), slice(dq, b, MEHDG_KEY_Q, gi),
                             reinterpret_cast<mehdg_stream>(g.stream));
    });
}

mehdg_err mehdg_batch_status(mehdg_batch* b, int32_t* status, mehdg_stream stream) {
    if (!b || !status) return MEHDG_EINVAL;
    (void)stream;
    mehdg_err first = MEHDG_OK;
    for (const auto& g : b->groups) {
        const mehdg_err e = mehdg_status(g.ctx, b->h_status.data() + g.first,
                                         reinterpret_cast<mehdg_stream>(g.stream));
        if (e == MEHDG_EINVAL || e == MEHDG_EHIP) return e;
        for (int64_t i = 0; i < g.count; ++i) status[b->order[(size_t)(g.first + i)]] = b->h_status[(size_t)(g.first + i)];
    }
    for (int64_t m = 0; m < b->n_macro; ++m)
        if (status[m] != 0) {
            first = static_cast<mehdg_err>(status[m]);
            break;
        }
    return first;
}

}  // extern "C"
