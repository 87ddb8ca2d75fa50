// Datatype table and typemap compiler.
//
// A datatype is MPI's typemap (list of basic entries and byte displacements)
// built by contiguous / vector / indexed from one basic type.  The compiler
// keeps the typemap of one element as byte segments in packed order and
// reduces it to one of two forms the copy kernels read:
//   REG  nblk blocks of blen bytes, block i at first + i * stride
//        (a basic type, contiguous, a vector of dense blocks, any indexed
//        type whose blocks turn out evenly spaced);
//   SEG  an explicit segment list (anything else), uploaded at commit into
//        device memory with the packed prefix of every segment.
// Composition never expands a REG layout unless the result is irregular, so
// vectors with millions of blocks stay O(1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <numeric>
#include <vector>

#include "runtime.h"

namespace mpixs {

namespace {

constexpr int64_t kMaxSegs = int64_t(1) << 24;
// granules of one element a segment-lookup table may map (16 MiB of table)
constexpr int64_t kMaxLut = int64_t(1) << 22;

// Handles index a fixed table that only grows; lookups take no lock (the
// enqueue path looks a datatype up on every call, from every rank thread).
constexpr int32_t kMaxTypes = 1 << 20;
std::mutex g_types_mu;                       // serialises creation and free
std::atomic<TypeObj *> *g_types = nullptr;   // kMaxTypes slots
std::atomic<int32_t> g_ntypes{64};           // handles below 64 are reserved

int64_t gcd64(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

void finish_reg(Layout &L) {
    if (L.nblk == 0 || L.blen == 0) {
        L.nblk = 0;
        L.blen = 0;
        L.stride = 0;
        L.first = 0;
        L.size = 0;
        L.lb = L.ub = L.extent = 0;
        L.overlap = false;
        L.gcd = 0;
        return;
    }
    if (L.nblk > 1 && L.stride == L.blen) {      // blocks touch: one dense block
        L.blen *= L.nblk;
        L.nblk = 1;
    }
    if (L.nblk == 1) L.stride = L.blen;
    const int64_t last = L.first + (L.nblk - 1) * L.stride;
    L.lb = std::min(L.first, last);
    L.ub = std::max(L.first, last) + L.blen;
    L.extent = L.ub - L.lb;
    L.size = L.nblk * L.blen;
    const int64_t as = L.stride < 0 ? -L.stride : L.stride;
    L.overlap = L.nblk > 1 && as < L.blen;
    L.gcd = gcd64(gcd64(L.first, L.blen), L.nblk > 1 ? L.stride : 0);
}

// Adopt a segment list: merge touching neighbours, then reduce to REG when
// the segments are evenly spaced blocks of one length.
void finish_seg(Layout &L, std::vector<std::pair<int64_t, int64_t>> segs) {
    std::vector<std::pair<int64_t, int64_t>> m;
    m.reserve(segs.size());
    for (auto &s : segs) {
        if (s.second == 0) continue;
        if (!m.empty() && m.back().first + m.back().second == s.first)
            m.back().second += s.second;
        else
            m.push_back(s);
    }
    L.segs.clear();
    if (m.empty()) {
        L.reg = true;
        L.nblk = 0;
        finish_reg(L);
        return;
    }
    bool regular = true;
    const int64_t len = m[0].second;
    const int64_t step = m.size() > 1 ? m[1].first - m[0].first : len;
    for (size_t i = 1; i < m.size() && regular; ++i)
        regular = m[i].second == len && m[i].first - m[i - 1].first == step;
    if (regular) {
        L.reg = true;
        L.nblk = int64_t(m.size());
        L.blen = len;
        L.stride = step;
        L.first = m[0].first;
        finish_reg(L);
        return;
    }
    L.reg = false;
    int64_t lb = m[0].first, ub = m[0].first + m[0].second, size = 0, g = 0;
    for (auto &s : m) {
        lb = std::min(lb, s.first);
        ub = std::max(ub, s.first + s.second);
        size += s.second;
        g = gcd64(gcd64(g, s.first), s.second);
    }
    L.lb = lb;
    L.ub = ub;
    L.extent = ub - lb;
    L.size = size;
    L.gcd = g;
    std::vector<std::pair<int64_t, int64_t>> sorted = m;
    std::sort(sorted.begin(), sorted.end());
    L.overlap = false;
    for (size_t i = 1; i < sorted.size(); ++i)
        if (sorted[i].first < sorted[i - 1].first + sorted[i - 1].second) L.overlap = true;
    L.segs = std::move(m);
}

bool expand(const Layout &T, std::vector<std::pair<int64_t, int64_t>> &out, int64_t shift,
            int64_t &budget) {
    if (T.reg) {
        if (T.nblk > budget) return false;
        budget -= T.nblk;
        for (int64_t i = 0; i < T.nblk; ++i) out.emplace_back(shift + T.first + i * T.stride, T.blen);
    } else {
        if (int64_t(T.segs.size()) > budget) return false;
        budget -= int64_t(T.segs.size());
        for (auto &s : T.segs) out.emplace_back(shift + s.first, s.second);
    }
    return true;
}

// n copies of T, copy i shifted by i * step bytes.
int hrepeat(int64_t n, int64_t step, const Layout &T, Layout &R) {
    R = Layout();
    R.basic = T.basic;
    R.esize = T.esize;
    if (n == 0 || T.size == 0) {
        R.reg = true;
        R.nblk = 0;
        finish_reg(R);
        return MPIXS_SUCCESS;
    }
    if (T.reg && T.nblk == 1) {
        R.reg = true;
        R.nblk = n;
        R.blen = T.blen;
        R.stride = step;
        R.first = T.first;
        finish_reg(R);
        return MPIXS_SUCCESS;
    }
    if (T.reg && step == T.nblk * T.stride) {
        R.reg = true;
        R.nblk = n * T.nblk;
        R.blen = T.blen;
        R.stride = T.stride;
        R.first = T.first;
        finish_reg(R);
        return MPIXS_SUCCESS;
    }
    std::vector<std::pair<int64_t, int64_t>> segs;
    int64_t budget = kMaxSegs;
    for (int64_t i = 0; i < n; ++i)
        if (!expand(T, segs, i * step, budget)) return MPIXS_ERR_NOMEM;
    finish_seg(R, std::move(segs));
    return MPIXS_SUCCESS;
}

std::atomic<TypeObj *> *types_table() {
    static std::atomic<TypeObj *> *tab = [] {
        auto *p = new std::atomic<TypeObj *>[kMaxTypes];
        for (int32_t i = 0; i < kMaxTypes; ++i) p[i].store(nullptr, std::memory_order_relaxed);
        return p;
    }();
    return tab;
}

int add_type(TypeObj *t, mpixs_datatype *out) {
    std::lock_guard<std::mutex> g(g_types_mu);
    g_types = types_table();
    const int32_t id = g_ntypes.load(std::memory_order_relaxed);
    if (id >= kMaxTypes) return MPIXS_ERR_NOMEM;
    g_types[id].store(t, std::memory_order_release);
    g_ntypes.store(id + 1, std::memory_order_release);
    *out = mpixs_datatype(id);
    return MPIXS_SUCCESS;
}

TypeObj *predefined(int basic) {
    static TypeObj basics[7];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int b = 1; b <= 6; ++b) {
            TypeObj &t = basics[b];
            t.predefined = true;
            t.committed = true;
            t.L.basic = b;
            t.L.esize = basic_size(b);
            t.L.reg = true;
            t.L.nblk = 1;
            t.L.blen = t.L.esize;
            t.L.first = 0;
            finish_reg(t.L);
        }
    });
    return &basics[basic];
}

TypeObj *any_type(mpixs_datatype dt) {
    if (dt >= 1 && dt <= 6) return predefined(dt);
    if (dt < 64 || dt >= g_ntypes.load(std::memory_order_acquire)) return nullptr;
    return types_table()[dt].load(std::memory_order_acquire);
}

int make_derived(const Layout &L, mpixs_datatype *newtype) {
    if (!newtype) return MPIXS_ERR_ARG;
    TypeObj *t = new TypeObj();
    t->L = L;
    return add_type(t, newtype);
}

}  // namespace

int basic_size(int basic) {
    switch (basic) {
    case MPIXS_UINT8:
    case MPIXS_INT8: return 1;
    case MPIXS_INT32:
    case MPIXS_FLOAT32: return 4;
    case MPIXS_INT64:
    case MPIXS_FLOAT64: return 8;
    default: return 0;
    }
}

const TypeObj *type_lookup(mpixs_datatype dt) {
    const TypeObj *t = any_type(dt);
    return (t && t->committed) ? t : nullptr;
}

const TypeObj *type_any(mpixs_datatype dt) { return any_type(dt); }

// Granule table of a SEG layout: the packed bytes of one element in
// granules of the largest power of two (<= 16) dividing every segment
// length, each mapped to the index of its segment -- one load instead of a
// binary search.  Any copy unit divides the segment lengths, so no unit
// straddles a granule.  False for elements of more than kMaxLut granules
// (they keep the search).
bool seg_lut(const Layout &L, std::vector<uint32_t> *lut, uint32_t *shift) {
    int64_t gl = 0;
    for (const auto &sg : L.segs) gl = gcd64(gl, sg.second);
    uint32_t s = 0;
    while (s < 4 && gl > 0 && ((gl >> s) & 1) == 0) ++s;
    const int64_t ngran = L.size >> s;
    if (ngran <= 0 || ngran > kMaxLut) return false;
    lut->assign(static_cast<size_t>(ngran), 0);
    int64_t pre = 0;
    for (size_t i = 0; i < L.segs.size(); ++i) {
        for (int64_t b = pre >> s; b < (pre + L.segs[i].second) >> s; ++b)
            (*lut)[size_t(b)] = uint32_t(i);
        pre += L.segs[i].second;
    }
    *shift = s;
    return true;
}

}  // namespace mpixs

using namespace mpixs;

extern "C" {

int mpixs_type_contiguous(int count, mpixs_datatype oldtype, mpixs_datatype *newtype) {
    const TypeObj *o = any_type(oldtype);
    if (!o) return MPIXS_ERR_TYPE;
    if (count < 0) return MPIXS_ERR_COUNT;
    Layout R;
    int rc = hrepeat(count, o->L.extent, o->L, R);
    if (rc) return rc;
    return make_derived(R, newtype);
}

int mpixs_type_vector(int count, int blocklength, int stride, mpixs_datatype oldtype,
                      mpixs_datatype *newtype) {
    const TypeObj *o = any_type(oldtype);
    if (!o) return MPIXS_ERR_TYPE;
    if (count < 0 || blocklength < 0) return MPIXS_ERR_COUNT;
    if (stride < 0) return MPIXS_ERR_TYPE;
    Layout block, R;
    int rc = hrepeat(blocklength, o->L.extent, o->L, block);
    if (rc) return rc;
    if (blocklength == 0 || o->L.size == 0) {
        rc = hrepeat(0, 0, block, R);
    } else {
        rc = hrepeat(count, int64_t(stride) * o->L.extent, block, R);
    }
    if (rc) return rc;
    return make_derived(R, newtype);
}

int mpixs_type_indexed(int count, const int blocklengths[], const int displacements[],
                       mpixs_datatype oldtype, mpixs_datatype *newtype) {
    const TypeObj *o = any_type(oldtype);
    if (!o) return MPIXS_ERR_TYPE;
    if (count < 0) return MPIXS_ERR_COUNT;
    if (count > 0 && (!blocklengths || !displacements)) return MPIXS_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        if (blocklengths[i] < 0) return MPIXS_ERR_COUNT;
        if (displacements[i] < 0) return MPIXS_ERR_TYPE;
    }
    std::vector<std::pair<int64_t, int64_t>> segs;
    int64_t budget = kMaxSegs;
    for (int i = 0; i < count; ++i) {
        Layout block;
        int rc = hrepeat(blocklengths[i], o->L.extent, o->L, block);
        if (rc) return rc;
        if (!expand(block, segs, int64_t(displacements[i]) * o->L.extent, budget))
            return MPIXS_ERR_NOMEM;
    }
    Layout R;
    R.basic = o->L.basic;
    R.esize = o->L.esize;
    finish_seg(R, std::move(segs));
    return make_derived(R, newtype);
}

int mpixs_type_commit(mpixs_datatype *type) {
    if (!type) return MPIXS_ERR_ARG;
    TypeObj *t = any_type(*type);
    if (!t) return MPIXS_ERR_TYPE;
    if (t->committed) return MPIXS_SUCCESS;
    if (!t->L.reg) {
        // the copy kernels binary-search the table for every unit, so it
        // lives in device memory (cached in L2), not in host memory
        const int64_t n = int64_t(t->L.segs.size());
        std::vector<SegEnt> host(static_cast<size_t>(n));
        int64_t pre = 0;
        for (int64_t i = 0; i < n; ++i) {
            host[size_t(i)].off = t->L.segs[size_t(i)].first;
            host[size_t(i)].pre = pre;
            pre += t->L.segs[size_t(i)].second;
        }
        SegEnt *tab = nullptr;
        if (hipMalloc(reinterpret_cast<void **>(&tab), size_t(n) * sizeof(SegEnt)) != hipSuccess)
            return MPIXS_ERR_NOMEM;
        if (hipMemcpy(tab, host.data(), size_t(n) * sizeof(SegEnt), hipMemcpyHostToDevice) !=
            hipSuccess) {
            (void)hipFree(tab);
            return MPIXS_ERR_GPU;
        }
        t->table = tab;
        t->nseg = n;
        std::vector<uint32_t> lut;
        uint32_t shift = 0;
        if (seg_lut(t->L, &lut, &shift)) {
            uint32_t *d = nullptr;
            const size_t nb = lut.size() * sizeof(uint32_t);
            if (hipMalloc(reinterpret_cast<void **>(&d), nb) == hipSuccess &&
                hipMemcpy(d, lut.data(), nb, hipMemcpyHostToDevice) == hipSuccess) {
                t->lut = d;
                t->lut_shift = shift;
            } else if (d) {
                (void)hipFree(d);   // the search still works without it
            }
        }
    }
    t->committed = true;
    return MPIXS_SUCCESS;
}

int mpixs_type_free(mpixs_datatype *type) {
    if (!type) return MPIXS_ERR_ARG;
    if (*type >= 1 && *type <= 6) return MPIXS_ERR_TYPE;
    std::lock_guard<std::mutex> g(g_types_mu);
    if (*type < 64 || *type >= g_ntypes.load() || !types_table()[*type].load()) return MPIXS_ERR_TYPE;
    // The object and its tables stay allocated: enqueued operations may still
    // read them, and freeing device memory can synchronise the device.
    types_table()[*type].store(nullptr, std::memory_order_release);
    *type = MPIXS_DATATYPE_NULL;
    return MPIXS_SUCCESS;
}

int mpixs_type_size(mpixs_datatype type, int64_t *bytes) {
    const TypeObj *t = any_type(type);
    if (!t) return MPIXS_ERR_TYPE;
    if (!bytes) return MPIXS_ERR_ARG;
    *bytes = t->L.size;
    return MPIXS_SUCCESS;
}

int mpixs_type_get_extent(mpixs_datatype type, int64_t *lb, int64_t *extent) {
    const TypeObj *t = any_type(type);
    if (!t) return MPIXS_ERR_TYPE;
    if (lb) *lb = t->L.lb;
    if (extent) *extent = t->L.extent;
    return MPIXS_SUCCESS;
}

}  // extern "C"
