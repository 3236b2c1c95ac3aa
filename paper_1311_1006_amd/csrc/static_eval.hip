// static_eval.hip -- the evaluation of fmm_evaluate with its working buffers
// in a fixed device array, for callers that cannot allocate device memory.
//
// The buffers an evaluation writes and reads back (strengths in tree order,
// the near-field source records, the near-field sums, the multipole and
// local coefficients, and the partial sums of lists split into work chunks)
// are carved out of `scratch`, a file-scope device array of kStaticBytes
// bytes.  Every GPU holds its own copy at its own address, taken once per
// device with hipGetSymbolAddress; host code uses that address only.  The
// kernels are the ones fmm_evaluate runs.  Calls on one GPU share its array,
// so calls that overlap on one GPU race; the array keeps the last call's
// contents, and nothing here needs it cleared (every buffer is written in
// full before it is read: the gather covers every point, P2P every target,
// P2M and M2M every box's multipole, M2L every box's local expansion).
#include <mutex>

#include "fmm_internal.h"
#include "plan_extra.h"

namespace fmm {

constexpr size_t kStaticBytes = size_t(64) << 20;
constexpr size_t kStaticAlign = 256;
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// the device address of `scratch` on `device` (the current device), taken
// on the first call there
static unsigned char* scratch_ptr(int device)
{
    static std::mutex mu;
    static unsigned char* ptr[kStaticMaxDevices] = {};
    if (device < 0 || device >= kStaticMaxDevices) throw Error(FMM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            throw Error(FMM_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        ptr[device] = static_cast<unsigned char*>(p);
    }
    return ptr[device];
}

namespace {

// points one plan buffer at a slice of the array for the length of a call
struct Slot {
    void* buf;                        // the DBuf
    void (*set)(void* buf, void* p);  // sets its pointer
    void* saved;                      // its own allocation
    size_t bytes;
};

template <class T>
void set_ptr(void* buf, void* p)
{
    static_cast<DBuf<T>*>(buf)->p = static_cast<T*>(p);
}

template <class T>
void add(std::vector<Slot>& v, DBuf<T>& b)
{
    if (b.p) v.push_back(Slot{&b, &set_ptr<T>, b.p, b.bytes()});
}

struct Swap {
    std::vector<Slot> slots;
    ~Swap()
    {
        for (auto& s : slots) s.set(s.buf, s.saved);
    }
};

}  // namespace

// Bytes of the array the evaluation of `pl` needs (each buffer rounded up
// to kStaticAlign).
size_t static_eval_bytes(Plan& pl)
{
    std::vector<Slot> v;
    add(v, pl.mtree);
    add(v, pl.near);
    add(v, pl.mpole);
    add(v, pl.local);
    add(v, pl.bal.partial);
    add(v, pl.bal_m2l.partial);
    size_t need = 0;
    for (auto& s : v) need += (s.bytes + kStaticAlign - 1) / kStaticAlign * kStaticAlign;
    return need;
}

// fmm_evaluate's evaluation on `s` with the working buffers in the array.
// The plan must be final (its lists built, split into chunks where needed);
// the plan's own buffers and its forward state (used by the adjoint) are
// left as they were.
void evaluate_static(Plan& pl, const double* m, double* phi, hipStream_t s)
{
    if (!pl.finalized)
        throw Error(FMM_ESTATE, "the plan's lists are not final yet: evaluate it once with fmm_evaluate, or call "
                                "fmm_plan_stats, before fmm_evaluate_static");
    int dev = -1;
    FMM_HIP(hipGetDevice(&dev));
    if (dev != pl.tree->device) throw Error(FMM_EINVAL, "fmm_evaluate_static must run on the tree's device");
    const size_t need = static_eval_bytes(pl);
    if (need > kStaticBytes)
        throw Error(FMM_EINVAL, "fmm_evaluate_static: the evaluation needs " + std::to_string(need) +
                                    " bytes of working memory, more than the fixed " +
                                    std::to_string(kStaticBytes) + " bytes");
    unsigned char* base = scratch_ptr(dev);
    Swap sw;
    add(sw.slots, pl.mtree);
    add(sw.slots, pl.near);
    add(sw.slots, pl.mpole);
    add(sw.slots, pl.local);
    add(sw.slots, pl.bal.partial);
    add(sw.slots, pl.bal_m2l.partial);
    size_t off = 0;
    for (auto& sl : sw.slots) {
        sl.set(sl.buf, base + off);
        off += (sl.bytes + kStaticAlign - 1) / kStaticAlign * kStaticAlign;
    }
    const bool had_forward = pl.have_forward;
    const int flags = pl.tune.flags;
    pl.tune.flags &= ~(FMM_FLAG_GRAPH | FMM_FLAG_PHASE_TIMING);
    try {
        evaluate_device(pl, m, phi, nullptr, nullptr, s, nullptr, nullptr);
    } catch (...) {
        pl.tune.flags = flags;
        pl.have_forward = had_forward;
        throw;
    }
    pl.tune.flags = flags;
    pl.have_forward = had_forward;
}

}  // namespace fmm
