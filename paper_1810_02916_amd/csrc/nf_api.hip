// nf_api.hip -- host side of the C ABI declared in include/nf.h: argument
// validation, workspace layout, descriptor upload and kernel dispatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nf.h"
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {
namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

// Descriptor bytes travel as a kernel argument (no host-to-device memcpy), so
// every call is a pure sequence of kernel launches.
constexpr int kChunkBytes = 2048;
struct Chunk {
    unsigned char bytes[kChunkBytes];
};

__global__ void k_put_bytes(Chunk c, unsigned char *dst, int nbytes) {
    for (int i = threadIdx.x; i < nbytes; i += blockDim.x) dst[i] = c.bytes[i];
}

hipError_t upload(const void *src, size_t nbytes, void *dst, hipStream_t s) {
    const unsigned char *p = static_cast<const unsigned char *>(src);
    unsigned char *d = static_cast<unsigned char *>(dst);
    for (size_t o = 0; o < nbytes; o += kChunkBytes) {
        Chunk c;
        int m = (int)std::min<size_t>(kChunkBytes, nbytes - o);
        std::memcpy(c.bytes, p + o, (size_t)m);
        hipLaunchKernelGGL(k_put_bytes, dim3(1), dim3(256), 0, s, c, d + o, m);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


// Device architecture check, cached per device.
std::mutex g_dev_mu;
std::vector<int> g_dev_ok;   // -1 unknown, 0 no, 1 yes

int check_device(std::string &why) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        why = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return NF_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((int)g_dev_ok.size() <= dev) g_dev_ok.resize(dev + 1, -1);
    if (g_dev_ok[dev] < 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) {
            why = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
            return NF_EHIP;
        }
        g_dev_ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
        if (!g_dev_ok[dev]) why = std::string("device is ") + prop.gcnArchName + ", not gfx950";
    }
    if (!g_dev_ok[dev]) {
        if (why.empty()) why = "device is not gfx950";
        return NF_EUNSUPPORTED;
    }
    return NF_OK;
}

// Validated sizes of a call.
struct Layout {
    int64_t N = 0, C = 0, max_n = 0, max_ncell = 0;
    std::vector<int64_t> base, cellbase;
    // workspace byte offsets
    size_t table_off = 0, table_bytes = 0;
    size_t keys_off[2] = {0, 0}, vals_off[2] = {0, 0};
    size_t hist_off = 0, cellcnt_off = 0, scan_off = 0;
    size_t cot_off = 0, cellinfo_off = 0, bucket_off = 0, totals_off = 0, dense_off = 0,
           light_off = 0, counter_off = 0;
    size_t stepio_off = 0, cellstat_off = 0, partial_off = 0, partstat_off = 0;
    size_t mp_base_off = 0, mp_first_off = 0, mp_first_bytes = 0;
    size_t mp_npieces_off = 0, mp_scan_off = 0, mp_pieces_off = 0, mp_partial_off = 0;
    int64_t mp_max_pieces = 0;
    int64_t max_dense = 0;
    size_t accel_end = 0;   // bytes an accelerations call uses (table + planner)
    // pair symmetry (flag NF_PAIR_SYMMETRIC), after the planner's tables
    size_t f4P_off = 0, f4nf_off = 0, f4slot_off = 0, f4item_cnt_off = 0, f4scan_off = 0,
           f4tot_off = 0, f4items_off = 0, f4part_off = 0, f4blk_off = 0;
    uint32_t f4cap_slots = 0, f4cap_items = 0;
    size_t total = 0;
    int64_t nblk = 0;
    int passes = 0;
    int radix_bits = 8;
    size_t offc_off = 0;
    int light_window = kDefaultLightWindow, narrow_window = kDefaultNarrowWindow;
};

int validate(int nbox, const nf_box *boxes, Layout &L, uint32_t flags = 0) {
    if (nbox < 1 || nbox > NF_MAX_BOXES)
        return fail(NF_EINVAL, "nbox must be in [1, NF_MAX_BOXES]");
    if (!boxes) return fail(NF_EINVAL, "boxes is NULL");
    L.base.resize(nbox);
    L.cellbase.resize(nbox);
    for (int b = 0; b < nbox; ++b) {
        const nf_box &B = boxes[b];
        char where[64];
        std::snprintf(where, sizeof where, "box %d: ", b);
        if (B.n < 0) return fail(NF_EINVAL, std::string(where) + "n < 0");
        if (B.K < 5) return fail(NF_EINVAL, std::string(where) + "K < 5 (the 5x5x5 block would alias)");
        if (!(B.L > 0) || !std::isfinite(B.L)) return fail(NF_EINVAL, std::string(where) + "L must be finite and > 0");
        if (!(B.eps_s > 0) || !std::isfinite(B.eps_s))
            return fail(NF_EINVAL, std::string(where) + "eps_s must be finite and > 0");
        const int64_t ncell = (int64_t)B.K * B.K * B.K;
        if (ncell + 1 > INT32_MAX) return fail(NF_EUNSUPPORTED, std::string(where) + "K^3 + 1 exceeds 2^31 - 1");
        if (B.n > INT32_MAX) return fail(NF_EUNSUPPORTED, std::string(where) + "n exceeds 2^31 - 1");
        if (!B.cell_start) return fail(NF_EINVAL, std::string(where) + "cell_start is NULL");
        if (B.dense_min != 0 && (B.dense_min < 2 || B.dense_min > 65))
            return fail(NF_EINVAL, std::string(where) + "dense_min must be 0 or in [2, 65]");
        if (B.narrow_max < 0 || B.narrow_max > 64)
            return fail(NF_EINVAL, std::string(where) + "narrow_max must be 0 or in [1, 64]");
        if (B.flush < 0 || B.flush > 256)
            return fail(NF_EINVAL, std::string(where) + "flush must be 0 or in [1, 256]");
        const int lw = B.light_window ? B.light_window : kDefaultLightWindow;
        const int nw = B.narrow_window ? B.narrow_window : kDefaultNarrowWindow;
        if (lw != 512 && lw != 1024 && lw != 2048)
            return fail(NF_EINVAL, std::string(where) + "light_window must be 0, 512, 1024 or 2048");
        if (nw != 128 && nw != 256 && nw != 512)
            return fail(NF_EINVAL, std::string(where) + "narrow_window must be 0, 128, 256 or 512");
        if (b == 0) {
            L.light_window = lw;
            L.narrow_window = nw;
        } else if (lw != L.light_window || nw != L.narrow_window) {
            return fail(NF_EINVAL, std::string(where) +
                                       "light_window and narrow_window must agree across the "
                                       "boxes of a call");
        }
        if (B.n > 0 && (!B.off || !B.order))
            return fail(NF_EINVAL, std::string(where) + "off/order is NULL");
        const double kappa = (double)B.K / B.L;
        if (!std::isfinite(kappa) || !std::isfinite(B.eps_s * kappa) || !(B.eps_s * kappa > 0))
            return fail(NF_EINVAL, std::string(where) + "K/L or eps_s*K/L is not a positive finite number");
        L.base[b] = L.N;
        L.cellbase[b] = L.C;
        L.N += B.n;
        L.C += ncell;
        L.max_n = std::max<int64_t>(L.max_n, B.n);
        // a cell of n sinks gives at most n / min(dense_min, 64) dense chunks
        const int dm = B.dense_min ? B.dense_min : kDefaultDenseMin;
        L.max_dense += B.n / std::min(dm, 64) + 1;
        L.max_ncell = std::max<int64_t>(L.max_ncell, ncell);
    }
    if (L.N > INT32_MAX) return fail(NF_EUNSUPPORTED, "total particles over all boxes exceed 2^31 - 1");
    if (L.C + 1 > INT32_MAX) return fail(NF_EUNSUPPORTED, "total cells over all boxes exceed 2^31 - 2");
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < L.C) ++bits;
    // 8-bit digits, or 9 when that saves a pass (18-bit keys: 2 passes, not 3)
    L.radix_bits = (bits + 8) / 9 < (bits + 7) / 8 ? 9 : 8;
    L.passes = (bits + L.radix_bits - 1) / L.radix_bits;
    L.nblk = std::max<int64_t>(1, (L.N + kSortTile - 1) / kSortTile);

    size_t o = 0;
    L.table_off = o;
    L.table_bytes = sizeof(DevBox) * (size_t)nbox;
    o = align_up(o + L.table_bytes, 256);
    const size_t scratch0 = o;
    for (int k = 0; k < 2; ++k) {
        L.keys_off[k] = o;
        o = align_up(o + 4 * (size_t)L.N, 256);
        L.vals_off[k] = o;
        o = align_up(o + 4 * (size_t)L.N, 256);
    }
    L.offc_off = o;
    o = align_up(o + 16 * (size_t)L.N, 256);
    L.hist_off = o;
    o = align_up(o + 4 * (size_t)(1 << L.radix_bits) * (size_t)L.nblk, 256);
    L.cellcnt_off = o;
    o = align_up(o + 4 * (size_t)(L.C + 1), 256);
    L.scan_off = o;
    const int64_t scan_words =
        std::max(scan_scratch_words((int64_t)(1 << L.radix_bits) * L.nblk),
                 scan_scratch_words(L.C + 1));
    o = align_up(o + 4 * (size_t)scan_words, 256);
    const size_t bin_end = o;
    // force scratch reuses the binning scratch region: the planner's tables
    // first, then the VJP's source records
    o = scratch0;
    L.cellinfo_off = o;
    o = align_up(o + 4 * (size_t)L.C, 256);
    L.bucket_off = o;
    o = align_up(o + 4 * 2 * (size_t)plan_buckets(), 256);
    L.totals_off = o;
    o = align_up(o + 16, 256);
    // dense items: at most max_dense (counted per box above); light: <= 1 per cell
    L.max_dense += 16;
    L.dense_off = o;
    o = align_up(o + sizeof(Item) * (size_t)L.max_dense, 256);
    L.light_off = o;
    o = align_up(o + sizeof(Item) * (size_t)(L.C + 16), 256);
    L.counter_off = o;
    o = align_up(o + 4 * (size_t)queue_words(), 256);
    L.accel_end = o;
    L.cot_off = o;   // VJP source records: 32 bytes per particle
    o = align_up(o + 32 * (size_t)L.N, 256);
    size_t force_end = o;
    if (flags & NF_PAIR_SYMMETRIC) {   // accelerations only: overlaps the VJP records
        if (L.N > ((int64_t)1 << 27))   // keeps 16 N + 65536 partial slots in 32 bits
            return fail(NF_EUNSUPPORTED, "NF_PAIR_SYMMETRIC supports up to 2^27 particles");
        L.f4cap_slots = (uint32_t)(16 * L.N + 65536);
        L.f4cap_items = (uint32_t)(L.N / 8 + 1024);
        o = L.accel_end;
        L.f4P_off = o;
        o = align_up(o + 4 * (size_t)L.C, 256);
        L.f4nf_off = o;
        o = align_up(o + 4 * (size_t)L.C, 256);
        L.f4slot_off = o;
        o = align_up(o + 4 * (size_t)(L.C + 1), 256);
        L.f4item_cnt_off = o;
        o = align_up(o + 4 * (size_t)(L.C + 1), 256);
        L.f4scan_off = o;
        o = align_up(o + 4 * (size_t)scan_scratch_words(L.C + 1), 256);
        L.f4tot_off = o;
        o = align_up(o + 16, 256);
        L.f4blk_off = o;   // 2 x 8 bytes per block of 256 cells of every box
        o = align_up(o + 16 * (size_t)(nbox * ((L.max_ncell + 255) / 256) + 1), 256);
        L.f4items_off = o;
        o = align_up(o + sizeof(PairItem) * (size_t)L.f4cap_items, 256);
        L.f4part_off = o;
        o = align_up(o + 2 * sizeof(float4) * (size_t)L.f4cap_slots, 256);
        force_end = std::max(force_end, o);
    }
    // step-statistics scratch, also over the binning scratch region
    o = scratch0;
    L.stepio_off = o;
    o = align_up(o + sizeof(StepIO) * (size_t)nbox, 256);
    L.cellstat_off = o;
    o = align_up(o + sizeof(CellStat) * (size_t)L.C, 256);
    L.partial_off = o;
    o = align_up(o + sizeof(CellStat) * (size_t)kStepBlocks * (size_t)nbox, 256);
    L.partstat_off = o;
    o = align_up(o + sizeof(PartStat) * (size_t)L.N, 256);
    const size_t step_end = o;
    // multipole partition, also over the binning scratch region
    o = scratch0;
    L.mp_base_off = o;
    o = align_up(o + 8 * ((size_t)nbox + 1), 256);
    L.mp_first_off = o;
    int64_t nranges = 0;
    for (int b = 0; b < nbox; ++b)
        nranges += multipole_ranges(boxes[b].n, (int64_t)boxes[b].K * boxes[b].K * boxes[b].K) + 1;
    L.mp_first_bytes = 4 * (size_t)nranges;
    o = align_up(o + L.mp_first_bytes, 256);
    // cells cut into pieces: counts then offsets, scan scratch, pieces, and
    // the pieces' double moments at the largest order
    L.mp_npieces_off = o;
    o = align_up(o + 4 * (size_t)(L.C + 1), 256);
    L.mp_scan_off = o;
    o = align_up(o + 4 * (size_t)scan_scratch_words(L.C + 1), 256);
    for (int b = 0; b < nbox; ++b) L.mp_max_pieces += multipole_max_pieces(boxes[b].n);
    L.mp_pieces_off = o;
    o = align_up(o + sizeof(MpPiece) * (size_t)L.mp_max_pieces, 256);
    L.mp_partial_off = o;
    o = align_up(o + 8 * (size_t)multipole_terms(multipole_max_order()) * (size_t)L.mp_max_pieces,
                 256);
    L.total = std::max(std::max(std::max(bin_end, force_end), step_end), o);
    return NF_OK;
}

int check_ws(const Layout &L, void *ws, size_t ws_bytes) {
    if (!ws) return fail(NF_EWORKSPACE, "workspace is NULL");
    if (ws_bytes < L.total) {
        char m[128];
        std::snprintf(m, sizeof m, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return fail(NF_EWORKSPACE, m);
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(NF_EWORKSPACE, "workspace must be 256-byte aligned");
    return NF_OK;
}

void fill_geometry(const nf_box &B, const Layout &L, int b, DevBox &d, bool plummer = false,
                   bool no_shortcut = false) {
    std::memset(&d, 0, sizeof d);
    d.n = (int32_t)B.n;
    d.K = B.K;
    d.ncell = B.K * B.K * B.K;
    d.base = L.base[b];
    d.cellbase = L.cellbase[b];
    d.kappa = (double)B.K / B.L;
    d.cellw = B.L / (double)B.K;
    const double eps = B.eps_s * d.kappa;
    d.eps = (float)eps;
    d.cA = (float)(10.0 / (eps * eps * eps));
    d.cB = (float)(-15.0 / (eps * eps * eps * eps));
    d.cC = (float)(6.0 / (eps * eps * eps * eps * eps));
    d.outer_newton = (eps <= 1.0 && !no_shortcut) ? 1 : 0;
    d.plummer = plummer ? 1 : 0;
    d.r2floor = plummer ? (float)(eps * eps) : kR2Floor;
    d.dense_min = B.dense_min ? B.dense_min : kDefaultDenseMin;
    d.narrow_max = B.narrow_max ? B.narrow_max : kDefaultNarrowMax;
    d.flush = B.flush ? B.flush : kDefaultFlush;
    d.pos = B.pos;
    d.off = reinterpret_cast<float4 *>(B.off);
    d.cell_start = B.cell_start;
    d.order = B.order;
    d.nbad = B.nbad;
}

}  // namespace
}  // namespace nf

// Scratch of the allocation-free accelerations (nf_accel_noalloc): one array
// per GPU, held from the library's load on that GPU until the process ends.
// Host code never uses the name `scratch` as an address (on the host it is a
// stand-in, not device memory): every use goes through the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[NF_NOALLOC_SCRATCH_BYTES];

namespace nf {
namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // per device: device address of `scratch`

// Device address of the current device's `scratch`, looked up once per device
// (with that device current) and kept.
int static_scratch(void *&ptr, std::string &why) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        why = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return NF_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return NF_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    ptr = g_scratch_ptr[dev];
    return NF_OK;
}

}  // namespace
}  // namespace nf

using namespace nf;

extern "C" {

int nf_version(void) { return NF_ABI_VERSION; }

const char *nf_strerror(int status) {
    switch (status) {
        case NF_OK: return "success";
        case NF_EINVAL: return "invalid argument";
        case NF_EWORKSPACE: return "workspace missing or too small";
        case NF_EHIP: return "HIP runtime error";
        case NF_EUNSUPPORTED: return "unsupported size or device";
        default: return "unknown status";
    }
}

const char *nf_last_error(void) { return g_last_error.c_str(); }

size_t nf_workspace_bytes(int nbox, const nf_box *boxes, uint32_t flags) {
    try {
        Layout L;
        if (validate(nbox, boxes, L, flags) != NF_OK) return 0;
        g_last_error.clear();
        return L.total;
    } catch (...) {
        fail(NF_EINVAL, "internal error");
        return 0;
    }
}

int nf_bin_particles(int nbox, const nf_box *boxes, void *ws, size_t ws_bytes, void *stream) {
    try {
        Layout L;
        int rc = validate(nbox, boxes, L);
        if (rc) return rc;
        for (int b = 0; b < nbox; ++b)
            if (boxes[b].n > 0 && !boxes[b].pos) return fail(NF_EINVAL, "pos is NULL");
        if ((rc = check_ws(L, ws, ws_bytes))) return rc;
        std::string why;
        if ((rc = check_device(why))) return fail(rc, why);
        std::vector<DevBox> tab((size_t)nbox);
        for (int b = 0; b < nbox; ++b) fill_geometry(boxes[b], L, b, tab[b]);
        hipStream_t s = static_cast<hipStream_t>(stream);
        char *w = static_cast<char *>(ws);
        DevBox *d_tab = reinterpret_cast<DevBox *>(w + L.table_off);
        hipError_t e = upload(tab.data(), sizeof(DevBox) * tab.size(), d_tab, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("upload: ") + hipGetErrorString(e));
        BinPlan p;
        p.N = L.N;
        p.C = L.C;
        p.max_n = L.max_n;
        p.max_ncell = L.max_ncell;
        p.nblk = L.nblk;
        p.passes = L.passes;
        p.radix_bits = L.radix_bits;
        for (int k = 0; k < 2; ++k) {
            p.sc.keys[k] = reinterpret_cast<uint32_t *>(w + L.keys_off[k]);
            p.sc.vals[k] = reinterpret_cast<uint32_t *>(w + L.vals_off[k]);
        }
        p.sc.offc = reinterpret_cast<float4 *>(w + L.offc_off);
        p.sc.hist = reinterpret_cast<uint32_t *>(w + L.hist_off);
        p.sc.cellcnt = reinterpret_cast<uint32_t *>(w + L.cellcnt_off);
        p.scan_scratch = reinterpret_cast<uint32_t *>(w + L.scan_off);
        e = bin_launch(d_tab, nbox, p, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("bin launch: ") + hipGetErrorString(e));
        g_last_error.clear();
        return NF_OK;
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}


// noalloc: the workspace is the static `scratch` array of the current device
// (ws and ws_bytes are ignored), and the force kernels run one after another
// on the caller's stream (no library side streams or events).
// The planner's tables inside the workspace.
static TilePlan tile_plan(const Layout &L, char *w) {
    TilePlan tp;
    tp.TG = L.C;
    tp.max_cells = L.max_ncell;
    tp.cellinfo = reinterpret_cast<uint32_t *>(w + L.cellinfo_off);
    tp.bucket_cnt = reinterpret_cast<uint32_t *>(w + L.bucket_off);
    tp.bucket_off = tp.bucket_cnt + plan_buckets();
    tp.totals = reinterpret_cast<uint32_t *>(w + L.totals_off);
    tp.dense = reinterpret_cast<Item *>(w + L.dense_off);
    tp.light = reinterpret_cast<Item *>(w + L.light_off);
    tp.counter = reinterpret_cast<uint32_t *>(w + L.counter_off);
    tp.light_window = L.light_window;
    tp.narrow_window = L.narrow_window;
    return tp;
}

static int force_common(int nbox, const nf_box *boxes, double gm, uint32_t flags,
                        const float *const *cot, float *const *out, void *ws, size_t ws_bytes,
                        void *stream, bool vjp, bool noalloc = false) {
    if (flags & ~(uint32_t)(NF_COMPENSATED | NF_SIMPLE | NF_PLUMMER | NF_SPLINE_EVERYWHERE |
                            NF_SERIAL | NF_PAIR_SYMMETRIC))
        return fail(NF_EINVAL, "unknown flag bits");
    const bool f4 = (flags & NF_PAIR_SYMMETRIC) != 0;
    if (f4 && vjp) return fail(NF_EINVAL, "NF_PAIR_SYMMETRIC applies to nf_accel only");
    if (f4 && (flags & NF_SIMPLE)) return fail(NF_EINVAL, "NF_PAIR_SYMMETRIC excludes NF_SIMPLE");
    if (f4 && noalloc)
        return fail(NF_EUNSUPPORTED, "NF_PAIR_SYMMETRIC needs a workspace (not allocation-free)");
    Layout L;
    int rc = validate(nbox, boxes, L, f4 ? (uint32_t)NF_PAIR_SYMMETRIC : 0u);
    if (rc) return rc;
    if (!std::isfinite(gm)) return fail(NF_EINVAL, "gm must be finite");
    if (!out) return fail(NF_EINVAL, "output pointer array is NULL");
    if (vjp && !cot) return fail(NF_EINVAL, "cotangent pointer array is NULL");
    for (int b = 0; b < nbox; ++b) {
        if (boxes[b].n > 0 && !out[b]) return fail(NF_EINVAL, "output pointer is NULL");
        if (vjp && boxes[b].n > 0 && !cot[b]) return fail(NF_EINVAL, "cotangent pointer is NULL");
    }
    std::string why;
    if (noalloc) {
        if (vjp) return fail(NF_EINVAL, "internal error");
        if (L.accel_end > (size_t)NF_NOALLOC_SCRATCH_BYTES) {
            char m[160];
            std::snprintf(m, sizeof m,
                          "the call needs %zu bytes of scratch; the allocation-free entry point "
                          "holds %zu",
                          L.accel_end, (size_t)NF_NOALLOC_SCRATCH_BYTES);
            return fail(NF_EUNSUPPORTED, m);
        }
        if ((rc = check_device(why))) return fail(rc, why);
        if ((rc = static_scratch(ws, why))) return fail(rc, why);
        ws_bytes = NF_NOALLOC_SCRATCH_BYTES;
    } else {
        if ((rc = check_ws(L, ws, ws_bytes))) return rc;
        if ((rc = check_device(why))) return fail(rc, why);
    }
    char *w = static_cast<char *>(ws);
    F4Plan fp;
    const bool use_f4 = f4 && L.N > 0;
    if (use_f4) {
        fp.C = L.C;
        fp.max_cells = L.max_ncell;
        fp.P = reinterpret_cast<int32_t *>(w + L.f4P_off);
        fp.nfwd = reinterpret_cast<int32_t *>(w + L.f4nf_off);
        fp.slotoff = reinterpret_cast<uint32_t *>(w + L.f4slot_off);
        fp.itemoff = reinterpret_cast<uint32_t *>(w + L.f4item_cnt_off);
        fp.scan = reinterpret_cast<uint32_t *>(w + L.f4scan_off);
        fp.tot = reinterpret_cast<uint32_t *>(w + L.f4tot_off);
        fp.blk = reinterpret_cast<uint64_t *>(w + L.f4blk_off);
        fp.items = reinterpret_cast<PairItem *>(w + L.f4items_off);
        fp.part = reinterpret_cast<float4 *>(w + L.f4part_off);
        fp.cap_slots = L.f4cap_slots;
        fp.cap_items = L.f4cap_items;
        // the pair kernel's queue is the last kQueueStride words of the counters
        fp.counter = reinterpret_cast<uint32_t *>(w + L.counter_off) + queue_words() -
                     f4_queue_words();
    }
    std::vector<DevBox> tab((size_t)nbox);
    for (int b = 0; b < nbox; ++b) {
        fill_geometry(boxes[b], L, b, tab[b], (flags & NF_PLUMMER) != 0,
                      (flags & NF_SPLINE_EVERYWHERE) != 0);
        const double k = tab[b].kappa;
        tab[b].scale = (float)(vjp ? gm * k * k * k : gm * k * k);
        tab[b].out = out[b];
        tab[b].cot = vjp ? cot[b] : nullptr;
        if (use_f4) {
            tab[b].f4tot = fp.tot;
            tab[b].f4P = fp.P;
            tab[b].f4nf = fp.nfwd;
            tab[b].f4off = fp.slotoff;
            tab[b].f4part = fp.part;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBox *d_tab = reinterpret_cast<DevBox *>(w + L.table_off);
    hipError_t e = upload(tab.data(), sizeof(DevBox) * tab.size(), d_tab, s);
    if (e != hipSuccess) return fail(NF_EHIP, std::string("upload: ") + hipGetErrorString(e));
    ForcePlan p;
    p.max_n = L.max_n;
    p.N = L.N;
    p.compensated = (flags & NF_COMPENSATED) != 0;
    p.simple = (flags & NF_SIMPLE) != 0;
    p.cot_sorted = reinterpret_cast<float4 *>(w + L.cot_off);
    if (p.simple || L.N == 0) {
        e = vjp ? vjp_launch(d_tab, nbox, p, s) : accel_launch(d_tab, nbox, p, s);
    } else {
        const TilePlan tp = tile_plan(L, w);
        e = vjp ? gather_cot_launch(d_tab, nbox, p, s) : hipSuccess;
        if (e == hipSuccess) e = plan_launch(d_tab, nbox, tp, s);
        if (e == hipSuccess && use_f4) e = f4_plan_launch(d_tab, nbox, fp, s);
        if (e == hipSuccess)
            e = tile_launch(d_tab, vjp ? 1 : 0, p.compensated, tp, p.cot_sorted,
                            !noalloc && !(flags & NF_SERIAL), s, use_f4 ? &fp : nullptr);
        if (e == hipSuccess && use_f4) e = f4_combine_launch(d_tab, nbox, fp, p.compensated, s);
    }
    if (e != hipSuccess) return fail(NF_EHIP, std::string("force launch: ") + hipGetErrorString(e));
    g_last_error.clear();
    return NF_OK;
}

int nf_accel(int nbox, const nf_box *boxes, double gm, uint32_t flags, float *const *acc,
             void *ws, size_t ws_bytes, void *stream) {
    try {
        return force_common(nbox, boxes, gm, flags, nullptr, acc, ws, ws_bytes, stream, false);
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

int nf_accel_noalloc(int nbox, const nf_box *boxes, double gm, uint32_t flags,
                     float *const *acc, void *stream) {
    try {
        return force_common(nbox, boxes, gm, flags, nullptr, acc, nullptr, 0, stream, false,
                            true);
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

int nf_accel_vjp(int nbox, const nf_box *boxes, double gm, uint32_t flags,
                 const float *const *cot, float *const *grad, void *ws, size_t ws_bytes,
                 void *stream) {
    try {
        return force_common(nbox, boxes, gm, flags, cot, grad, ws, ws_bytes, stream, true);
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

int nf_plan_items(int nbox, const nf_box *boxes, int32_t *items, int64_t max_items,
                  int64_t *counts, void *ws, size_t ws_bytes, void *stream) {
    try {
        Layout L;
        int rc = validate(nbox, boxes, L);
        if (rc) return rc;
        if (!counts) return fail(NF_EINVAL, "counts is NULL");
        if (max_items < 0) return fail(NF_EINVAL, "max_items < 0");
        if (max_items > 0 && !items) return fail(NF_EINVAL, "items is NULL");
        if ((rc = check_ws(L, ws, ws_bytes))) return rc;
        std::string why;
        if ((rc = check_device(why))) return fail(rc, why);
        char *w = static_cast<char *>(ws);
        std::vector<DevBox> tab((size_t)nbox);
        for (int b = 0; b < nbox; ++b) fill_geometry(boxes[b], L, b, tab[b]);
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBox *d_tab = reinterpret_cast<DevBox *>(w + L.table_off);
        hipError_t e = upload(tab.data(), sizeof(DevBox) * tab.size(), d_tab, s);
        const TilePlan tp = tile_plan(L, w);
        if (e == hipSuccess) e = plan_launch(d_tab, nbox, tp, s);
        if (e == hipSuccess) e = plan_export_launch(tp, items, max_items, counts, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("plan launch: ") + hipGetErrorString(e));
        g_last_error.clear();
        return NF_OK;
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

// Validation, descriptor and StepIO upload shared by the two stepping calls.
static int step_common(int nbox, const nf_box *boxes, const std::vector<StepIO> &io, void *ws,
                       size_t ws_bytes, hipStream_t s, Layout &L, DevBox *&d_tab,
                       StepIO *&d_io) {
    if ((int)io.size() != nbox) return fail(NF_EINVAL, "internal error");
    int rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    std::string why;
    if ((rc = check_device(why))) return fail(rc, why);
    std::vector<DevBox> tab((size_t)nbox);
    for (int b = 0; b < nbox; ++b) fill_geometry(boxes[b], L, b, tab[b]);
    char *w = static_cast<char *>(ws);
    d_tab = reinterpret_cast<DevBox *>(w + L.table_off);
    d_io = reinterpret_cast<StepIO *>(w + L.stepio_off);
    hipError_t e = upload(tab.data(), sizeof(DevBox) * tab.size(), d_tab, s);
    if (e == hipSuccess) e = upload(io.data(), sizeof(StepIO) * io.size(), d_io, s);
    if (e != hipSuccess) return fail(NF_EHIP, std::string("upload: ") + hipGetErrorString(e));
    return NF_OK;
}

int nf_step_stats(int nbox, const nf_box *boxes, const float *const *acc,
                  const float *const *vel, float *const *amax, float *const *vrms, double *glob,
                  void *ws, size_t ws_bytes, void *stream) {
    try {
        Layout L;
        int rc = validate(nbox, boxes, L);
        if (rc) return rc;
        if (!acc || !vel || !amax || !vrms || !glob)
            return fail(NF_EINVAL, "acc, vel, amax, vrms and glob must not be NULL");
        std::vector<StepIO> io((size_t)nbox);
        for (int b = 0; b < nbox; ++b) {
            if (boxes[b].n > 0 && (!acc[b] || !vel[b]))
                return fail(NF_EINVAL, "acc/vel pointer is NULL");
            if (!amax[b] || !vrms[b]) return fail(NF_EINVAL, "amax/vrms pointer is NULL");
            io[b] = StepIO{acc[b], vel[b], nullptr, nullptr, amax[b], vrms[b], nullptr, nullptr};
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBox *d_tab = nullptr;
        StepIO *d_io = nullptr;
        if ((rc = step_common(nbox, boxes, io, ws, ws_bytes, s, L, d_tab, d_io))) return rc;
        char *w = static_cast<char *>(ws);
        hipError_t e = step_stats_launch(d_tab, d_io, nbox, L.max_n, L.max_ncell,
                                         reinterpret_cast<PartStat *>(w + L.partstat_off),
                                         reinterpret_cast<CellStat *>(w + L.cellstat_off),
                                         reinterpret_cast<CellStat *>(w + L.partial_off), glob, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("step stats: ") + hipGetErrorString(e));
        g_last_error.clear();
        return NF_OK;
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

int nf_step_choose(int nbox, const nf_box *boxes, const float *const *amax,
                   const float *const *vrms, const double *glob, double dlna_max, double hubble,
                   double eta, double *bounds, void *ws, size_t ws_bytes, void *stream) {
    try {
        Layout L;
        int rc = validate(nbox, boxes, L);
        if (rc) return rc;
        if (!amax || !vrms || !glob || !bounds)
            return fail(NF_EINVAL, "amax, vrms, glob and bounds must not be NULL");
        if (!(dlna_max > 0) || !std::isfinite(dlna_max) || !(hubble > 0) ||
            !std::isfinite(hubble) || !(eta > 0) || !std::isfinite(eta))
            return fail(NF_EINVAL, "dlna_max, hubble and eta must be finite and > 0");
        std::vector<StepIO> io((size_t)nbox);
        for (int b = 0; b < nbox; ++b) {
            if (!amax[b] || !vrms[b]) return fail(NF_EINVAL, "amax/vrms pointer is NULL");
            io[b] = StepIO{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, amax[b], vrms[b]};
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBox *d_tab = nullptr;
        StepIO *d_io = nullptr;
        if ((rc = step_common(nbox, boxes, io, ws, ws_bytes, s, L, d_tab, d_io))) return rc;
        char *w = static_cast<char *>(ws);
        const StepChoice ch{dlna_max, hubble, eta};
        hipError_t e = step_choose_launch(d_tab, d_io, nbox,
                                          reinterpret_cast<double *>(w + L.partial_off), glob, ch,
                                          bounds, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("step choice: ") + hipGetErrorString(e));
        g_last_error.clear();
        return NF_OK;
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

int nf_kick_drift(int nbox, const nf_box *boxes, const float *const *acc, float *const *vel,
                  double *const *pos, double kick, double drift, void *ws, size_t ws_bytes,
                  void *stream) {
    try {
        Layout L;
        int rc = validate(nbox, boxes, L);
        if (rc) return rc;
        if (!std::isfinite(kick) || !std::isfinite(drift))
            return fail(NF_EINVAL, "kick and drift must be finite");
        if (!acc || !vel || !pos) return fail(NF_EINVAL, "acc, vel and pos must not be NULL");
        std::vector<StepIO> io((size_t)nbox);
        for (int b = 0; b < nbox; ++b) {
            if (boxes[b].n > 0 && (!acc[b] || !vel[b] || !pos[b]))
                return fail(NF_EINVAL, "acc/vel/pos pointer is NULL");
            io[b] = StepIO{acc[b], nullptr, vel[b], pos[b], nullptr, nullptr, nullptr, nullptr};
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBox *d_tab = nullptr;
        StepIO *d_io = nullptr;
        if ((rc = step_common(nbox, boxes, io, ws, ws_bytes, s, L, d_tab, d_io))) return rc;
        hipError_t e = kick_drift_launch(d_tab, d_io, nbox, L.max_n, kick, drift, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("kick/drift: ") + hipGetErrorString(e));
        g_last_error.clear();
        return NF_OK;
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

int nf_multipoles(int nbox, const nf_box *boxes, int order, float *const *mom, void *ws,
                  size_t ws_bytes, void *stream) {
    try {
        Layout L;
        int rc = validate(nbox, boxes, L);
        if (rc) return rc;
        if (order < 0 || order > NF_MAX_ORDER || order > multipole_max_order())
            return fail(NF_EINVAL, "order must be in [0, NF_MAX_ORDER]");
        if (!mom) return fail(NF_EINVAL, "moment pointer array is NULL");
        for (int b = 0; b < nbox; ++b)
            if (!mom[b]) return fail(NF_EINVAL, "moment pointer is NULL");
        if ((rc = check_ws(L, ws, ws_bytes))) return rc;
        std::string why;
        if ((rc = check_device(why))) return fail(rc, why);
        std::vector<DevBox> tab((size_t)nbox);
        std::vector<int64_t> rbase((size_t)nbox + 1, 0);
        int64_t max_ranges = 1;
        for (int b = 0; b < nbox; ++b) {
            fill_geometry(boxes[b], L, b, tab[b]);
            tab[b].out = mom[b];
            const int64_t r = multipole_ranges(boxes[b].n, (int64_t)tab[b].ncell);
            rbase[b + 1] = rbase[b] + r;
            max_ranges = std::max(max_ranges, r);
        }
        if (max_ranges > INT32_MAX || L.mp_max_pieces > INT32_MAX ||
            (size_t)(rbase[nbox] + nbox) * 4 > L.mp_first_bytes)
            return fail(NF_EUNSUPPORTED, "multipole partition exceeds the workspace plan");
        hipStream_t s = static_cast<hipStream_t>(stream);
        char *w = static_cast<char *>(ws);
        DevBox *d_tab = reinterpret_cast<DevBox *>(w + L.table_off);
        int64_t *d_rbase = reinterpret_cast<int64_t *>(w + L.mp_base_off);
        MpPlan mp;
        mp.C = L.C;
        mp.max_ncell = L.max_ncell;
        mp.max_ranges = max_ranges;
        mp.max_pieces = L.mp_max_pieces;
        mp.range_base = d_rbase;
        mp.first = reinterpret_cast<int32_t *>(w + L.mp_first_off);
        mp.npieces = reinterpret_cast<uint32_t *>(w + L.mp_npieces_off);
        mp.scan = reinterpret_cast<uint32_t *>(w + L.mp_scan_off);
        mp.pieces = reinterpret_cast<MpPiece *>(w + L.mp_pieces_off);
        mp.partial = reinterpret_cast<double *>(w + L.mp_partial_off);
        hipError_t e = upload(tab.data(), sizeof(DevBox) * tab.size(), d_tab, s);
        if (e == hipSuccess) e = upload(rbase.data(), sizeof(int64_t) * rbase.size(), d_rbase, s);
        if (e == hipSuccess) e = multipole_launch(d_tab, nbox, mp, order, s);
        if (e != hipSuccess) return fail(NF_EHIP, std::string("multipoles: ") + hipGetErrorString(e));
        g_last_error.clear();
        return NF_OK;
    } catch (...) {
        return fail(NF_EINVAL, "internal error");
    }
}

}  // extern "C"
