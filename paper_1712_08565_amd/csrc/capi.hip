// C ABI of the library (declared in include/wqfd.h): argument checks, host
// set-up, workspace carving and uploads, and dispatch to the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/wqfd.h"
#include "device.h"
#include "host_setup.h"
#include "krylov.h"

struct wq_op_s {
    wqfd::WqOp op;
};
struct fd_pc_s {
    wqfd::FdPc pc;
};
struct wq_eval_s {
    wqfd::EvalOp E;
};

namespace {

thread_local std::string g_err;
thread_local int g_ir_fallbacks = 0;       // ir_solve calls of this thread that switched to FP64 inner solves

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return WQ_EHIP;
}

#define HIP_TRY(x, where)                        \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

int nthreads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min(16u, h);
}

// Host staging of banded factors.  Variants share the window start and width.
struct HostBand {
    int rows = 0, cols = 0, L = 0;
    std::vector<int> start;
    std::vector<std::vector<double>> c;   // per variant [rows][L]
};

HostBand make_band(const std::vector<const std::vector<double>*>& mats, int rows, int cols, bool transpose) {
    // element (r, c) of the banded operator: transpose ? M[c][r] : M[r][c]
    auto at = [&](const std::vector<double>& M, int r, int c) {
        return transpose ? M[(size_t)c * rows + r] : M[(size_t)r * cols + c];
    };
    HostBand hb;
    hb.rows = rows;
    hb.cols = cols;
    std::vector<int> lo(rows, -1), hi(rows, -1);
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) {
            bool nz = false;
            for (auto* M : mats) nz |= at(*M, r, c) != 0.0;
            if (nz) {
                if (lo[r] < 0) lo[r] = c;
                hi[r] = c;
            }
        }
    int L = 1;
    for (int r = 0; r < rows; ++r)
        if (lo[r] >= 0) L = std::max(L, hi[r] - lo[r] + 1);
    L = std::min(L, cols);
    hb.L = L;
    hb.start.resize(rows);
    hb.c.assign(mats.size(), std::vector<double>((size_t)rows * L, 0.0));
    for (int r = 0; r < rows; ++r) {
        int st = lo[r] < 0 ? 0 : std::min(lo[r], cols - L);
        hb.start[r] = st;
        for (size_t v = 0; v < mats.size(); ++v)
            for (int s = 0; s < L; ++s) hb.c[v][(size_t)r * L + s] = at(*mats[v], r, st + s);
    }
    return hb;
}

// Packs host bands into one byte buffer; records offsets to patch device pointers.
struct Packer {
    std::vector<char> buf;
    size_t add(const void* p, size_t bytes) {
        size_t off = al256(buf.size());
        buf.resize(off + al256(bytes));
        std::memcpy(buf.data() + off, p, bytes);
        return off;
    }
};

template <typename T>
struct BandOffsets {
    int rows, cols, L;
    size_t start;
    std::vector<size_t> c;
};

template <typename T>
BandOffsets<T> pack_band(Packer& pk, const HostBand& hb, size_t start_off) {
    BandOffsets<T> bo;
    bo.rows = hb.rows;
    bo.cols = hb.cols;
    bo.L = hb.L;
    bo.start = start_off;
    for (auto& cv : hb.c) {
        std::vector<T> tmp(cv.begin(), cv.end());
        bo.c.push_back(pk.add(tmp.data(), tmp.size() * sizeof(T)));
    }
    return bo;
}

template <typename T>
void patch(wqfd::Band<T>* dst, const BandOffsets<T>& bo, int v, const char* base) {
    dst->rows = bo.rows;
    dst->cols = bo.cols;
    dst->L = bo.L;
    dst->start = reinterpret_cast<const int*>(base + bo.start);
    dst->c = reinterpret_cast<const T*>(base + bo.c[v]);
}

int check_knots_args(int p, const int32_t nknots[3], const double* const knots[3]) {
    if (!nknots || !knots) return fail(WQ_EINVAL, "null knot arguments");
    for (int l = 0; l < 3; ++l)
        if (!knots[l]) return fail(WQ_EINVAL, "null knot vector");
    if (p < 2 || p > wqfd::kMaxDegree) return fail(WQ_EINVAL, "degree p outside [2, 10]");
    return WQ_OK;
}

// Tables of the fused apply: dense 16 x 16 blocks of the x and y factors per
// 16-point tile and the z windows per quadrature plane (see fused.h).
struct FusedHost {
    int ntile[2] = {0, 0};
    std::vector<double> tiles[2];   // [t][6][256]
    std::vector<int> J[2], I[2];
    std::vector<int> band[2];       // [tile][16]: first nonzero (local) j of the B / B-dot rows of the tile's points
    std::vector<int> bs3, wts3;
    std::vector<double> cz;         // [nq3][2(p+1) + 4(p+2)]
    std::vector<double> czT;        // the same rows for the transposed kernel (ring slot order for p >= FUSED_RING_MIN_P)
    std::vector<int> rotT;          // [nq3][2]: transposed rings' offsets (input, output) when plane k is processed
    int zchunk = 0;
    std::vector<int> sched;         // interval records (wqfd::FusedSched), all z ranges
    std::vector<int> sched_off;     // first record of each z range, plus the total
    std::vector<int> schedT, schedT_off;   // the same for the transposed apply
};

// Length of the z range of one workgroup of the fused apply.  The grid is
// tiles x ranges workgroups; each range also pays for the p + 2 halo planes at
// its two ends, and the launch runs in ceil(workgroups / resident slots)
// rounds, so the estimated time is rounds x (zchunk / 2 + p + 3) DOF-plane
// steps.  Ranges are capped at FUSED_MAX_Z quadrature planes.
int choose_zchunk(int nq3, int tiles, int slots, int p) {
    const int zmax = wqfd::FUSED_MAX_Z;
    int best = zmax;
    long best_cost = -1;
    for (int nzc = (nq3 + zmax - 1) / zmax; nzc <= nq3; ++nzc) {
        const int zc = (nq3 + nzc - 1) / nzc;
        const long rounds = ((long)tiles * nzc + slots - 1) / slots;
        const long cost = rounds * (zc + 2 * (p + 3));          // in half DOF-plane steps
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
        if (zc <= p + 2) break;
    }
    return best;
}

// Interval schedule of the fused apply for quadrature planes k0..k1-1 (the
// pipeline described in wq_fused.hip).  Column waves: per interval up to two
// quadrature planes, at most one trial plane entering the window and one output
// plane retired, each placed before the plane that needs it.  MFMA waves, one
// interval behind: contract the plane retired in the previous interval, reduce
// the partials written in the previous interval, produce the next U plane (at
// most NU - 1 planes ahead of the window) and stage the DOF plane after it.
// Returns false if the windows do not advance by at most one plane per
// quadrature plane (the kernel then is not used).
// ins/IN: start and length of the input window of DOF planes per quadrature
// plane (forward: B3 band, p + 1; transposed: W3 band, p + 2); outs/OUT: the
// same for the output ring (forward: W3, p + 2; transposed: B3, p + 1).
bool fused_schedule(const std::vector<int>& ins, int IN, const std::vector<int>& outs, int OUT, int n3, int k0,
                    int k1, int CZ, std::vector<int>& out, std::vector<int>* rot) {
    const int RT = IN, RO = OUT, NU = 3;
    const std::vector<int>& bs3 = ins;
    const std::vector<int>& wts3 = outs;
    const int tmax = bs3[k1 - 1] + RT - 1;
    int tnext = bs3[k0], nwin = 0, tprod = tnext, tstage = tnext, obase = wts3[k0], k = k0, eflush = 0;
    int nfw = 0, nred = 0, fl_slot = 0, red_slot = 0, red_i3 = 0, fl_i3 = 0;
    bool fl_prev = false, red_prev = false;
    for (int guard = 0; guard < 8 * (k1 - k0) + 4 * (RT + RO) + 64; ++guard) {
        int nv = 0, in_at = -1, out_at = -1;
        bool done = false;
        if (nwin < RT) {
            if (tnext < tprod) in_at = 0;
        } else if (k < k1) {
            for (int j = 0; j < 2 && k + j < k1; ++j) {
                const int bk = bs3[k + j], wk = wts3[k + j];
                const bool need_in = tnext + (in_at >= 0) - RT < bk;
                const bool need_out = obase + (out_at >= 0) < wk;
                if (need_in && (in_at >= 0 || tnext >= tprod)) break;
                if (need_out && out_at >= 0) break;
                if (need_in) in_at = j;
                if (need_out) out_at = j;
                // after this plane's events the windows must sit exactly on it
                if (tnext + (in_at >= 0) - RT != bk || obase + (out_at >= 0) != wk) return false;
                ++nv;
            }
        } else if (eflush < RO) {
            out_at = 0;
        } else if (!fl_prev && !red_prev) {
            done = true;
        }
        if (done) return true;
        const bool c_in = in_at >= 0, c_out = out_at >= 0;
        const int i3 = obase;
        const bool c_wr = c_out && i3 >= 0 && i3 < n3;
        const bool m_prod = tprod < tstage && tprod - NU < tnext && tprod <= tmax;
        const bool m_stage = tstage <= tprod + 1 && tstage <= tmax;
        const int f = nv | (in_at + 1) << 2 | (out_at + 1) << 4 | int(c_wr) << 6 | int(m_prod) << 7 |
                      int(m_stage) << 8 | int(fl_prev) << 9 | int(red_prev) << 10 | (tnext % NU) << 11 |
                      (nfw & 1) << 13 | fl_slot << 14 | red_slot << 15 | (nred & 1) << 16 | (tprod & 1) << 17 |
                      (tprod % NU) << 18 | (tstage & 1) << 20;
        // column-role events per step j = 0, 1: entry, retirement, plane processed;
        // ring slots of the entry and the retirement; and, per processed plane, the
        // ring offsets: after e entries and r retirements window position s sits in
        // slots (e + s) mod IN and (r + s) mod OUT
        const int e_before = tnext - bs3[k0], r_before = obase - wts3[k0];
        int ev = (e_before % IN) << 8 | (r_before % OUT) << 12;
        for (int j = 0; j < 2; ++j) {
            ev |= (int(in_at == j) | int(out_at == j) << 1 | int(nv > j) << 2) << (3 * j);
            if (rot && nv > j) {
                (*rot)[2 * (k + j)] = (e_before + int(c_in && in_at <= j)) % IN;
                (*rot)[2 * (k + j) + 1] = (r_before + int(c_out && out_at <= j)) % OUT;
            }
        }
        const int cn0 = std::min(k + nv, k1 - 1), cn1 = std::min(k + nv + 1, k1 - 1);
        out.insert(out.end(), {f, k, red_i3, tstage, ev, (std::min(k, k1 - 1) - k0) * CZ, cn0, cn1});
        // advance
        const bool red_now = fl_prev;
        if (red_now) {
            red_slot = nred & 1;
            red_i3 = fl_i3;
            ++nred;
        }
        red_prev = red_now;
        fl_prev = c_wr;
        if (c_wr) {
            fl_slot = nfw & 1;
            fl_i3 = i3;
            ++nfw;
        }
        if (c_out) {
            ++obase;
            if (k >= k1) ++eflush;
        }
        if (c_in) {
            ++tnext;
            ++nwin;
        }
        k += nv;
        if (m_prod) ++tprod;
        if (m_stage) ++tstage;
    }
    return false;                                   // no progress: schedule rejected
}

bool build_fused_tables(const wqfd::Space1D* sp, int p, FusedHost& fh) {
    if (p > 7) return false;
    // the kernels address one coefficient plane and one vector with 32-bit
    // byte offsets (buffer loads)
    const size_t Nq_all = (size_t)sp[0].nq * sp[1].nq * sp[2].nq, N_all = (size_t)sp[0].n * sp[1].n * sp[2].n;
    if (Nq_all * sizeof(double) >= (size_t(1) << 31) || N_all * sizeof(double) >= (size_t(1) << 31)) return false;
    for (int l = 0; l < 2; ++l) {
        const wqfd::Space1D& S = sp[l];
        const int n = S.n, nq = S.nq, nt = (nq + 15) / 16;
        fh.ntile[l] = nt;
        fh.tiles[l].assign((size_t)nt * 6 * 256, 0.0);
        fh.J[l].assign(nt, 0);
        fh.I[l].assign(nt, 0);
        fh.band[l].assign((size_t)nt * 16, 0);
        const std::vector<double>* Wv[4] = {&S.W[0][0], &S.W[0][1], &S.W[1][0], &S.W[1][1]};
        for (int t = 0; t < nt; ++t) {
            const int Q = 16 * t, qe = std::min(Q + 16, nq);
            int jmin = n, jmax = -1, imin = n, imax = -1;
            for (int q = Q; q < qe; ++q)
                for (int j = 0; j < n; ++j)
                    if (S.B[0][(size_t)q * n + j] != 0.0 || S.B[1][(size_t)q * n + j] != 0.0) {
                        jmin = std::min(jmin, j);
                        jmax = std::max(jmax, j);
                    }
            for (int i = 0; i < n; ++i)
                for (int q = Q; q < qe; ++q) {
                    bool nz = false;
                    for (auto* W : Wv) nz |= (*W)[(size_t)i * nq + q] != 0.0;
                    if (nz) {
                        imin = std::min(imin, i);
                        imax = std::max(imax, i);
                    }
                }
            if (jmax < 0) jmin = jmax = 0;
            if (imax < 0) imin = imax = 0;
            if (jmax - jmin >= 16 || imax - imin >= 16) return false;
            fh.J[l][t] = jmin;
            fh.I[l][t] = imin;
            // per point: local start of the p + 1 trial functions that can be nonzero there
            for (int a = 0; a < 16; ++a) {
                const int q = Q + a;
                int lo = -1, hi = -1;
                if (q < nq)
                    for (int j = 0; j < n; ++j)
                        if (S.B[0][(size_t)q * n + j] != 0.0 || S.B[1][(size_t)q * n + j] != 0.0) {
                            if (lo < 0) lo = j;
                            hi = j;
                        }
                int st = lo < 0 ? 0 : lo - jmin;
                if (lo >= 0 && hi - lo > p) return false;   // more than p + 1 functions at one point
                st = std::max(0, std::min(st, 16 - (p + 1)));
                fh.band[l][(size_t)t * 16 + a] = st;
            }
            double* blk = &fh.tiles[l][(size_t)t * 6 * 256];
            for (int a = 0; a < 16; ++a)
                for (int b = 0; b < 16; ++b) {
                    const int q = Q + a, j = jmin + b;       // B_d[q][j]
                    if (q < nq && j < n) {
                        blk[0 * 256 + a * 16 + b] = S.B[0][(size_t)q * n + j];
                        blk[1 * 256 + a * 16 + b] = S.B[1][(size_t)q * n + j];
                    }
                    const int i = imin + a, qq = Q + b;      // W_v[i][q]
                    if (i < n && qq < nq)
                        for (int v = 0; v < 4; ++v) blk[(2 + v) * 256 + a * 16 + b] = (*Wv[v])[(size_t)i * nq + qq];
                }
        }
    }
    const wqfd::Space1D& S3 = sp[2];
    const int n3 = S3.n, nq3 = S3.nq, RT = p + 1, RO = p + 2, CZ = 2 * RT + 4 * RO;
    HostBand hB = make_band({&S3.B[0], &S3.B[1]}, nq3, n3, false);
    HostBand hWT = make_band({&S3.W[0][0], &S3.W[0][1], &S3.W[1][0], &S3.W[1][1]}, nq3, n3, true);
    if (hB.L > RT || hWT.L > RO) return false;
    fh.bs3 = hB.start;
    fh.wts3 = hWT.start;
    for (int k = 1; k < nq3; ++k)
        if (fh.bs3[k] < fh.bs3[k - 1] || fh.wts3[k] < fh.wts3[k - 1]) return false;
    fh.cz.assign((size_t)nq3 * CZ, 0.0);
    const std::vector<double>* Wv[4] = {&S3.W[0][0], &S3.W[0][1], &S3.W[1][0], &S3.W[1][1]};
    for (int k = 0; k < nq3; ++k) {
        double* c = &fh.cz[(size_t)k * CZ];
        for (int s = 0; s < RT; ++s) {
            const int j = fh.bs3[k] + s;
            if (j < n3) {
                c[s] = S3.B[0][(size_t)k * n3 + j];
                c[RT + s] = S3.B[1][(size_t)k * n3 + j];
            }
        }
        for (int v = 0; v < 4; ++v)
            for (int s = 0; s < RO; ++s) {
                const int i = fh.wts3[k] + s;
                if (i < n3) c[2 * RT + v * RO + s] = (*Wv[v])[(size_t)i * nq3 + k];
            }
    }
    // z range length from the device's resident workgroups (WQFD_ZCHUNKS fixes
    // the number of ranges), then the interval schedule of every range
    const int zmax = wqfd::FUSED_MAX_Z;
    if (const char* e = std::getenv("WQFD_ZCHUNKS")) {
        const int nzc = std::max((nq3 + zmax - 1) / zmax, std::min(nq3, std::atoi(e)));
        fh.zchunk = (nq3 + nzc - 1) / nzc;
    } else {
        int slots = 0;
        if (wqfd::fused_resident_slots(p, &slots) != hipSuccess) {
            (void)hipGetLastError();                  // no device (size query on a host): assume 256 slots
            slots = 256;
        }
        fh.zchunk = choose_zchunk(nq3, fh.ntile[0] * fh.ntile[1], slots, p);
    }
    fh.sched.clear();
    fh.rotT.assign(2 * (size_t)nq3, -1);
    fh.sched_off.clear();
    fh.schedT.clear();
    fh.schedT_off.clear();
    for (int k0 = 0; k0 < nq3; k0 += fh.zchunk) {
        const int k1 = std::min(nq3, k0 + fh.zchunk);
        fh.sched_off.push_back((int)(fh.sched.size() / wqfd::FUSED_REC));
        fh.schedT_off.push_back((int)(fh.schedT.size() / wqfd::FUSED_REC));
        if (!fused_schedule(fh.bs3, RT, fh.wts3, RO, n3, k0, k1, CZ, fh.sched, nullptr)) return false;
        if (!fused_schedule(fh.wts3, RO, fh.bs3, RT, n3, k0, k1, CZ, fh.schedT, &fh.rotT)) return false;
    }
    // transposed kernel's rows: the W rows multiply its input ring, the B rows its output ring
    fh.czT = fh.cz;
    if (p >= wqfd::FUSED_RING_MIN_P) {
        for (int x : fh.rotT)
            if (x < 0) return false;                  // a plane no range processed
        for (int k = 0; k < nq3; ++k) {
            const double* c = &fh.cz[(size_t)k * CZ];
            double* cT = &fh.czT[(size_t)k * CZ];
            const int wT = fh.rotT[2 * k], bT = fh.rotT[2 * k + 1];
            for (int d = 0; d < 2; ++d)
                for (int s = 0; s < RT; ++s) cT[d * RT + (bT + s) % RT] = c[d * RT + s];
            for (int v = 0; v < 4; ++v)
                for (int s = 0; s < RO; ++s) cT[2 * RT + v * RO + (wT + s) % RO] = c[2 * RT + v * RO + s];
        }
    }
    fh.sched_off.push_back((int)(fh.sched.size() / wqfd::FUSED_REC));
    fh.schedT_off.push_back((int)(fh.schedT.size() / wqfd::FUSED_REC));
    // the kernels hold a range's records one per lane of a wave
    for (size_t r = 0; r + 1 < fh.sched_off.size(); ++r)
        if (fh.sched_off[r + 1] - fh.sched_off[r] > 64 || fh.schedT_off[r + 1] - fh.schedT_off[r] > 64) return false;
    return true;
}

uint16_t f32_to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;                                                    // round to nearest even
    return (uint16_t)(u >> 16);
}

}  // namespace

// ---------------------------------------------------------------- allocation-free FD apply
// The intermediate buffer of fd_apply_noalloc: one file-scope device array,
// instantiated on every device the library's code object is loaded on and held
// until the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress reports, looked up once per device.
namespace {
constexpr size_t kFdNoAllocBytes = size_t(32) << 20;   // WQ_FD_NOALLOC_BYTES
constexpr int kMaxDevices = 64;
static_assert(kFdNoAllocBytes == WQ_FD_NOALLOC_BYTES, "header and library disagree on the scratch size");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kFdNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (first call per device
// looks it up with that device current).
int noalloc_scratch(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(WQ_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(WQ_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return WQ_OK;
}
}  // namespace

extern "C" {

const char* wq_last_error(void) { return g_err.c_str(); }
const char* wq_version(void) { return "wqfd 0.1 (gfx950)"; }

// wq_setup, wq_setup_nurbs and wq_setup_gauss: the same operator set-up for the
// two quadrature rules and for polynomial or rational (weights != null) maps
static int setup_impl(int rule, int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl,
                      const double* weights, int k_kind, const double* K_q, int prec_mask, void* ws, size_t ws_bytes, size_t* ws_needed,
                      wq_stream_t s_, wq_op* out) {
    g_err.clear();
    hipStream_t s = reinterpret_cast<hipStream_t>(s_);
    int rc = check_knots_args(p, nknots, knots);
    if (rc) return rc;
    if (!ctrl) return fail(WQ_EINVAL, "null control points");
    if (k_kind != WQ_K_IDENTITY && k_kind != WQ_K_SCALAR && k_kind != WQ_K_SYM6)
        return fail(WQ_EINVAL, "unknown k_kind");
    if (k_kind != WQ_K_IDENTITY && !K_q && ws) return fail(WQ_EINVAL, "K_q is required for this k_kind");
    if (prec_mask == 0 || (prec_mask & ~(WQ_F64 | WQ_F32))) return fail(WQ_EINVAL, "prec_mask must be WQ_F64 | WQ_F32");
    if (!ws && !ws_needed) return fail(WQ_EINVAL, "need ws or ws_needed");
    if (ws && !out) return fail(WQ_EINVAL, "null output handle");

    wqfd::Space1D sp[3];
    std::string err;
    for (int l = 0; l < 3; ++l) {
        rc = wqfd::build_space(p, nknots[l], knots[l], true, sp[l], err, rule);
        if (rc) return fail(rc, "direction " + std::to_string(l + 1) + ": " + err);
    }
    auto op = std::make_unique<wq_op_s>();
    wqfd::WqOp& o = op->op;
    o.p = p;
    o.prec_mask = prec_mask;
    o.k_kind = k_kind;
    for (int l = 0; l < 3; ++l) {
        o.n[l] = sp[l].n;
        o.nq[l] = sp[l].nq;
        o.xq[l] = sp[l].xq;
    }
    o.N = (size_t)o.n[0] * o.n[1] * o.n[2];
    o.Nq = (size_t)o.nq[0] * o.nq[1] * o.nq[2];

    // banded factors, both precisions
    Packer pk;
    struct DirOff {
        BandOffsets<double> B, W, BT, WT;
        BandOffsets<float> B32, W32, BT32, WT32;
    } doff[3];
    for (int l = 0; l < 3; ++l) {
        const auto& S = sp[l];
        HostBand hB = make_band({&S.B[0], &S.B[1]}, S.nq, S.n, false);
        HostBand hW = make_band({&S.W[0][0], &S.W[0][1], &S.W[1][0], &S.W[1][1]}, S.n, S.nq, false);
        HostBand hBT = make_band({&S.B[0], &S.B[1]}, S.n, S.nq, true);
        HostBand hWT = make_band({&S.W[0][0], &S.W[0][1], &S.W[1][0], &S.W[1][1]}, S.nq, S.n, true);
        const size_t sB = pk.add(hB.start.data(), hB.start.size() * sizeof(int));
        const size_t sW = pk.add(hW.start.data(), hW.start.size() * sizeof(int));
        const size_t sBT = pk.add(hBT.start.data(), hBT.start.size() * sizeof(int));
        const size_t sWT = pk.add(hWT.start.data(), hWT.start.size() * sizeof(int));
        doff[l].B = pack_band<double>(pk, hB, sB);
        doff[l].W = pack_band<double>(pk, hW, sW);
        doff[l].BT = pack_band<double>(pk, hBT, sBT);
        doff[l].WT = pack_band<double>(pk, hWT, sWT);
        doff[l].B32 = pack_band<float>(pk, hB, sB);
        doff[l].W32 = pack_band<float>(pk, hW, sW);
        doff[l].BT32 = pack_band<float>(pk, hBT, sBT);
        doff[l].WT32 = pack_band<float>(pk, hWT, sWT);
    }
    // fused-apply tables, both precisions
    FusedHost fh;
    const bool fused_ok = build_fused_tables(sp, p, fh) && !std::getenv("WQFD_STAGED");
    size_t f_tiles64[2] = {0, 0}, f_tiles32[2] = {0, 0}, f_J[2] = {0, 0}, f_I[2] = {0, 0}, f_band[2] = {0, 0};
    size_t f_bs3 = 0, f_wts3 = 0, f_cz64 = 0, f_cz32 = 0, f_czT64 = 0, f_czT32 = 0, f_sched = 0, f_soff = 0,
           f_schedT = 0, f_soffT = 0;
    if (fused_ok) {
        for (int l = 0; l < 2; ++l) {
            f_tiles64[l] = pk.add(fh.tiles[l].data(), fh.tiles[l].size() * 8);
            std::vector<float> t32(fh.tiles[l].begin(), fh.tiles[l].end());
            f_tiles32[l] = pk.add(t32.data(), t32.size() * 4);
            f_J[l] = pk.add(fh.J[l].data(), fh.J[l].size() * sizeof(int));
            f_band[l] = pk.add(fh.band[l].data(), fh.band[l].size() * sizeof(int));
            f_I[l] = pk.add(fh.I[l].data(), fh.I[l].size() * sizeof(int));
        }
        f_bs3 = pk.add(fh.bs3.data(), fh.bs3.size() * sizeof(int));
        f_wts3 = pk.add(fh.wts3.data(), fh.wts3.size() * sizeof(int));
        f_cz64 = pk.add(fh.cz.data(), fh.cz.size() * 8);
        std::vector<float> c32(fh.cz.begin(), fh.cz.end());
        f_cz32 = pk.add(c32.data(), c32.size() * 4);
        f_czT64 = pk.add(fh.czT.data(), fh.czT.size() * 8);
        std::vector<float> cT32(fh.czT.begin(), fh.czT.end());
        f_czT32 = pk.add(cT32.data(), cT32.size() * 4);
        f_sched = pk.add(fh.sched.data(), fh.sched.size() * sizeof(int));
        f_soff = pk.add(fh.sched_off.data(), fh.sched_off.size() * sizeof(int));
        f_schedT = pk.add(fh.schedT.data(), fh.schedT.size() * sizeof(int));
        f_soffT = pk.add(fh.schedT_off.data(), fh.schedT_off.size() * sizeof(int));
    }
    // per-direction non-zero B-splines at the quadrature points (device geometry)
    size_t g_first[3], g_B[3], g_D[3];
    for (int l = 0; l < 3; ++l) {
        const wqfd::Space1D& S = sp[l];
        std::vector<int> first(S.nq);
        std::vector<double> gb((size_t)S.nq * (p + 1)), gd((size_t)S.nq * (p + 1));
        for (int q = 0; q < S.nq; ++q)
            first[q] = wqfd::eval_nonzero(S.knots, p, S.m, S.xq[q], &gb[(size_t)q * (p + 1)],
                                          &gd[(size_t)q * (p + 1)]) - p;
        g_first[l] = pk.add(first.data(), first.size() * sizeof(int));
        g_B[l] = pk.add(gb.data(), gb.size() * 8);
        g_D[l] = pk.add(gd.data(), gd.size() * 8);
    }
    // workspace layout
    size_t off = 0;
    const size_t o_tab = off;
    off += al256(pk.buf.size());
    const size_t o_detj = off;
    off += al256(o.Nq * 8);
    const size_t o_jinv = off;
    off += al256(9 * o.Nq * 8);
    const size_t o_F = off;
    off += al256(3 * o.Nq * 8);
    const size_t o_c64 = off;
    off += al256(6 * o.Nq * 8);
    size_t o_c32 = 0;
    if (prec_mask & WQ_F32) {
        o_c32 = off;
        off += al256(6 * o.Nq * 4);
    }
    // reaction plane alpha det J (written by wq_set_alpha)
    const size_t o_cm64 = off;
    off += al256(o.Nq * 8);
    size_t o_cm32 = 0;
    if (prec_mask & WQ_F32) {
        o_cm32 = off;
        off += al256(o.Nq * 4);
    }
    const size_t o_scr = off;
    o.fused = fused_ok;                 // (the gradient's scratch need depends on it; tables filled below)
    o.scratch_bytes = wqfd::wq_scratch_bytes(o, prec_mask);
    off += al256(o.scratch_bytes);
    const size_t o_red = off;
    off += al256(wqfd::norm2_ws_bytes());
    if (ws_needed) *ws_needed = off;
    if (!ws) return WQ_OK;
    if (ws_bytes < off) return fail(WQ_ENOMEM, "workspace too small for wq_setup");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(WQ_EINVAL, "workspace must be 256-byte aligned");

    // geometry: on the device when its intermediates fit the operator's own memory
    // (Z and the control net in the scratch region, Y in the FP64 coefficient
    // planes, which set_coef fills afterwards), else on the host
    const int mm[3] = {sp[0].m, sp[1].m, sp[2].m};
    const size_t M = (size_t)mm[0] * mm[1] * mm[2];
    const size_t zb = (size_t)o.nq[2] * mm[1] * mm[0] * 8 * 8, yb = (size_t)o.nq[2] * o.nq[1] * mm[0] * 12 * 8;
    const bool dev_geom = !std::getenv("WQFD_HOST_GEOMETRY") && al256(zb) + al256(M * 32) + 256 <= o.scratch_bytes &&
                          yb <= 6 * o.Nq * 8;
    std::vector<double> hdet, hjinv, hF, hom;
    if (dev_geom) {
        hom.resize(M * 4);
        for (size_t k = 0; k < M; ++k) {
            const double w = weights ? weights[k] : 1.0;
            if (!(w > 0.0)) return fail(WQ_EINVAL, "rational map: every control weight must be positive");
            for (int a = 0; a < 3; ++a) hom[4 * k + a] = w * ctrl[3 * k + a];
            hom[4 * k + 3] = w;
        }
    } else {
        hdet.resize(o.Nq);
        hjinv.resize(9 * o.Nq);
        hF.resize(3 * o.Nq);
        rc = wqfd::geometry_at_quad(sp, ctrl, weights, hdet.data(), hjinv.data(), hF.data(), err, nthreads());
        if (rc) return fail(rc, err);
    }

    char* base = static_cast<char*>(ws);
    HIP_TRY(hipMemcpyAsync(base + o_tab, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice, s), "upload tables");
    o.detJ = reinterpret_cast<double*>(base + o_detj);
    o.Jinv = reinterpret_cast<double*>(base + o_jinv);
    o.F = reinterpret_cast<double*>(base + o_F);
    o.C64 = reinterpret_cast<double*>(base + o_c64);
    o.C32 = (prec_mask & WQ_F32) ? reinterpret_cast<float*>(base + o_c32) : nullptr;
    o.Cm64 = reinterpret_cast<double*>(base + o_cm64);
    o.Cm32 = (prec_mask & WQ_F32) ? reinterpret_cast<float*>(base + o_cm32) : nullptr;
    o.scratch = base + o_scr;
    o.red = base + o_red;
    if (dev_geom) {
        wqfd::GeomArgs g;
        g.p = p;
        for (int l = 0; l < 3; ++l) {
            g.m[l] = mm[l];
            g.nq[l] = o.nq[l];
            g.first[l] = reinterpret_cast<const int*>(base + o_tab + g_first[l]);
            g.B[l] = reinterpret_cast<const double*>(base + o_tab + g_B[l]);
            g.D[l] = reinterpret_cast<const double*>(base + o_tab + g_D[l]);
        }
        g.Nq = o.Nq;
        char* scr = static_cast<char*>(o.scratch);
        g.Z = reinterpret_cast<double*>(scr);
        double* dctrl = reinterpret_cast<double*>(scr + al256(zb));
        g.ctrl = dctrl;
        g.bad = reinterpret_cast<int*>(scr + al256(zb) + al256(M * 32));
        g.Y = o.C64;
        g.detJ = o.detJ;
        g.Jinv = o.Jinv;
        g.F = o.F;
        int zero = 0, bad = 0;
        HIP_TRY(hipMemcpyAsync(dctrl, hom.data(), M * 32, hipMemcpyHostToDevice, s), "upload control net");
        HIP_TRY(hipMemcpyAsync(g.bad, &zero, sizeof(int), hipMemcpyHostToDevice, s), "clear flag");
        HIP_TRY(wqfd::launch_geometry(g, s), "geometry");
        HIP_TRY(hipMemcpyAsync(&bad, g.bad, sizeof(int), hipMemcpyDeviceToHost, s), "read flag");
        HIP_TRY(hipStreamSynchronize(s), "geometry sync");
        if (bad) return fail(WQ_EGEOM, "geometry map is not orientation preserving: det J <= 0 at a quadrature point");
    } else {
        HIP_TRY(hipMemcpyAsync(o.detJ, hdet.data(), o.Nq * 8, hipMemcpyHostToDevice, s), "upload detJ");
        HIP_TRY(hipMemcpyAsync(o.Jinv, hjinv.data(), 9 * o.Nq * 8, hipMemcpyHostToDevice, s), "upload Jinv");
        HIP_TRY(hipMemcpyAsync(o.F, hF.data(), 3 * o.Nq * 8, hipMemcpyHostToDevice, s), "upload F");
    }
    const char* tb = base + o_tab;
    for (int l = 0; l < 3; ++l) {
        auto& d64 = o.t64.dir[l];
        auto& d32 = o.t32.dir[l];
        for (int v = 0; v < 2; ++v) {
            patch(&d64.B[v], doff[l].B, v, tb);
            patch(&d64.BT[v], doff[l].BT, v, tb);
            patch(&d32.B[v], doff[l].B32, v, tb);
            patch(&d32.BT[v], doff[l].BT32, v, tb);
        }
        for (int v = 0; v < 4; ++v) {
            patch(&d64.W[v], doff[l].W, v, tb);
            patch(&d64.WT[v], doff[l].WT, v, tb);
            patch(&d32.W[v], doff[l].W32, v, tb);
            patch(&d32.WT[v], doff[l].WT32, v, tb);
        }
    }
    if (fused_ok) {
        auto fill = [&](auto& fz, size_t ot0, size_t ot1, size_t ocz, size_t oczT, auto* Cp) {
            using T = std::remove_pointer_t<decltype(Cp)>;
            fz.C = Cp;
            fz.n1 = o.n[0];
            fz.n2 = o.n[1];
            fz.n3 = o.n[2];
            fz.nq1 = o.nq[0];
            fz.nq2 = o.nq[1];
            fz.nq3 = o.nq[2];
            fz.Nq = o.Nq;
            fz.tilesX = reinterpret_cast<const T*>(tb + ot0);
            fz.tilesY = reinterpret_cast<const T*>(tb + ot1);
            fz.JX = reinterpret_cast<const int*>(tb + f_J[0]);
            fz.IX = reinterpret_cast<const int*>(tb + f_I[0]);
            fz.JY = reinterpret_cast<const int*>(tb + f_J[1]);
            fz.IY = reinterpret_cast<const int*>(tb + f_I[1]);
            fz.bandX = reinterpret_cast<const int*>(tb + f_band[0]);
            fz.bandY = reinterpret_cast<const int*>(tb + f_band[1]);
            fz.bs3 = reinterpret_cast<const int*>(tb + f_bs3);
            fz.wts3 = reinterpret_cast<const int*>(tb + f_wts3);
            fz.cz = reinterpret_cast<const T*>(tb + ocz);
            fz.czT = reinterpret_cast<const T*>(tb + oczT);
            fz.ntx = fh.ntile[0];
            fz.nty = fh.ntile[1];
            fz.zchunk = fh.zchunk;
            fz.sched = reinterpret_cast<const int*>(tb + f_sched);
            fz.sched_off = reinterpret_cast<const int*>(tb + f_soff);
            fz.schedT = reinterpret_cast<const int*>(tb + f_schedT);
            fz.schedT_off = reinterpret_cast<const int*>(tb + f_soffT);
        };
        fill(o.fz64, f_tiles64[0], f_tiles64[1], f_cz64, f_czT64, o.C64);
        fill(o.fz32, f_tiles32[0], f_tiles32[1], f_cz32, f_czT32, o.C32);
        o.fused = true;
    }
    HIP_TRY(wqfd::launch_set_coef(o, k_kind, K_q, s), "set_coef");
    HIP_TRY(hipStreamSynchronize(s), "wq_setup sync");
    *out = op.release();
    return WQ_OK;
}

int wq_setup(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl, int k_kind,
             const double* K_q, int prec_mask, void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s,
             wq_op* out) {
    return setup_impl(wqfd::kRuleWQ, p, nknots, knots, ctrl, nullptr, k_kind, K_q, prec_mask, ws, ws_bytes, ws_needed,
                      s, out);
}

int wq_setup_nurbs(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl,
                   const double* weights, int k_kind, const double* K_q, int prec_mask, void* ws, size_t ws_bytes,
                   size_t* ws_needed, wq_stream_t s, wq_op* out) {
    if (!weights) return fail(WQ_EINVAL, "null weights");
    return setup_impl(wqfd::kRuleWQ, p, nknots, knots, ctrl, weights, k_kind, K_q, prec_mask, ws, ws_bytes,
                      ws_needed, s, out);
}

int wq_setup_gauss(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl, int k_kind,
                   const double* K_q, int prec_mask, void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s,
                   wq_op* out) {
    return setup_impl(wqfd::kRuleGauss, p, nknots, knots, ctrl, nullptr, k_kind, K_q, prec_mask, ws, ws_bytes,
                      ws_needed, s, out);
}

int wq_dims(wq_op A, int32_t n[3], int32_t nq[3]) {
    if (!A) return fail(WQ_EINVAL, "null handle");
    for (int l = 0; l < 3; ++l) {
        if (n) n[l] = A->op.n[l];
        if (nq) nq[l] = A->op.nq[l];
    }
    return WQ_OK;
}

int wq_quad_points(wq_op A, double* xq, double* Fq, wq_stream_t s) {
    if (!A) return fail(WQ_EINVAL, "null handle");
    if (xq) {
        size_t o = 0;
        for (int l = 0; l < 3; ++l) {
            std::memcpy(xq + o, A->op.xq[l].data(), A->op.xq[l].size() * 8);
            o += A->op.xq[l].size();
        }
    }
    if (Fq)
        HIP_TRY(hipMemcpyAsync(Fq, A->op.F, 3 * A->op.Nq * 8, hipMemcpyDeviceToDevice,
                               reinterpret_cast<hipStream_t>(s)),
                "copy F");
    return WQ_OK;
}

int wq_detj(wq_op A, double* detj, wq_stream_t s) {
    if (!A || !detj) return fail(WQ_EINVAL, "null argument");
    HIP_TRY(hipMemcpyAsync(detj, A->op.detJ, A->op.Nq * 8, hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(s)),
            "copy detJ");
    return WQ_OK;
}

int wq_set_coef(wq_op A, int k_kind, const double* K_q, wq_stream_t s) {
    if (!A) return fail(WQ_EINVAL, "null handle");
    if (k_kind != WQ_K_IDENTITY && k_kind != WQ_K_SCALAR && k_kind != WQ_K_SYM6)
        return fail(WQ_EINVAL, "unknown k_kind");
    if (k_kind != WQ_K_IDENTITY && !K_q) return fail(WQ_EINVAL, "K_q is required for this k_kind");
    A->op.k_kind = k_kind;
    HIP_TRY(wqfd::launch_set_coef(A->op, k_kind, K_q, reinterpret_cast<hipStream_t>(s)), "set_coef");
    return WQ_OK;
}

int wq_set_alpha(wq_op A, const double* alpha_q, wq_stream_t s) {
    if (!A) return fail(WQ_EINVAL, "null handle");
    if (!alpha_q) {
        A->op.mass = false;
        return WQ_OK;
    }
    HIP_TRY(wqfd::launch_set_alpha(A->op, alpha_q, reinterpret_cast<hipStream_t>(s)), "set_alpha");
    A->op.mass = true;
    return WQ_OK;
}

int wq_alpha_mean(wq_op A, double* mean, wq_stream_t s) {
    if (!A || !mean) return fail(WQ_EINVAL, "null argument");
    if (!A->op.mass) return fail(WQ_EINVAL, "no reaction coefficient set (wq_set_alpha)");
    std::string err;
    double sum = 0.0;
    if (wqfd::sum_all(A->op.Cm64, A->op.Nq, A->op.red, &sum, err, reinterpret_cast<hipStream_t>(s)))
        return fail(WQ_EHIP, "wq_alpha_mean: " + err);
    *mean = sum / (double)A->op.Nq;
    return WQ_OK;
}

static int apply_common(wq_op A, int prec, const void* v, void* w, wq_stream_t s, bool tr, bool acc) {
    if (!A || !v || !w) return fail(WQ_EINVAL, "null argument");
    if ((prec != WQ_F64 && prec != WQ_F32) || !(A->op.prec_mask & prec))
        return fail(WQ_EINVAL, "precision not prepared for this operator");
    if (v == w) return fail(WQ_EINVAL, "v and w must not alias");
    if (acc && !A->op.fused) return fail(WQ_EINVAL, "accumulating apply needs the fused kernels (p <= 7)");
    // the fused kernels add into w; with acc they skip clearing it first
    HIP_TRY(wqfd::launch_apply(A->op, prec, v, w, tr, reinterpret_cast<hipStream_t>(s), acc),
            acc ? "wq_apply_acc" : tr ? "wq_apply_T" : "wq_apply");
    return WQ_OK;
}

int wq_apply(wq_op A, int prec, const void* v, void* w, wq_stream_t s) {
    return apply_common(A, prec, v, w, s, false, false);
}
int wq_apply_T(wq_op A, int prec, const void* v, void* w, wq_stream_t s) {
    return apply_common(A, prec, v, w, s, true, false);
}
int wq_apply_acc(wq_op A, int prec, const void* v, void* w, wq_stream_t s) {
    return apply_common(A, prec, v, w, s, false, true);
}

int wq_apply_mass(wq_op A, int prec, const void* v, void* w, wq_stream_t s) {
    if (!A || !v || !w) return fail(WQ_EINVAL, "null argument");
    if ((prec != WQ_F64 && prec != WQ_F32) || !(A->op.prec_mask & prec))
        return fail(WQ_EINVAL, "precision not prepared for this operator");
    if (v == w) return fail(WQ_EINVAL, "v and w must not alias");
    if (!A->op.mass) return fail(WQ_EINVAL, "no reaction coefficient set (wq_set_alpha)");
    HIP_TRY(wqfd::launch_apply_mass(A->op, prec, v, w, reinterpret_cast<hipStream_t>(s)), "wq_apply_mass");
    return WQ_OK;
}

int wq_rhs(wq_op A, const double* f_q, double* b, wq_stream_t s) {
    if (!A || !f_q || !b) return fail(WQ_EINVAL, "null argument");
    HIP_TRY(wqfd::launch_rhs(A->op, f_q, b, reinterpret_cast<hipStream_t>(s)), "wq_rhs");
    return WQ_OK;
}

int wq_grad_K(wq_op A, const double* lam, const double* u, double* gK, wq_stream_t s) {
    if (!A || !lam || !u || !gK) return fail(WQ_EINVAL, "null argument");
    HIP_TRY(wqfd::launch_grad_K(A->op, lam, u, gK, reinterpret_cast<hipStream_t>(s)), "wq_grad_K");
    return WQ_OK;
}

int wq_grad_f(wq_op A, const double* lam, double* gf, wq_stream_t s) {
    if (!A || !lam || !gf) return fail(WQ_EINVAL, "null argument");
    HIP_TRY(wqfd::launch_grad_f(A->op, lam, gf, reinterpret_cast<hipStream_t>(s)), "wq_grad_f");
    return WQ_OK;
}

int wq_grad_Kf(wq_op A, const double* lam, const double* u, double* gK, double* gf, wq_stream_t s) {
    if (!A || !lam || !u || !gK || !gf) return fail(WQ_EINVAL, "null argument");
    HIP_TRY(wqfd::launch_grad_Kf(A->op, lam, u, gK, gf, reinterpret_cast<hipStream_t>(s)), "wq_grad_Kf");
    return WQ_OK;
}

int wq_grad_alpha(wq_op A, const double* lam, const double* u, double* g, wq_stream_t s) {
    if (!A || !lam || !u || !g) return fail(WQ_EINVAL, "null argument");
    if (!(A->op.prec_mask & WQ_F64)) return fail(WQ_EINVAL, "FP64 not prepared");
    HIP_TRY(wqfd::launch_grad_alpha(A->op, lam, u, g, reinterpret_cast<hipStream_t>(s)), "wq_grad_alpha");
    return WQ_OK;
}

void wq_destroy(wq_op A) { delete A; }

// ------------------------------------------------------------------------ FD
int fd_setup(int p, const int32_t nknots[3], const double* const knots[3], int prec_mask, void* ws, size_t ws_bytes,
             size_t* ws_needed, wq_stream_t s_, fd_pc* out) {
    g_err.clear();
    hipStream_t s = reinterpret_cast<hipStream_t>(s_);
    int rc = check_knots_args(p, nknots, knots);
    if (rc) return rc;
    if (prec_mask == 0 || (prec_mask & ~(WQ_F64 | WQ_F32 | WQ_BF16)))
        return fail(WQ_EINVAL, "prec_mask must combine WQ_F64, WQ_F32, WQ_BF16");
    if (!ws && !ws_needed) return fail(WQ_EINVAL, "need ws or ws_needed");
    if (ws && !out) return fail(WQ_EINVAL, "null output handle");
    wqfd::Space1D sp[3];
    std::string err;
    for (int l = 0; l < 3; ++l) {
        rc = wqfd::build_space(p, nknots[l], knots[l], false, sp[l], err);
        if (rc) return fail(rc, "direction " + std::to_string(l + 1) + ": " + err);
    }
    auto P = std::make_unique<fd_pc_s>();
    wqfd::FdPc& f = P->pc;
    f.prec_mask = prec_mask;
    for (int l = 0; l < 3; ++l) f.n[l] = sp[l].n;
    f.N = (size_t)f.n[0] * f.n[1] * f.n[2];
    size_t off = 0, o_u64[3], o_u32[3], o_ubf[3], o_lam[3];
    for (int l = 0; l < 3; ++l) {
        const size_t n = f.n[l];
        const size_t np = (n + 63) / 64 * 64;
        o_u64[l] = off;
        off += 2 * al256(n * n * 8);
        o_lam[l] = off;
        off += al256(n * 8);
        o_u32[l] = off;
        if (prec_mask & WQ_F32) off += 2 * al256(n * n * 4);
        o_ubf[l] = off;
        if (prec_mask & WQ_BF16) off += al256(2 * np * np * 2);
    }
    const int nmax = std::max(f.n[0], std::max(f.n[1], f.n[2]));
    const int ldp = nmax <= 144 ? (nmax + 15) / 16 * 16 : 0;
    size_t o_pad64 = 0, o_pad32 = 0;
    if (ldp) {
        const size_t blk = al256((size_t)ldp * ldp * 8);
        o_pad64 = off;
        off += 6 * blk;
        o_pad32 = off;
        if (prec_mask & WQ_F32) off += 6 * al256((size_t)ldp * ldp * 4);
    }
    const size_t o_scr = off;
    off += al256(f.N * 8);
    if (ws_needed) *ws_needed = off;
    if (!ws) return WQ_OK;
    if (ws_bytes < off) return fail(WQ_ENOMEM, "workspace too small for fd_setup");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(WQ_EINVAL, "workspace must be 256-byte aligned");
    char* base = static_cast<char*>(ws);
    for (int l = 0; l < 3; ++l) {
        const int n = f.n[l];
        rc = wqfd::gen_eig(n, sp[l].Ki, sp[l].Mi, f.hlam[l], f.hU[l], err);
        if (rc) return fail(rc, err);
        std::vector<double> ut((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) ut[(size_t)i * n + j] = f.hU[l][(size_t)j * n + i];
        f.U64[l] = reinterpret_cast<double*>(base + o_u64[l]);
        f.UT64[l] = reinterpret_cast<double*>(base + o_u64[l] + al256((size_t)n * n * 8));
        f.lam[l] = reinterpret_cast<double*>(base + o_lam[l]);
        HIP_TRY(hipMemcpy(f.U64[l], f.hU[l].data(), (size_t)n * n * 8, hipMemcpyHostToDevice), "upload U");
        HIP_TRY(hipMemcpy(f.UT64[l], ut.data(), (size_t)n * n * 8, hipMemcpyHostToDevice), "upload U^T");
        HIP_TRY(hipMemcpy(f.lam[l], f.hlam[l].data(), (size_t)n * 8, hipMemcpyHostToDevice), "upload lam");
        if (prec_mask & WQ_F32) {
            std::vector<float> u32(f.hU[l].begin(), f.hU[l].end()), ut32(ut.begin(), ut.end());
            f.U32[l] = reinterpret_cast<float*>(base + o_u32[l]);
            f.UT32[l] = reinterpret_cast<float*>(base + o_u32[l] + al256((size_t)n * n * 4));
            HIP_TRY(hipMemcpy(f.U32[l], u32.data(), (size_t)n * n * 4, hipMemcpyHostToDevice), "upload U32");
            HIP_TRY(hipMemcpy(f.UT32[l], ut32.data(), (size_t)n * n * 4, hipMemcpyHostToDevice), "upload U32^T");
        }
        if (prec_mask & WQ_BF16) {
            const int np = (n + 63) / 64 * 64;
            std::vector<uint16_t> ub(2 * (size_t)np * np, 0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    ub[(size_t)i * np + j] = f32_to_bf16_bits((float)f.hU[l][(size_t)j * n + i]);          // U^T
                    ub[(size_t)np * np + (size_t)i * np + j] = f32_to_bf16_bits((float)f.hU[l][(size_t)i * n + j]);  // U
                }
            f.Ubf[l] = reinterpret_cast<uint16_t*>(base + o_ubf[l]);
            HIP_TRY(hipMemcpy(f.Ubf[l], ub.data(), ub.size() * 2, hipMemcpyHostToDevice), "upload Ubf");
        }
    }
    if (ldp) {
        f.ldp = ldp;
        const size_t blk64 = al256((size_t)ldp * ldp * 8), blk32 = al256((size_t)ldp * ldp * 4);
        for (int l = 0; l < 3; ++l) {
            const int n = f.n[l];
            std::vector<double> up((size_t)ldp * ldp, 0.0), utp((size_t)ldp * ldp, 0.0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    up[(size_t)i * ldp + j] = f.hU[l][(size_t)i * n + j];
                    utp[(size_t)i * ldp + j] = f.hU[l][(size_t)j * n + i];
                }
            f.Up64[l] = reinterpret_cast<double*>(base + o_pad64 + (2 * l) * blk64);
            f.UTp64[l] = reinterpret_cast<double*>(base + o_pad64 + (2 * l + 1) * blk64);
            HIP_TRY(hipMemcpy(f.Up64[l], up.data(), up.size() * 8, hipMemcpyHostToDevice), "upload padded U");
            HIP_TRY(hipMemcpy(f.UTp64[l], utp.data(), utp.size() * 8, hipMemcpyHostToDevice), "upload padded U^T");
            if (prec_mask & WQ_F32) {
                std::vector<float> up32(up.begin(), up.end()), utp32(utp.begin(), utp.end());
                f.Up32[l] = reinterpret_cast<float*>(base + o_pad32 + (2 * l) * blk32);
                f.UTp32[l] = reinterpret_cast<float*>(base + o_pad32 + (2 * l + 1) * blk32);
                HIP_TRY(hipMemcpy(f.Up32[l], up32.data(), up32.size() * 4, hipMemcpyHostToDevice), "upload padded U32");
                HIP_TRY(hipMemcpy(f.UTp32[l], utp32.data(), utp32.size() * 4, hipMemcpyHostToDevice),
                        "upload padded U32^T");
            }
        }
    }
    f.scratch = base + o_scr;
    (void)s;
    *out = P.release();
    return WQ_OK;
}

int fd_apply(fd_pc P, int prec, const void* r, void* z, wq_stream_t s) {
    if (!P || !r || !z) return fail(WQ_EINVAL, "null argument");
    if ((prec != WQ_F64 && prec != WQ_F32 && prec != WQ_BF16) || !(P->pc.prec_mask & prec))
        return fail(WQ_EINVAL, "precision not prepared for this preconditioner");
    HIP_TRY(wqfd::launch_fd_apply(P->pc, prec, r, z, reinterpret_cast<hipStream_t>(s)), "fd_apply");
    return WQ_OK;
}

int fd_apply_noalloc(fd_pc P, int prec, const void* r, void* z, wq_stream_t s) {
    if (!P || !r || !z) return fail(WQ_EINVAL, "null argument");
    if ((prec != WQ_F64 && prec != WQ_F32 && prec != WQ_BF16) || !(P->pc.prec_mask & prec))
        return fail(WQ_EINVAL, "precision not prepared for this preconditioner");
    // the passes keep N values between them; reserve 8 bytes per value (the
    // bound fd_setup reserves in its workspace, for every precision)
    if (P->pc.N > kFdNoAllocBytes / 8)
        return fail(WQ_ENOMEM, "fd_apply_noalloc: N = " + std::to_string(P->pc.N) +
                                   " exceeds the static scratch (at most " + std::to_string(kFdNoAllocBytes / 8) +
                                   " unknowns); use fd_apply");
    void* tmp = nullptr;
    int rc = noalloc_scratch(&tmp);
    if (rc) return rc;
    HIP_TRY(wqfd::launch_fd_apply(P->pc, prec, r, z, tmp, reinterpret_cast<hipStream_t>(s)), "fd_apply_noalloc");
    return WQ_OK;
}

int fd_set_shift(fd_pc P, double sigma, wq_stream_t s) {
    if (!P) return fail(WQ_EINVAL, "null handle");
    auto& f = P->pc;
    if (!std::isfinite(sigma)) return fail(WQ_EINVAL, "shift must be finite");
    double lmin = sigma;
    for (int l = 0; l < 3; ++l) lmin += *std::min_element(f.hlam[l].begin(), f.hlam[l].end());
    if (!(lmin > 0.0)) return fail(WQ_EINVAL, "shift makes the FD diagonal non-positive");
    std::vector<double> l3(f.hlam[2]);
    for (double& x : l3) x += sigma;
    hipStream_t st = reinterpret_cast<hipStream_t>(s);
    HIP_TRY(hipMemcpyAsync(f.lam[2], l3.data(), l3.size() * 8, hipMemcpyHostToDevice, st), "upload shifted lam3");
    HIP_TRY(hipStreamSynchronize(st), "fd_set_shift sync");
    f.shift = sigma;
    return WQ_OK;
}

int fd_factors(fd_pc P, int l, double* lam, double* U) {
    if (!P || l < 0 || l > 2) return fail(WQ_EINVAL, "bad argument");
    const auto& f = P->pc;
    if (lam) std::memcpy(lam, f.hlam[l].data(), f.hlam[l].size() * 8);
    if (U) std::memcpy(U, f.hU[l].data(), f.hU[l].size() * 8);
    return WQ_OK;
}

void fd_destroy(fd_pc P) { delete P; }

// ------------------------------------------------------------------------ host-only inspection
int wq_space_1d(int p, int nknots, const double* knots, int32_t* n, int32_t* nq, double* xq, double* B, double* W) {
    g_err.clear();
    if (!knots || !n || !nq) return fail(WQ_EINVAL, "null argument");
    wqfd::Space1D S;
    std::string err;
    int rc = wqfd::build_space(p, nknots, knots, B != nullptr || W != nullptr, S, err);
    if (rc) return fail(rc, err);
    *n = S.n;
    *nq = S.nq;
    if (xq) std::memcpy(xq, S.xq.data(), S.xq.size() * 8);
    if (B)
        for (int d = 0; d < 2; ++d) std::memcpy(B + (size_t)d * S.nq * S.n, S.B[d].data(), S.B[d].size() * 8);
    if (W)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                std::memcpy(W + (size_t)(2 * a + b) * S.n * S.nq, S.W[a][b].data(), S.W[a][b].size() * 8);
    return WQ_OK;
}

int fd_eig_1d(int p, int nknots, const double* knots, double* lam, double* U) {
    g_err.clear();
    if (!knots) return fail(WQ_EINVAL, "null argument");
    wqfd::Space1D S;
    std::string err;
    int rc = wqfd::build_space(p, nknots, knots, false, S, err);
    if (rc) return fail(rc, err);
    std::vector<double> l, u;
    rc = wqfd::gen_eig(S.n, S.Ki, S.Mi, l, u, err);
    if (rc) return fail(rc, err);
    if (lam) std::memcpy(lam, l.data(), l.size() * 8);
    if (U) std::memcpy(U, u.data(), u.size() * 8);
    return WQ_OK;
}

int wq_geometry_host(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl,
                     const double* weights, double* detJ, double* Jinv, double* F) {
    g_err.clear();
    int rc = check_knots_args(p, nknots, knots);
    if (rc) return rc;
    if (!ctrl || !detJ || !Jinv || !F) return fail(WQ_EINVAL, "null argument");
    wqfd::Space1D sp[3];
    std::string err;
    for (int l = 0; l < 3; ++l) {
        rc = wqfd::build_space(p, nknots[l], knots[l], false, sp[l], err);
        if (rc) return fail(rc, err);
    }
    rc = wqfd::geometry_at_quad(sp, ctrl, weights, detJ, Jinv, F, err, nthreads());
    return rc ? fail(rc, err) : WQ_OK;
}

// ------------------------------------------------------------------------ evaluation at Gauss points
int wq_eval_setup(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl,
                  const double* weights, int ng, void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s_,
                  wq_eval* out) {
    g_err.clear();
    hipStream_t s = reinterpret_cast<hipStream_t>(s_);
    int rc = check_knots_args(p, nknots, knots);
    if (rc) return rc;
    if (!ctrl) return fail(WQ_EINVAL, "null control points");
    if (!ws && !ws_needed) return fail(WQ_EINVAL, "need ws or ws_needed");
    if (ws && !out) return fail(WQ_EINVAL, "null output handle");
    wqfd::GaussSpace1D G[3];
    std::string err;
    for (int l = 0; l < 3; ++l) {
        rc = wqfd::gauss_space(p, nknots[l], knots[l], ng, G[l], err);
        if (rc) return fail(rc, "direction " + std::to_string(l + 1) + ": " + err);
    }
    const size_t M = (size_t)G[0].m * G[1].m * G[2].m;
    std::vector<double> hom(M * 4);
    for (size_t k = 0; k < M; ++k) {
        const double w = weights ? weights[k] : 1.0;
        if (!(w > 0.0)) return fail(WQ_EINVAL, "every control weight must be positive");
        for (int a = 0; a < 3; ++a) hom[4 * k + a] = w * ctrl[3 * k + a];
        hom[4 * k + 3] = w;
    }
    Packer pk;
    size_t o_first[3], o_B[3], o_D[3], o_w[3];
    for (int l = 0; l < 3; ++l) {
        o_first[l] = pk.add(G[l].first.data(), G[l].first.size() * sizeof(int));
        o_B[l] = pk.add(G[l].B.data(), G[l].B.size() * 8);
        o_D[l] = pk.add(G[l].D.data(), G[l].D.size() * 8);
        o_w[l] = pk.add(G[l].w.data(), G[l].w.size() * 8);
    }
    const size_t o_ctrl = pk.add(hom.data(), hom.size() * 8);
    if (ws_needed) *ws_needed = pk.buf.size();
    if (!ws) return WQ_OK;
    if (ws_bytes < pk.buf.size()) return fail(WQ_ENOMEM, "workspace too small for wq_eval_setup");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(WQ_EINVAL, "workspace must be 256-byte aligned");
    char* base = static_cast<char*>(ws);
    HIP_TRY(hipMemcpyAsync(base, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice, s), "upload eval tables");
    auto h = std::make_unique<wq_eval_s>();
    wqfd::EvalOp& E = h->E;
    E.p = p;
    E.ng = ng;
    for (int l = 0; l < 3; ++l) {
        E.ne[l] = G[l].n_el;
        E.nq[l] = G[l].nq;
        E.m[l] = G[l].m;
        E.n[l] = G[l].m - 2;
        E.first[l] = reinterpret_cast<const int*>(base + o_first[l]);
        E.B[l] = reinterpret_cast<const double*>(base + o_B[l]);
        E.D[l] = reinterpret_cast<const double*>(base + o_D[l]);
        E.w[l] = reinterpret_cast<const double*>(base + o_w[l]);
    }
    E.ctrl = reinterpret_cast<const double*>(base + o_ctrl);
    HIP_TRY(hipStreamSynchronize(s), "wq_eval_setup sync");
    *out = h.release();
    return WQ_OK;
}

int wq_eval_dims(wq_eval E, int32_t ne[3], int32_t nq[3]) {
    if (!E) return fail(WQ_EINVAL, "null handle");
    for (int l = 0; l < 3; ++l) {
        if (ne) ne[l] = E->E.ne[l];
        if (nq) nq[l] = E->E.nq[l];
    }
    return WQ_OK;
}

int wq_eval_slab(wq_eval E, const double* u, int e3_begin, int e3_end, double* X, double* wdet, double* uh,
                 double* grad, wq_stream_t s) {
    if (!E || !u || !X || !wdet || !uh || !grad) return fail(WQ_EINVAL, "null argument");
    if (e3_begin < 0 || e3_end > E->E.ne[2] || e3_begin > e3_end) return fail(WQ_EINVAL, "element range outside [0, n_el3]");
    HIP_TRY(wqfd::launch_eval_slab(E->E, u, e3_begin, e3_end, X, wdet, uh, grad, reinterpret_cast<hipStream_t>(s)),
            "wq_eval_slab");
    return WQ_OK;
}

void wq_eval_destroy(wq_eval E) { delete E; }

// ------------------------------------------------------------------------ Krylov
size_t krylov_ws_bytes(wq_op A) { return A ? wqfd::krylov_bytes(A->op.N, false) : 0; }

int krylov_solve(wq_op A, fd_pc P, int transpose, const double* b, double* x, double rtol, int maxit, void* ws,
                 size_t ws_bytes, int* iters, double* relres, wq_stream_t s_) {
    g_err.clear();
    if (!A || !P || !b || !x || !ws || !iters || !relres) return fail(WQ_EINVAL, "null argument");
    if (!(A->op.prec_mask & WQ_F64) || !(P->pc.prec_mask & WQ_F64)) return fail(WQ_EINVAL, "FP64 not prepared");
    if (P->pc.N != A->op.N) return fail(WQ_EINVAL, "operator and preconditioner sizes differ");
    if (!(rtol > 0) || maxit < 1) return fail(WQ_EINVAL, "need rtol > 0 and maxit >= 1");
    if (ws_bytes < krylov_ws_bytes(A)) return fail(WQ_ENOMEM, "Krylov workspace too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(s_);
    const wqfd::WqOp* op = &A->op;
    const wqfd::FdPc* pc = &P->pc;
    wqfd::LinOp Aop = [op, transpose](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_apply(*op, WQ_F64, in, o, transpose != 0, st);
    };
    wqfd::LinOp Aacc = [op, transpose](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_apply(*op, WQ_F64, in, o, transpose != 0, st, true);
    };
    wqfd::LinOp Mop = [pc](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_fd_apply(*pc, WQ_F64, in, o, st);
    };
    std::string err;
    int rc = wqfd::bicgstab<double>(Aop, Mop, op->N, b, x, false, rtol, maxit, ws, iters, relres, err, s,
                                    op->fused ? &Aacc : nullptr);
    if (rc) return fail(rc, err);
    return WQ_OK;
}

size_t ir_ws_bytes(wq_op A) {
    if (!A) return 0;
    const size_t N = A->op.N;
    // the inner BiCGStab workspace is sized for FP64, which the stagnation fallback uses
    return al256(N * 8) * 2 + al256(N * 4) * 2 + al256(wqfd::krylov_bytes(N, false)) + al256(wqfd::norm2_ws_bytes());
}

int ir_fallback_count(void) { return g_ir_fallbacks; }

int krylov_restart_count(void) { return wqfd::bicgstab_restart_count(); }

int ir_solve(wq_op A, fd_pc P, int fd_prec, const double* b, double* x, double rtol, double tau_inner, int max_outer,
             int maxit_inner, void* ws, size_t ws_bytes, int* outer, int* inner_total, double* relres,
             wq_stream_t s_) {
    g_err.clear();
    if (!A || !P || !b || !x || !ws || !outer || !inner_total || !relres) return fail(WQ_EINVAL, "null argument");
    if (!(A->op.prec_mask & WQ_F64) || !(A->op.prec_mask & WQ_F32))
        return fail(WQ_EINVAL, "operator needs both WQ_F64 and WQ_F32");
    if ((fd_prec != WQ_F32 && fd_prec != WQ_BF16) || !(P->pc.prec_mask & fd_prec))
        return fail(WQ_EINVAL, "fd_prec must be a prepared WQ_F32 or WQ_BF16");
    if (P->pc.N != A->op.N) return fail(WQ_EINVAL, "operator and preconditioner sizes differ");
    if (!(rtol > 0) || !(tau_inner > 0) || max_outer < 1 || maxit_inner < 1) return fail(WQ_EINVAL, "bad tolerances");
    if (ws_bytes < ir_ws_bytes(A)) return fail(WQ_ENOMEM, "IR workspace too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(s_);
    const wqfd::WqOp* op = &A->op;
    const wqfd::FdPc* pc = &P->pc;
    const size_t N = op->N;
    char* c = static_cast<char*>(ws);
    double* r64 = reinterpret_cast<double*>(c);
    c += al256(N * 8);
    double* t64 = reinterpret_cast<double*>(c);
    c += al256(N * 8);
    float* b32 = reinterpret_cast<float*>(c);
    c += al256(N * 4);
    float* d32 = reinterpret_cast<float*>(c);
    c += al256(N * 4);
    double* d64 = reinterpret_cast<double*>(b32);   // FP64 inner solution: the FP32 pair's space (2 al256(4N) >= 8N)
    void* kws = c;
    c += al256(wqfd::krylov_bytes(N, false));
    void* nws = c;
    wqfd::LinOp A32 = [op](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_apply(*op, WQ_F32, in, o, false, st);
    };
    wqfd::LinOp A32acc = [op](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_apply(*op, WQ_F32, in, o, false, st, true);
    };
    wqfd::LinOp M32 = [pc, fd_prec](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_fd_apply(*pc, fd_prec, in, o, st);
    };
    // stagnation fallback: FP64 inner solves (FP64 apply, FP64 FD)
    wqfd::LinOp A64 = [op](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_apply(*op, WQ_F64, in, o, false, st);
    };
    wqfd::LinOp A64acc = [op](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_apply(*op, WQ_F64, in, o, false, st, true);
    };
    wqfd::LinOp M64 = [pc](const void* in, void* o, hipStream_t st) {
        return wqfd::launch_fd_apply(*pc, WQ_F64, in, o, st);
    };
    const bool can_fall_back = (pc->prec_mask & WQ_F64) != 0;
    bool fp64_inner = false;
    std::string err;
    double nb = 0, nr = 0;
    int rc = wqfd::norm2(b, N, nws, &nb, err, s);
    if (rc) return fail(rc, err);
    *outer = 0;
    *inner_total = 0;
    if (!std::isfinite(nb)) return fail(WQ_ENONFINITE, "non-finite value in the right-hand side");
    if (nb == 0.0) {
        HIP_TRY(hipMemsetAsync(x, 0, N * 8, s), "zero x");
        *relres = 0;
        return WQ_OK;
    }
    auto residual = [&]() -> int {
        hipError_t e = wqfd::launch_apply(*op, WQ_F64, x, r64, false, s);
        if (e != hipSuccess) return hip_fail(e, "ir residual apply");
        HIP_TRY(wqfd::launch_resid(b, r64, N, s), "ir resid");
        int r2 = wqfd::norm2(r64, N, nws, &nr, err, s);
        return r2 ? fail(r2, err) : WQ_OK;
    };
    rc = residual();
    if (rc) return rc;
    *relres = nr / nb;
    // (a NaN residual compares false with everything: test it before the stopping test)
    while (true) {
        if (!std::isfinite(nr)) return fail(WQ_ENONFINITE, "non-finite residual in iterative refinement");
        if (nr / nb <= rtol || *outer >= max_outer) break;
        int it = 0;
        double rel = 0;
        const double nr_before = nr;
        if (!fp64_inner) {
            HIP_TRY(wqfd::launch_cast_f64_to_f32(r64, b32, N, 1.0 / nr, s), "ir cast");
            const double tol = std::max(tau_inner, 0.5 * rtol * nb / nr);
            rc = wqfd::bicgstab<float>(A32, M32, N, b32, d32, true, tol, maxit_inner, kws, &it, &rel, err, s,
                                       op->fused ? &A32acc : nullptr, false);
            *inner_total += it;
            if (rc && rc != WQ_ENOCONV && rc != WQ_EBREAKDOWN) return fail(rc, err);
            HIP_TRY(wqfd::launch_axpy_f32_to_f64(d32, x, N, nr, s), "ir update");
        } else {
            // the residual equation solved in FP64 to the accuracy the outer target needs
            HIP_TRY(hipMemcpyAsync(t64, r64, N * 8, hipMemcpyDeviceToDevice, s), "ir copy");
            const double tol = std::max(0.5 * rtol * nb / nr, 1e-14);
            rc = wqfd::bicgstab<double>(A64, M64, N, t64, d64, true, tol, maxit_inner, kws, &it, &rel, err, s,
                                        op->fused ? &A64acc : nullptr, false);
            *inner_total += it;
            if (rc && rc != WQ_ENOCONV && rc != WQ_EBREAKDOWN) return fail(rc, err);
            HIP_TRY(wqfd::launch_axpy_f64(d64, x, N, 1.0, s), "ir update");
        }
        ++*outer;
        rc = residual();
        if (rc) return rc;
        *relres = nr / nb;
        // stagnation: an outer step that does not halve the FP64 residual means the
        // low-precision inner solve no longer yields a useful correction (FP32
        // operator error against the conditioning, or an inner tolerance too loose);
        // the remaining steps solve the residual equation in FP64
        if (!fp64_inner && can_fall_back && std::isfinite(nr) && nr > 0.5 * nr_before) {
            fp64_inner = true;
            ++g_ir_fallbacks;
        }
    }
    if (nr / nb > rtol) return fail(WQ_ENOCONV, "iterative refinement reached max_outer");
    return WQ_OK;
}

}  // extern "C"
