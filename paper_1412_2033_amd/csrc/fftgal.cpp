// Host side of the fftgal C ABI: plan and workspace layout, input validation,
// material setup, the device-resident CG driver and the bounds.
#include "../../include/fftgal.h"
#include "fftgal_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace fftgal;

namespace {

thread_local std::string g_plan_error = "no error";

constexpr int kMaxHist = 20000;      // CG history entries kept per solve
// Device argument tables of the specialised kernels: one zero offset, the
// captured passes of the current solve, its CG items, and a ring for
// one-off launches (set-up, right-hand side).
constexpr size_t kArgSlot = 1024;    // bytes per argument slot (>= sizeof PencilArgs / RowArgs)
constexpr int kMaxPasses = 40;  // operator passes of one CG iteration (reduced Ga, 3D: 5 x 8)
constexpr int kIterSlots = kMaxPasses + 2;  // passes, then the update and the CG item
constexpr int kRingSlots = 32;
constexpr size_t kArgsBytes = kArgSlot * (2 + kIterSlots + kRingSlots);
constexpr double kFloor64 = 1e-14;   // residual floor relative to ||A_M E|| (FP64)
constexpr double kFloor32 = 1e-7;    // (FP32 iterations)
constexpr int kCkptEvery = 64;       // FP32 iterations between best-iterate checkpoints

int smooth_odd(int m) {
    for (int n = std::max(1, m);; ++n) {
        if (n % 2 == 0) continue;
        int x = n;
        for (int p : {3, 5, 7})
            while (x % p == 0) x /= p;
        if (x == 1) return n;
    }
}

bool is_smooth_odd(int n) { return n >= 1 && smooth_odd(n) == n; }

// Complex table entries a transform of length n takes (stage twiddles of a
// smooth n; for a Bluestein transform those of L plus the chirp and the filter).
size_t fft_table_len(int n) {
    if (is_smooth_odd(n)) return (size_t)n;
    const int L = smooth_odd(2 * n - 1);
    return (size_t)L + (size_t)n + (size_t)L;
}

// Radices of the Stockham stages of a 3,5,7-smooth length n: the schedule of
// the specialised kernels for their lengths; otherwise the 7s, then 3 * 3
// merged into radix 9 and a remaining 3 * 5 into 15 (fewer stages and barriers
// per transform: 405 = 9 9 5 instead of 5 3 3 3 3), the 5s kept single (a
// generic radix-25 stage made 175 = 7 25 slower than 7 5 5).
std::vector<int> factor(int n) {
    std::vector<int> f;
    const int fi = fast_index(n);
    if (fi >= 0) {  // the schedule the specialised kernels are compiled for
        for (int s = 0; s < kFastSched[fi].nst; ++s) f.push_back(kFastSched[fi].r[s]);
        return f;
    }
    int c[3] = {0, 0, 0};  // multiplicities of 7, 5, 3
    const int pr[3] = {7, 5, 3};
    for (int i = 0; i < 3; ++i)
        while (n % pr[i] == 0) {
            ++c[i];
            n /= pr[i];
        }
    for (; c[0] > 0; --c[0]) f.push_back(7);
    for (; c[2] >= 2; c[2] -= 2) f.push_back(9);
    if (c[1] && c[2]) {
        f.push_back(15);
        --c[1];
        --c[2];
    }
    for (; c[1] > 0; --c[1]) f.push_back(5);
    if (c[2]) f.push_back(3);
    return f;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Sizes that fix the workspace layout.
struct Dims {
    int d = 0;
    int N[3] = {1, 1, 1};
    int M[3] = {1, 1, 1};
    int L[3] = {1, 1, 1};   // 2N - 1: the support Z_{2N-1} of the material series
    int P[3] = {1, 1, 1};   // largest voxel resolution to provision for
    int Nh = 1;             // (N_d + 1) / 2 stored entries along the last axis
    int Lh = 1;             // N_d: stored entries of Z_{2N_d - 1} along the last axis
    long Ns = 0;            // state entries per component
    long Mtot = 0;          // |M|
    int nc_max = 1;
    int nshift = 1;         // material fields: 2^d shifted grids for the reduced Ga, else 1
    int nfield = 1;         // fields per material side: d (d + 1) / 2 with FFTGAL_TENSOR, else 1
};

// Plan schemes: the Ga on the double grid, GaNi on the grid of the order N,
// and the reduced Ga (Lemma reduce_grid) with 2^d shifted transforms of size N.
enum Scheme { kSchemeGa = 0, kSchemeGani = 1, kSchemeReduced = 2 };

// GaNi: the transforms run on the grid of the approximation order N itself
// (Def. GaNi, Algorithm 1).  Reduced Ga: the material series keeps its support
// Z_{2N-1}, the transforms run on the N-grid (2^d shifted copies).  Lengths
// that are not 3,5,7-smooth are transformed by Bluestein's algorithm.
// Smallest length with specialised kernels that is at least m, or 0.
int fast_length_at_least(int m) {
    int best = 0;
    for (int i = 0; i < kNumFast; ++i)
        if (kFastSched[i].n >= m && (best == 0 || kFastSched[i].n < best)) best = kFastSched[i].n;
    return best;
}

bool make_dims(int d, const int32_t *N, const int32_t *P, Dims *o, int scheme = kSchemeGa, bool tensor = false,
               bool fast_grid = false) {
    if ((d != 2 && d != 3) || N == nullptr) return false;
    const bool gani = scheme == kSchemeGani, red = scheme == kSchemeReduced;
    o->d = d;
    for (int a = 0; a < d; ++a) {
        if (N[a] < 1 || N[a] % 2 == 0 || N[a] > 100000) return false;
        if (P && (P[a] < 1 || P[a] % 2 == 0 || P[a] > 100000)) return false;
        o->N[a] = N[a];
        o->L[a] = gani ? N[a] : 2 * N[a] - 1;
        o->M[a] = (gani || red) ? N[a] : smooth_odd(2 * N[a] - 1);
    }
    if (fast_grid && !gani && !red) {
        // the specialised length at least 2N - 1 on every axis whose default
        // length is at least 9, if the grid then holds at most four times the
        // points, or at most 2^21 points (small grids, where the memory does
        // not matter and the generic kernels' launches set the time; every
        // M >= 2N - 1 integrates exactly)
        int Mf[3] = {0, 0, 0};
        double ratio = 1.0, pts = 1.0;
        for (int a = 0; a < d; ++a) {
            const int f = fast_length_at_least(2 * N[a] - 1);
            if (f > 0 && o->M[a] >= 9) {
                Mf[a] = f;
                ratio *= (double)f / (double)o->M[a];
            }
            pts *= (double)(Mf[a] > 0 ? Mf[a] : o->M[a]);
        }
        if (ratio <= 4.0 || pts <= (double)(1 << 21))
            for (int a = 0; a < d; ++a)
                if (Mf[a] > 0) o->M[a] = Mf[a];
    }
    for (int a = 0; a < d; ++a) o->P[a] = P ? std::max<int>(P[a], o->M[a]) : o->M[a];
    o->Nh = (o->N[d - 1] + 1) / 2;
    o->Lh = gani ? o->Nh : o->N[d - 1];
    o->Ns = (d == 3 ? (long)o->N[0] * o->N[1] : (long)o->N[0]) * o->Nh;
    o->Mtot = 1;
    for (int a = 0; a < d; ++a) o->Mtot *= o->M[a];
    o->nc_max = std::max(1, d - 1);
    o->nshift = red ? 1 << d : 1;
    o->nfield = tensor ? d * (d + 1) / 2 : 1;
    return true;
}

// Device scratch the voxel setup needs for an image of resolution P: the
// image (or its partially transformed form) and the R2C rows.
void voxel_scratch(const Dims &D, const int *P, size_t *need_u, size_t *need_w) {
    const int d = D.d;
    long Ptot = 1;
    for (int a = 0; a < d; ++a) Ptot *= P[a];
    *need_u = (size_t)Ptot * 8;
    *need_w = (size_t)(Ptot / P[d - 1]) * D.Lh * 16;
    if (d == 3) {
        *need_u = std::max(*need_u, (size_t)P[0] * D.L[1] * D.Lh * 16);
        *need_w = std::max(*need_w, (size_t)D.L[0] * D.L[1] * D.Lh * 16);
    }
}

struct Layout {
    size_t tw64, tw32, twP64, twP32, T1, T2, r, p, q, xsol, xsol64, bvec, xbest, gA64, gB64, gA32, gB32, part_a,
        part_b, part_c, gram, args, margs, status, hist, total;
    size_t tw_len, twP_len;  // complex entries per table region
    size_t part_len;         // doubles per partial region
    // reduced Ga: the intermediates of one shift (d components, complex
    // entries) in T1 / T2, so that the 2^d shifts of an operator pass can run
    // in one launch, each on its own slot
    size_t t1_slot, t2_slot;
    // solve slots: the per-solve region [T1 .. part_c] repeated nslots times
    int nslots;
    size_t slot_bytes;
};

constexpr size_t kMultiArgsBytes = 64 * 1024;  // argument tables of multi-shift passes

// grouped: reduced Ga with one intermediate slot and one projected vector per
// shift (the shifts of a pass share a launch); otherwise one of each.
// nsl: solve slots -- copies of the per-solve region (transform intermediates,
// CG vectors, partial sums), so that nsl solves of the plan can run at once.
Layout make_layout(const Dims &D, int precision, bool grouped = true, int nsl = 1) {
    const bool slots = grouped && D.nshift > 1;
    Layout L{};
    const int d = D.d;
    const size_t c16 = 16;
    const long d2 = (long)d * d;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    // twiddle tables: one per axis length M_a (<= sum of lengths entries)
    L.tw_len = 0;
    for (int a = 0; a < d; ++a) L.tw_len += fft_table_len(D.M[a]);
    L.twP_len = 0;
    for (int a = 0; a < d; ++a) L.twP_len += fft_table_len(D.P[a]);
    L.tw64 = take(L.tw_len * c16);
    L.tw32 = take(L.tw_len * 8);
    L.twP64 = take(L.twP_len * c16);
    L.twP32 = take(L.twP_len * 8);
    // transform intermediates (also the material setup scratch)
    size_t t1, t2;
    if (d == 3) {
        t1 = (size_t)d2 * D.M[0] * D.N[1] * D.Nh;
        t2 = (size_t)d2 * D.M[0] * D.M[1] * D.Nh;
        const size_t Lh = D.Lh;
        const size_t s_u = std::max({(size_t)D.L[0] * D.L[1] * Lh, (size_t)D.M[0] * D.M[1] * Lh,
                                     (size_t)D.P[0] * D.L[1] * Lh, (size_t)D.P[0] * D.P[1] * D.P[2] / 2 + 1});
        const size_t s_w = std::max({(size_t)D.M[0] * D.L[1] * Lh, (size_t)D.P[0] * D.P[1] * Lh,
                                     (size_t)D.L[0] * D.L[1] * Lh, (size_t)D.M[0] * D.M[1] * Lh});
        t2 = std::max(t2, s_u);
        t1 = std::max(t1, s_w + 4096);
        L.t1_slot = (size_t)d * D.M[0] * D.N[1] * D.Nh;
        L.t2_slot = (size_t)d * D.M[0] * D.M[1] * D.Nh;
    } else {
        t1 = (size_t)d2 * D.M[0] * D.Nh;
        t2 = 0;
        const size_t Lh = D.Lh;
        const size_t s_u = std::max({(size_t)D.L[0] * Lh, (size_t)D.P[0] * D.P[1] / 2 + 1});
        const size_t s_w = std::max({(size_t)D.P[0] * Lh, (size_t)D.M[0] * Lh});
        t2 = s_u;
        t1 = std::max(t1, s_w + 4096);
        L.t1_slot = (size_t)d * D.M[0] * D.Nh;
        L.t2_slot = 0;
    }
    if (slots) {
        t1 = std::max(t1, (size_t)D.nshift * L.t1_slot);
        t2 = std::max(t2, (size_t)D.nshift * L.t2_slot);
    }
    // per-solve region (one copy per solve slot)
    const size_t vec = (size_t)D.nc_max * D.Ns * c16;
    L.T1 = take(t1 * c16);
    L.T2 = take(t2 * c16);
    L.r = take(vec);
    L.p = take(vec);
    L.q = take(vec * (slots ? D.nshift : 1));  // grouped reduced Ga: one projected vector per shift
    // FP32 iterations: the right-hand side and the best iterate so far
    L.bvec = take(precision == FFTGAL_FP32_ITER ? vec : 0);
    L.xbest = take(precision == FFTGAL_FP32_ITER ? vec : 0);
    // partial sums: the largest work-group count of any reducing launch
    // (worst case: one pencil / one row per work-group)
    long nwg = update_blocks(2L * D.Ns);  // CG update of at most two coefficient components
    const long nbz = (d == 3) ? (long)D.N[1] * D.Nh : D.Nh;
    const long nrows = (d == 3) ? (long)D.M[0] * D.M[1] : D.M[0];
    nwg = std::max<long>(nwg, nbz);
    nwg = std::max<long>(nwg, (nrows + 1) * d2);
    L.part_len = (size_t)nwg + 64;
    L.part_a = take(L.part_len * 8);
    L.part_b = take(L.part_len * 8);
    L.part_c = take(L.part_len * 8);
    L.nslots = std::max(1, nsl);
    L.slot_bytes = off - L.T1;
    off += (size_t)(L.nslots - 1) * L.slot_bytes;
    L.xsol = take((size_t)2 * d * vec);  // [kind][alpha][nc][Ns]
    L.xsol64 = take(precision == FFTGAL_FP32_ITER ? (size_t)d * vec : 0);
    const size_t nfld = (size_t)D.nshift * D.nfield * D.Mtot;
    L.gA64 = take(nfld * 8);
    L.gB64 = take(nfld * 8);
    L.gA32 = take(precision == FFTGAL_FP32_ITER ? nfld * 4 : 0);
    L.gB32 = take(precision == FFTGAL_FP32_ITER ? nfld * 4 : 0);
    L.gram = take(64 * 8);
    L.args = take(kArgsBytes);
    L.margs = take(slots ? kMultiArgsBytes : 0);
    L.status = take(6 * sizeof(CgStatus));
    L.hist = take((size_t)6 * 2 * (kMaxHist + 1) * 8);
    L.total = align256(off);
    return L;
}

constexpr long double kPiL = 3.141592653589793238462643383279502884L;

// Stage twiddles of a smooth length m, appended at entry `pos` of tab.
void stage_twiddles(int m, size_t &pos, std::vector<double> &tab, FftDesc *f) {
    std::vector<int> rad = factor(m);
    f->nst = (int)rad.size();
    int p = 1;
    for (int s = 0; s < f->nst; ++s) {
        const int r = rad[s];
        f->radix[s] = r;
        f->twoff[s] = (int)pos;
        for (int q = 1; q < r; ++q)
            for (int k = 0; k < p; ++k) {
                const long double ang = -2.0L * kPiL * (long double)(q * k) / (long double)(p * r);
                tab.push_back((double)cosl(ang));
                tab.push_back((double)sinl(ang));
            }
        pos += (size_t)(r - 1) * p;
        p *= r;
    }
}

void build_fft(int n, size_t tw_base_entry, std::vector<double> &tab, FftDesc *f) {
    size_t pos = tw_base_entry;
    f->n = n;
    f->L = n;
    f->blue = 0;
    f->choff = f->hoff = 0;
    if (is_smooth_odd(n)) {
        stage_twiddles(n, pos, tab, f);
        return;
    }
    // Bluestein (see FftDesc): chirp c_m = exp(i pi m^2 / n), angles reduced
    // exactly with m^2 mod 2n; H = DFT_L^-(v) / L with v_m = conj(c_m) at
    // m mod L for |m| < n, evaluated directly in long double
    const int L = smooth_odd(2 * n - 1);
    f->L = L;
    f->blue = 1;
    stage_twiddles(L, pos, tab, f);
    f->choff = (int)pos;
    std::vector<long double> cr(n), ci(n);
    for (int m = 0; m < n; ++m) {
        const long long q = ((long long)m * m) % (2LL * n);
        const long double ang = kPiL * (long double)q / (long double)n;
        cr[m] = cosl(ang);
        ci[m] = sinl(ang);
        tab.push_back((double)cr[m]);
        tab.push_back((double)ci[m]);
    }
    pos += (size_t)n;
    f->hoff = (int)pos;
    std::vector<long double> vr(L, 0.0L), vi(L, 0.0L);
    for (int m = -(n - 1); m <= n - 1; ++m) {
        const int am = m < 0 ? -m : m;
        const int idx = ((m % L) + L) % L;
        vr[idx] = cr[am];
        vi[idx] = -ci[am];
    }
    // the angle of term (m, k) depends only on q = m k mod L: one cosine and
    // sine per residue instead of per term
    std::vector<long double> wc(L), ws(L);
    for (int q = 0; q < L; ++q) {
        const long double ang = -2.0L * kPiL * (long double)q / (long double)L;
        wc[q] = cosl(ang);
        ws[q] = sinl(ang);
    }
    for (int k = 0; k < L; ++k) {
        long double hr = 0.0L, hi = 0.0L;
        for (int m = 0; m < L; ++m) {
            if (vr[m] == 0.0L && vi[m] == 0.0L) continue;
            const int q = (int)(((long long)m * k) % L);
            const long double c = wc[q], sn = ws[q];
            hr += vr[m] * c - vi[m] * sn;
            hi += vr[m] * sn + vi[m] * c;
        }
        tab.push_back((double)(hr / L));
        tab.push_back((double)(hi / L));
    }
    pos += (size_t)L;
}

}  // namespace

// One captured pass launch (see Plan::capture).
struct PassRec {
    int type;  // 0 pencil, 1 row
    int cls;
    int nouter;
    int grid;
    bool fp64;
    PencilArgs pa;
    RowArgs ra;
    // a pass over several problems (the shifts of the reduced Ga) in one
    // launch: np argument sets and their work-group offsets, uploaded to the
    // multi-argument region at table_off / woff_off (bytes)
    int np = 1;
    std::vector<PencilArgs> pas;
    std::vector<RowArgs> ras;
    std::vector<int> woff;
    size_t table_off = 0, woff_off = 0;
};

struct fftgal_plan {
    Dims D;
    Layout Lo;
    int precision = FFTGAL_FP64;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    FftDesc fM[3];  // transform along axis a on the M-grid
    FftDesc fP[3];  // transform along axis a of a voxel image
    int Pcur[3] = {0, 0, 0};
    bool have_mat = false;
    bool separate_gB = false;
    bool gen = false;  // the material uses the d (d + 1) / 2 general fields
    double A0[9], DA[9], B0[9], DB[9];
    bool solved[2][3] = {{false, false, false}, {false, false, false}};
    bool warm[2][3] = {{false, false, false}, {false, false, false}};  // x holds an initial iterate
    bool hist_valid[2][3] = {{false, false, false}, {false, false, false}};
    // voxel setup scratch: the layout's regions, or the workspace tail beyond
    // the layout when the image resolution exceeds what the layout provisions
    size_t vox_tw64 = 0, vox_tw32 = 0, vox_u = 0, vox_w = 0;
    fftgal_info last_info[2][3];
    int busy = 0;          // solves of this plan that are members of a batch
    size_t bws_off = 0, bws_len = 0;  // workspace of the internal batch (FFTGAL_CONCURRENT)
    std::vector<char> slot_used;                               // solve slots held by batch members
    bool in_batch[2][3] = {{false, false, false}, {false, false, false}};  // (kind, alpha) in a batch
    bool hist_on = false;  // per-iteration (rr, alpha) history; only when maxit <= kMaxHist
    int cur_alpha = 0;
    double btol = 0.0;  // bound tolerance of the stopping test (fftgal_set_bound_tol)
    bool gani = false;     // material sampled at the grid points of the order-N grid
    bool reduced = false;  // reduced Ga: 2^d shifted transforms of size N (Lemma reduce_grid)
    bool solo = true;      // small 2D grids: whole CG iterations in one work-group per solve
    // kernel timing (fftgal_set_timing): classes recorded
    unsigned timing_mask = 0;
    struct Ev {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Ev> evs;
    std::vector<hipEvent_t> pool;
    double t_ms[FFTGAL_K_COUNT] = {0};
    int32_t t_cnt[FFTGAL_K_COUNT] = {0};
    // pass capture: while non-null, pass launches are recorded instead of run
    std::vector<PassRec> *capture = nullptr;
    // intermediate slot of the operator passes being built (reduced Ga: one
    // per shift, so that the shifts of a pass can share a launch)
    int islot = 0;
    bool grouped = false;  // reduced Ga laid out with one slot per shift
    char *T1s() { return ws + so(Lo.T1) + (size_t)islot * Lo.t1_slot * 16; }
    char *T2s() { return ws + so(Lo.T2) + (size_t)islot * Lo.t2_slot * 16; }
    // solve slot whose per-solve region the passes being built use
    int slot = 0;
    size_t so(size_t off) const { return off + (size_t)slot * Lo.slot_bytes; }
    std::vector<unsigned char> margs_host;  // staging of the multi-shift argument tables
    int ring = 0;
    unsigned char ring_host[kRingSlots][kArgSlot] = {};
    unsigned char iter_host[kIterSlots][kArgSlot] = {};  // host images of the iteration slots
    char *arg_slot(int i) { return ws + Lo.args + kArgSlot * (size_t)i; }  // 0: offsets {0}
    char *iter_slot(int i) { return arg_slot(2 + i); }
    char *ring_slot(int i) { return arg_slot(2 + kIterSlots + i); }
    std::string err = "no error";
    int static_dev = -1;  // device whose static workspace this plan holds, or -1

    template <typename T> T *at(size_t off) { return reinterpret_cast<T *>(ws + off); }
    bool fp64_iter() const { return precision == FFTGAL_FP64; }
    int nc(int kind) const { return kind == KIND_E ? 1 : std::max(1, D.d - 1); }
    size_t vec_bytes() const { return (size_t)D.nc_max * D.Ns * 16; }
    void *xsol(int kind, int alpha) { return ws + Lo.xsol + ((size_t)kind * D.d + alpha) * vec_bytes(); }
    CgStatus *status(int kind, int alpha) { return at<CgStatus>(Lo.status) + kind * 3 + alpha; }
    double *hist(int kind, int alpha) {
        return at<double>(Lo.hist) + (size_t)(kind * 3 + alpha) * 2 * (kMaxHist + 1);
    }
};

typedef struct fftgal_plan Plan;  // the C function of the same name hides the tag in C++

namespace {

hipEvent_t pool_event(Plan *pl) {
    if (!pl->pool.empty()) {
        hipEvent_t e = pl->pool.back();
        pl->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches issued during its lifetime with two events of class
// `cls` when the plan's timing is on.
// Timing of one specialised launch: the dispatch records the two events at
// its own start and end (the kernel's duration, no marker packets).
struct TimedLaunch {
    Plan *pl;
    int cls;
    LaunchEv ev;
    TimedLaunch(Plan *p, int c) : pl(p), cls(c) {
        if ((pl->timing_mask >> cls) & 1u) {
            ev.start = pool_event(pl);
            ev.stop = ev.start ? pool_event(pl) : nullptr;
            if (ev.start && !ev.stop) {
                pl->pool.push_back(ev.start);
                ev.start = nullptr;
            }
        }
    }
    ~TimedLaunch() {
        if (ev.start) pl->evs.push_back({cls, ev.start, ev.stop});
    }
};

// Timing of a span of stream work between two recorded events.
struct Timed {
    Plan *pl;
    int cls;
    hipEvent_t a = nullptr;
    Timed(Plan *p, int c) : pl(p), cls(c) {
        if ((pl->timing_mask >> cls) & 1u) {
            a = pool_event(pl);
            if (a) (void)hipEventRecord(a, pl->stream);
        }
    }
    ~Timed() {
        if (a) {
            hipEvent_t b = pool_event(pl);
            if (b) {
                (void)hipEventRecord(b, pl->stream);
                pl->evs.push_back({cls, a, b});
            } else {
                pl->pool.push_back(a);
            }
        }
    }
};

}  // namespace

namespace {

int fail(Plan *pl, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (pl)
        pl->err = buf;
    else
        g_plan_error = buf;
    return code;
}

#define HIPCHECK(pl, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(pl, FFTGAL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---- pass builders -------------------------------------------------------

PencilArgs base_pencil(Plan *pl, const FftDesc &f, bool fp64, bool tabP = false) {
    PencilArgs a{};
    a.f = f;
    a.tw = pl->ws + (fp64 ? (tabP ? pl->vox_tw64 : pl->Lo.tw64) : (tabP ? pl->vox_tw32 : pl->Lo.tw32));
    a.d = pl->D.d;
    a.Nh = pl->D.Nh;
    a.Nmid = pl->D.d == 3 ? pl->D.N[1] : 0;
    a.scale = 1.0;
    a.nsol = 1;
    return a;
}

// Copy a specialised kernel's arguments into the next ring slot (stream
// ordered) and return the device address.
template <typename A>
void *ring_upload(Plan *pl, const A &a, hipError_t *err) {
    static_assert(sizeof(A) <= kArgSlot, "argument slot too small");
    const int i = pl->ring;
    pl->ring = (pl->ring + 1) % kRingSlots;
    std::memcpy(pl->ring_host[i], &a, sizeof(A));
    *err = hipMemcpyAsync(pl->ring_slot(i), pl->ring_host[i], sizeof(A), hipMemcpyHostToDevice, pl->stream);
    return pl->ring_slot(i);
}

// The generic kernels on small grids: fewer pencils (row pairs) per
// work-group while a launch has fewer work-groups than CUs and the halved
// batch (pencils times the components transformed together) still holds a
// point per thread of the work-group; a handful of
// work-groups, each transforming many long pencils one stage and one barrier
// at a time, otherwise sets the time of the pass (2D order 201: 114 -> 70 us
// per iteration), while batches of short pencils shrunk to one per
// work-group leave most threads idle (3D GaNi of order 41: 1.6x slower), and
// launches with a work-group per CU already lose by it (175^3: 5 % slower
// when aiming at two per CU).
constexpr long kGenericMinWorkGroups = 256;
constexpr int kGenericMinPoints = 256;

void configure_pencil_spread(PencilArgs &a, int nouter, bool fp64) {
    configure_pencil(a, fp64);
    if (a.fast) return;
    while (a.B > 1 && (long)pencil_grid_x(a) * nouter < kGenericMinWorkGroups &&
           (a.B / 2) * a.f.L * a.cb >= kGenericMinPoints) {
        a.B /= 2;
        fit_pencil_components(a, fp64);
    }
}

void configure_row_spread(RowArgs &r, bool fp64) {
    configure_row(r, fp64);
    if (r.fast) return;
    while (r.RP > 1 && row_grid(r) < kGenericMinWorkGroups && (r.RP / 2) * r.f.L >= kGenericMinPoints) {
        r.RP /= 2;
        fit_row_batch(r, fp64);
    }
}

int run_pencil(Plan *pl, PencilArgs &a, int nouter, bool fp64, int cls) {
    configure_pencil_spread(a, nouter, fp64);
    if (pencil_lds_bytes(a, fp64) > 160 * 1024)
        return fail(pl, FFTGAL_EINVAL, "transform length %d too large for one work-group", a.f.n);
    if (pl->capture) {
        PassRec r{};
        r.type = 0;
        r.cls = cls;
        r.nouter = nouter;
        r.grid = pencil_grid(a, nouter);
        r.fp64 = fp64;
        r.pa = a;
        pl->capture->push_back(r);
        return FFTGAL_OK;
    }
    if (a.fast) {
        hipError_t e;
        void *dev = ring_upload(pl, a, &e);
        HIPCHECK(pl, e);
        TimedLaunch t(pl, cls);
        HIPCHECK(pl, launch_pencil_multi(a, reinterpret_cast<const PencilArgs *>(dev),
                                         reinterpret_cast<const int *>(pl->arg_slot(0)), 1, pencil_grid(a, nouter),
                                         fp64, pl->stream, t.ev));
        return FFTGAL_OK;
    }
    Timed t(pl, cls);
    HIPCHECK(pl, launch_pencil(a, nouter, fp64, pl->stream));
    return FFTGAL_OK;
}

int run_row(Plan *pl, RowArgs &r, bool fp64, int cls) {
    configure_row_spread(r, fp64);
    const int nz = r.mode == ROW_GRAM ? r.ncomp : r.d;
    if (row_lds_bytes(r, fp64) > 160 * 1024)
        return fail(pl, FFTGAL_EINVAL, "row length %d with %d components too large for one work-group", r.f.n, nz);
    if (pl->capture) {
        PassRec rec{};
        rec.type = 1;
        rec.cls = cls;
        rec.nouter = 1;
        rec.grid = row_grid(r);
        rec.fp64 = fp64;
        rec.ra = r;
        pl->capture->push_back(rec);
        return FFTGAL_OK;
    }
    if (r.fast) {
        hipError_t e;
        void *dev = ring_upload(pl, r, &e);
        HIPCHECK(pl, e);
        TimedLaunch t(pl, cls);
        HIPCHECK(pl, launch_row_multi(r, reinterpret_cast<const RowArgs *>(dev),
                                      reinterpret_cast<const int *>(pl->arg_slot(0)), 1, row_grid(r), fp64,
                                      pl->stream, t.ev));
        return FFTGAL_OK;
    }
    Timed t(pl, cls);
    HIPCHECK(pl, launch_row(r, fp64, pl->stream));
    return FFTGAL_OK;
}

// Shift s (bit d-1-a of s is s_a) of the reduced Ga on an EXPAND or PROJECT pass.
void set_shift(Plan *pl, PencilArgs &a, int shift) {
    for (int x = 0; x < 3; ++x) {
        a.shift[x] = x < pl->D.d ? (shift >> (pl->D.d - 1 - x)) & 1 : 0;
        a.Nfull[x] = pl->D.N[x];
    }
}

// The inverse half of the operator: CG state (n_c components per solution)
// -> d spatial components per solution on the M-grid, stored as half-spectrum
// rows along the last axis (T1 in 2D, T2 in 3D).
int inverse_passes(Plan *pl, bool fp64, int kind, const void *state, long st_ss, int nsol,
                   bool update_p, const CgStatus *st, void **rows_out, int cls_expand, int cls_inv, int shift = 0) {
    const Dims &D = pl->D;
    const int d = D.d;
    const size_t es = fp64 ? 16 : 8;
    // several solutions (the energy quadrature): one launch per solution, so
    // that each takes the specialised kernels; solution s fills the
    // components s d .. s d + d - 1 of the intermediates
    for (int s = 0; s < nsol; ++s) {
        PencilArgs a = base_pencil(pl, pl->fM[0], fp64);
        set_shift(pl, a, shift);
        a.pro = PRO_EXPAND;
        a.epi = EPI_PLAIN;
        a.kind = kind;
        a.nc = pl->nc(kind);
        a.ncomp = d;
        a.nsol = 1;
        a.sgn = +1;
        a.L_in = D.N[0];
        a.L_out = D.M[0];
        a.st_cs = D.Ns;
        a.st_ss = st_ss;
        a.update_p = update_p ? 1 : 0;
        a.status = st;
        if (update_p) {
            a.st_r = pl->ws + pl->so(pl->Lo.r);
            a.st_p = pl->ws + pl->so(pl->Lo.p);
        } else {
            a.st_x = state == nullptr ? nullptr : static_cast<const char *>(state) + (size_t)s * st_ss * es;
        }
        if (d == 3) {
            a.nb = D.N[1] * D.Nh;
            a.in_ls = (long)D.N[1] * D.Nh;
            a.out_ls = (long)D.N[1] * D.Nh;
            a.out_cs = (long)D.M[0] * D.N[1] * D.Nh;
        } else {
            a.nb = D.Nh;
            a.in_ls = D.Nh;
            a.out_ls = D.Nh;
            a.out_cs = (long)D.M[0] * D.Nh;
        }
        a.out = pl->T1s() + (size_t)s * d * a.out_cs * es;
        int rc = run_pencil(pl, a, 1, fp64, cls_expand);
        if (rc) return rc;
    }
    if (d == 2) {
        *rows_out = pl->T1s();
        return FFTGAL_OK;
    }
    for (int s = 0; s < nsol; ++s) {
        PencilArgs b = base_pencil(pl, pl->fM[1], fp64);
        b.pro = PRO_PLAIN;
        b.epi = EPI_PLAIN;
        b.ncomp = d;
        b.sgn = +1;
        b.L_in = D.N[1];
        b.L_out = D.M[1];
        b.status = st;
        b.nb = D.Nh;
        b.in_cs = (long)D.M[0] * D.N[1] * D.Nh;
        b.in_os = (long)D.N[1] * D.Nh;
        b.in_ls = D.Nh;
        b.out_cs = (long)D.M[0] * D.M[1] * D.Nh;
        b.out_os = (long)D.M[1] * D.Nh;
        b.out_ls = D.Nh;
        b.in = pl->T1s() + (size_t)s * d * b.in_cs * es;
        b.out = pl->T2s() + (size_t)s * d * b.out_cs * es;
        const int rc = run_pencil(pl, b, D.M[0], fp64, cls_inv);
        if (rc) return rc;
    }
    *rows_out = pl->T2s();
    return FFTGAL_OK;
}

// The forward half: half-spectrum rows -> projected CG vector q (scaled),
// plus partial sums of (dot, q) (or (q, q) when dot == nullptr).
int forward_passes(Plan *pl, bool fp64, int kind, void *rows, void *q, const void *dot, double scale,
                   const CgStatus *st, double *partial, int *nparts, int cls_fwd, int cls_proj, int shift = 0,
                   bool accumulate = false) {
    const Dims &D = pl->D;
    const int d = D.d;
    void *src = rows;
    if (d == 3) {
        PencilArgs b = base_pencil(pl, pl->fM[1], fp64);
        b.pro = PRO_PLAIN;
        b.epi = EPI_PLAIN;
        b.ncomp = d;
        b.sgn = -1;
        b.L_in = D.M[1];
        b.L_out = D.N[1];
        b.status = st;
        b.in = rows;
        b.out = pl->T1s();
        b.nb = D.Nh;
        b.in_cs = (long)D.M[0] * D.M[1] * D.Nh;
        b.in_os = (long)D.M[1] * D.Nh;
        b.in_ls = D.Nh;
        b.out_cs = (long)D.M[0] * D.N[1] * D.Nh;
        b.out_os = (long)D.N[1] * D.Nh;
        b.out_ls = D.Nh;
        int rc = run_pencil(pl, b, D.M[0], fp64, cls_fwd);
        if (rc) return rc;
        src = pl->T1s();
    }
    PencilArgs a = base_pencil(pl, pl->fM[0], fp64);
    set_shift(pl, a, shift);
    a.accumulate = accumulate ? 1 : 0;
    a.pro = PRO_PLAIN;
    a.epi = EPI_PROJECT;
    a.kind = kind;
    a.nc = pl->nc(kind);
    a.ncomp = d;
    a.sgn = -1;
    a.scale = scale;
    a.L_in = D.M[0];
    a.L_out = D.N[0];
    a.status = st;
    a.in = src;
    a.out = q;
    a.st_dot = dot;
    a.partial = partial;
    if (d == 3) {
        a.nb = D.N[1] * D.Nh;
        a.in_cs = (long)D.M[0] * D.N[1] * D.Nh;
        a.in_ls = (long)D.N[1] * D.Nh;
        a.out_ls = (long)D.N[1] * D.Nh;
    } else {
        a.nb = D.Nh;
        a.in_cs = (long)D.M[0] * D.Nh;
        a.in_ls = D.Nh;
        a.out_ls = D.Nh;
    }
    a.out_cs = D.Ns;
    int rc = run_pencil(pl, a, 1, fp64, cls_proj);
    if (rc) return rc;
    *nparts = pencil_grid_x(a);
    return FFTGAL_OK;
}

RowArgs base_row(Plan *pl, bool fp64, int mode, void *rows, int kind, int shift = 0) {
    const Dims &D = pl->D;
    RowArgs r{};
    r.data = rows;
    r.nrows = (D.d == 3) ? D.M[0] * D.M[1] : D.M[0];
    r.Nh_row = D.Nh;
    r.cs = (long)r.nrows * D.Nh;
    r.f = pl->fM[D.d - 1];
    r.tw = pl->ws + (fp64 ? pl->Lo.tw64 : pl->Lo.tw32);
    r.d = D.d;
    r.ncomp = D.d;
    r.mode = mode;
    r.scale = 1.0;
    const bool gsep = pl->separate_gB && kind == KIND_J;
    if (fp64)
        r.g = pl->ws + (gsep ? pl->Lo.gB64 : pl->Lo.gA64) + (size_t)shift * D.Mtot * 8;
    else
        r.g = pl->ws + (gsep ? pl->Lo.gB32 : pl->Lo.gA32) + (size_t)shift * D.Mtot * 4;
    r.nfield = 1;
    r.gstride = D.Mtot;
    if (pl->gen) {
        r.nfield = D.nfield;
        r.iso = 0;
        for (int i = 0; i < 9; ++i) r.A0[i] = r.D[i] = 0.0;
        return r;
    }
    const double *c0 = kind == KIND_E ? pl->A0 : pl->B0;
    const double *c1 = kind == KIND_E ? pl->DA : pl->DB;
    for (int i = 0; i < 9; ++i) {
        r.A0[i] = c0[i];
        r.D[i] = c1[i];
    }
    // isotropic when both matrices are exact multiples of the identity
    r.iso = 1;
    for (int i = 0; i < D.d; ++i)
        for (int j = 0; j < D.d; ++j) {
            const int k = i * D.d + j;
            if (i == j ? (c0[k] != c0[0] || c1[k] != c1[0]) : (c0[k] != 0.0 || c1[k] != 0.0)) r.iso = 0;
        }
    return r;
}

// ---- material setup --------------------------------------------------------

// Inverse transforms of a Fourier half-grid (stored wrapped, layout
// [n1][n2][n3 >= 0]; extents Li[0], Li[1] and Lhi along the last axis; by
// default Z_{2N-1}) into a real field on the M-grid (eq. MBA_GA).
int series_to_field(Plan *pl, void *coef, double *field, const int *Li = nullptr, int Lhi = 0) {
    const Dims &D = pl->D;
    const int d = D.d;
    const int L0 = Li ? Li[0] : D.L[0], L1 = Li ? Li[1] : D.L[1], Lh = Li ? Lhi : D.Lh;
    void *U = pl->ws + pl->so(pl->Lo.T2);
    void *W = pl->ws + pl->so(pl->Lo.T1);
    void *cur = coef;
    PencilArgs a = base_pencil(pl, pl->fM[0], true);
    a.pro = PRO_PLAIN;
    a.epi = EPI_PLAIN;
    a.ncomp = 1;
    a.sgn = +1;
    a.L_in = L0;
    a.L_out = D.M[0];
    a.in = cur;
    void *dst1 = (cur == U) ? W : U;
    a.out = dst1;
    if (d == 3) {
        a.nb = L1 * Lh;
        a.in_ls = a.out_ls = (long)L1 * Lh;
    } else {
        a.nb = Lh;
        a.in_ls = a.out_ls = Lh;
    }
    int rc = run_pencil(pl, a, 1, true, FFTGAL_K_SETUP);
    if (rc) return rc;
    cur = dst1;
    if (d == 3) {
        PencilArgs b = base_pencil(pl, pl->fM[1], true);
        b.pro = PRO_PLAIN;
        b.epi = EPI_PLAIN;
        b.ncomp = 1;
        b.sgn = +1;
        b.L_in = L1;
        b.L_out = D.M[1];
        b.in = cur;
        void *dst2 = (cur == U) ? W : U;
        b.out = dst2;
        b.nb = Lh;
        b.in_os = (long)L1 * Lh;
        b.in_ls = Lh;
        b.out_os = (long)D.M[1] * Lh;
        b.out_ls = Lh;
        rc = run_pencil(pl, b, D.M[0], true, FFTGAL_K_SETUP);
        if (rc) return rc;
        cur = dst2;
    }
    RowArgs r{};
    r.data = cur;
    r.nrows = (d == 3) ? D.M[0] * D.M[1] : D.M[0];
    r.Nh_row = Lh;
    r.cs = 0;
    r.f = pl->fM[d - 1];
    r.tw = pl->ws + pl->Lo.tw64;
    r.ncomp = 1;
    r.d = d;
    r.mode = ROW_C2R;
    r.real_out = field;
    r.real_stride = D.M[d - 1];
    r.scale = 1.0;
    return run_row(pl, r, true, FFTGAL_K_SETUP);
}

// Reduced Ga (Lemma reduce_grid): the double-grid field at the points
// (2r - s) / (2N) of each shift s is the size-N inverse DFT of the series
// folded onto Z_N with the phase of s.  The series is parked in the solution
// region (free while the material is set), each fold goes to W and is
// transformed into field + s |N|.
int series_to_shifted_fields(Plan *pl, void *coef, double *field) {
    const Dims &D = pl->D;
    const int d = D.d;
    const size_t nser = (size_t)(d == 3 ? (long)D.L[0] * D.L[1] : (long)D.L[0]) * D.Lh * 16;
    if (nser > (size_t)2 * d * pl->vec_bytes()) return fail(pl, FFTGAL_EINVAL, "series scratch too small");
    void *ser = pl->ws + pl->Lo.xsol;
    void *W = pl->ws + pl->so(pl->Lo.T1);
    HIPCHECK(pl, hipMemcpyAsync(ser, coef, nser, hipMemcpyDeviceToDevice, pl->stream));
    const int Ni[2] = {D.N[0], D.N[1]};
    for (int s = 0; s < D.nshift; ++s) {
        int sh[3];
        for (int a = 0; a < 3; ++a) sh[a] = a < d ? (s >> (d - 1 - a)) & 1 : 0;
        {
            Timed t(pl, FFTGAL_K_SETUP);
            HIPCHECK(pl, launch_fold_series(W, ser, d, D.N, D.L, D.Lh, sh, pl->stream));
        }
        const int rc = series_to_field(pl, W, field + (size_t)s * D.Mtot, Ni, D.Nh);
        if (rc) return rc;
    }
    return FFTGAL_OK;
}

// Voxel image (host, P^d doubles, row-major) -> truncated/extended Fourier
// half-grid on Z_{2N-1} times the sinc window of psi = rect_{1/P}
// (Lemma grid_compos, Remark eval_with_FFT), left in the returned buffer.
int voxel_series(Plan *pl, const double *img_dev, int imgmap, double vmax, void **coef_out) {
    const Dims &D = pl->D;
    const int d = D.d;
    const int *P = pl->Pcur;
    void *U = pl->ws + pl->vox_u;
    void *W = pl->ws + pl->vox_w;
    long Ptot = 1;
    for (int a = 0; a < d; ++a) Ptot *= P[a];
    // rows along the last axis: R2C, keep n_d in [0, N_d)
    RowArgs r{};
    r.data = W;
    r.nrows = (int)(Ptot / P[d - 1]);
    r.Nh_row = D.Lh;
    r.cs = 0;
    r.f = pl->fP[d - 1];
    r.tw = pl->ws + pl->vox_tw64;
    r.ncomp = 1;
    r.d = d;
    r.mode = ROW_R2C;
    r.real_in = img_dev;
    r.real_stride = P[d - 1];
    r.imgmap = imgmap;
    r.vmax = vmax;
    r.scale = 1.0;
    int rc = run_row(pl, r, true, FFTGAL_K_SETUP);
    if (rc) return rc;
    void *cur = W;
    if (d == 3) {
        PencilArgs b = base_pencil(pl, pl->fP[1], true, true);
        b.pro = PRO_PLAIN;
        b.epi = EPI_PLAIN;
        b.ncomp = 1;
        b.sgn = -1;
        b.L_in = P[1];
        b.L_out = D.L[1];
        b.in = W;
        b.out = U;
        b.nb = D.Lh;
        b.in_os = (long)P[1] * D.Lh;
        b.in_ls = D.Lh;
        b.out_os = (long)D.L[1] * D.Lh;
        b.out_ls = D.Lh;
        rc = run_pencil(pl, b, P[0], true, FFTGAL_K_SETUP);
        if (rc) return rc;
        cur = U;
    }
    PencilArgs a = base_pencil(pl, pl->fP[0], true, true);
    a.pro = PRO_PLAIN;
    a.epi = EPI_WINDOW;
    a.ncomp = 1;
    a.sgn = -1;
    a.L_in = P[0];
    a.L_out = D.L[0];
    a.in = cur;
    void *dst = (cur == U) ? W : U;
    a.out = dst;
    a.Nh = D.Lh;
    a.Nmid = (d == 3) ? D.L[1] : 0;
    a.Pw[0] = P[0];
    a.Pw[1] = P[1];
    a.Pw[2] = d == 3 ? P[2] : 1;
    a.winscale = 1.0 / (double)Ptot;
    if (d == 3) {
        a.nb = D.L[1] * D.Lh;
        a.in_ls = a.out_ls = (long)D.L[1] * D.Lh;
    } else {
        a.nb = D.Lh;
        a.in_ls = a.out_ls = D.Lh;
    }
    rc = run_pencil(pl, a, 1, true, FFTGAL_K_SETUP);
    if (rc) return rc;
    *coef_out = dst;
    return FFTGAL_OK;
}

bool chol_spd(const double *A, int d) {
    double L[9] = {0};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * d + j];
            for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
            if (i == j) {
                if (!(s > 0.0) || !std::isfinite(s)) return false;
                L[i * d + i] = std::sqrt(s);
            } else {
                L[i * d + j] = s / L[j * d + j];
            }
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            if (std::fabs(A[i * d + j] - A[j * d + i]) > 1e-12 * (std::fabs(A[i * d + j]) + std::fabs(A[j * d + i])))
                return false;
    return true;
}

bool inv_small(const double *A, int d, double *out) {
    long double m[3][6];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < 2 * d; ++j) m[i][j] = j < d ? A[i * d + j] : (j - d == i ? 1.0L : 0.0L);
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int i = c + 1; i < d; ++i)
            if (fabsl(m[i][c]) > fabsl(m[piv][c])) piv = i;
        if (m[piv][c] == 0.0L) return false;
        if (piv != c)
            for (int j = 0; j < 2 * d; ++j) std::swap(m[c][j], m[piv][j]);
        const long double inv = 1.0L / m[c][c];
        for (int j = 0; j < 2 * d; ++j) m[c][j] *= inv;
        for (int i = 0; i < d; ++i)
            if (i != c) {
                const long double f = m[i][c];
                for (int j = 0; j < 2 * d; ++j) m[i][j] -= f * m[c][j];
            }
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) out[i * d + j] = (double)m[i][d + j];
    return true;
}

bool is_iso(const double *A, int d, double *a) {
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            if (i != j && A[i * d + j] != 0.0) return false;
    for (int i = 1; i < d; ++i)
        if (A[i * d + i] != A[0]) return false;
    *a = A[0];
    return true;
}

double min_image(double x) { return x - std::nearbyint(x); }

bool overlap(int d, int s1, const double *c1, const double *h1, int s2, const double *c2, const double *h2) {
    double dc[3];
    for (int a = 0; a < d; ++a) dc[a] = std::fabs(min_image(c1[a] - c2[a]));
    if (s1 == FFTGAL_RECT && s2 == FFTGAL_RECT) {
        for (int a = 0; a < d; ++a)
            if (dc[a] >= 0.5 * (h1[a] + h2[a])) return false;
        return true;
    }
    if (s1 == FFTGAL_CIRC && s2 == FFTGAL_CIRC) {
        double s = 0;
        for (int a = 0; a < d; ++a) s += dc[a] * dc[a];
        return std::sqrt(s) < h1[0] + h2[0];
    }
    const double *hb = s1 == FFTGAL_RECT ? h1 : h2;
    const double r = s1 == FFTGAL_CIRC ? h1[0] : h2[0];
    double s = 0;
    for (int a = 0; a < d; ++a) {
        const double e = std::max(0.0, dc[a] - 0.5 * hb[a]);
        s += e * e;
    }
    return std::sqrt(s) < r;
}

// ---- CG driver ---------------------------------------------------------------

// One CG iteration of a solve in captured form: its transform passes (in
// order) and the arguments of the multi-problem CG kernels.
struct IterCfg {
    std::vector<PassRec> passes;
    UpdArgs upd;
    CgItem item;
    bool fp64 = true;
};

// Group the per-shift passes of a reduced-Ga iteration (k passes per shift,
// shift-major) into passes over all shifts: the EXPAND of shift 0 alone (it
// forms p, which the other shifts read), the EXPAND of the other shifts
// together, then each later pass of all shifts together, every shift on its
// own intermediate slot.  False (and no change) unless every pass runs a
// specialised kernel and the argument tables fit their region.
bool group_shifts(std::vector<PassRec> &ps, int nshift) {
    if (nshift < 2 || ps.empty() || ps.size() % nshift) return false;
    for (const auto &r : ps)
        if (!(r.type == 0 ? r.pa.fast : r.ra.fast)) return false;
    const size_t k = ps.size() / nshift;
    std::vector<PassRec> out;
    out.push_back(ps[0]);
    size_t off = 0;
    auto group = [&](size_t j, int s0) {
        PassRec g = ps[s0 * k + j];
        g.np = nshift - s0;
        int tot = 0;
        for (int sh = s0; sh < nshift; ++sh) {
            const PassRec &m = ps[sh * k + j];
            g.woff.push_back(tot);
            tot += m.grid;
            if (m.type == 0)
                g.pas.push_back(m.pa);
            else
                g.ras.push_back(m.ra);
        }
        g.grid = tot;
        g.table_off = off;
        off += ((size_t)g.np * (g.type == 0 ? sizeof(PencilArgs) : sizeof(RowArgs)) + 255) / 256 * 256;
        g.woff_off = off;
        off += ((size_t)g.np * sizeof(int) + 255) / 256 * 256;
        out.push_back(std::move(g));
    };
    group(0, 1);
    for (size_t j = 1; j < k; ++j) group(j, 0);
    if (off > kMultiArgsBytes) return false;
    ps.swap(out);
    return true;
}

int capture_iteration(Plan *pl, int kind, int alpha, bool fp64, IterCfg *cfg) {
    const Dims &D = pl->D;
    CgStatus *st = pl->status(kind, alpha);
    void *x = pl->xsol(kind, alpha);
    cfg->fp64 = fp64;
    // reduced Ga: q = sum_s 2^{-d} S*(s) F A(s) F^{-1} S(s) p over the shifted
    // grids (Algorithm 3); the first shift also forms p = r + beta p.  With
    // specialised kernels every shift gets its own intermediates and its own
    // projected vector q_s (summed by the update pass in shift order), so that
    // the shifts of each pass share a launch; otherwise the shifts run one
    // after another, accumulating into q.
    const bool multi = pl->grouped;
    int npq = 0, npq_shift = 0;
    auto build = [&](bool grouped) -> int {
        cfg->passes.clear();
        pl->capture = &cfg->passes;
        void *rows = nullptr;
        int rc = FFTGAL_OK;
        for (int s = 0; s < D.nshift && !rc; ++s) {
            pl->islot = grouped ? s : 0;
            rc = inverse_passes(pl, fp64, kind, s == 0 ? nullptr : pl->ws + pl->so(pl->Lo.p), 0, 1, s == 0, st, &rows,
                                FFTGAL_K_EXPAND, FFTGAL_K_PENCIL_INV, s);
            if (!rc) {
                RowArgs r = base_row(pl, fp64, ROW_OPER, rows, kind, s);
                r.status = st;
                rc = run_row(pl, r, fp64, FFTGAL_K_ROW);
            }
            if (!rc) {
                char *q = pl->ws + pl->so(pl->Lo.q) + (grouped ? (size_t)s * pl->vec_bytes() : 0);
                double *part = pl->at<double>(pl->so(pl->Lo.part_a)) + (grouped ? (size_t)s * npq_shift : 0);
                rc = forward_passes(pl, fp64, kind, rows, q, pl->ws + pl->so(pl->Lo.p), 1.0 / ((double)D.nshift * D.Mtot),
                                    st, part, &npq, FFTGAL_K_PENCIL_FWD, FFTGAL_K_PROJECT, s, !grouped && s > 0);
                if (s == 0) npq_shift = npq;
            }
        }
        pl->islot = 0;
        pl->capture = nullptr;
        return rc;
    };
    bool grouped = multi;
    int rc = build(grouped);
    if (!rc && grouped) {
        if ((size_t)D.nshift * npq_shift > pl->Lo.part_len || !group_shifts(cfg->passes, D.nshift)) {
            grouped = false;
            rc = build(false);
        }
    }
    if (rc) return rc;
    const int nc = pl->nc(kind);
    UpdArgs u{};
    u.x = x;
    u.r = pl->ws + pl->so(pl->Lo.r);
    u.p = pl->ws + pl->so(pl->Lo.p);
    u.q = pl->ws + pl->so(pl->Lo.q);
    u.n_per_comp = D.Ns;
    u.cs = D.Ns;
    u.nc = nc;
    u.Nh = D.Nh;
    u.nblocks = update_blocks((long)nc * D.Ns);
    u.st = st;
    u.partial = pl->at<double>(pl->so(pl->Lo.part_c));
    u.pq_part = pl->at<double>(pl->so(pl->Lo.part_a));
    u.npq = grouped ? D.nshift * npq_shift : npq;
    u.nq = grouped ? D.nshift : 1;
    u.q_ss = (long)(pl->vec_bytes() / (fp64 ? 16 : 8));
    cfg->upd = u;
    CgItem it{};
    it.st = st;
    it.rr_part = pl->at<double>(pl->so(pl->Lo.part_c));
    it.nrr = u.nblocks;
    it.hist = pl->hist_on ? pl->hist(kind, alpha) : nullptr;
    it.hist_cap = kMaxHist + 1;
    it.mirror = nullptr;
    cfg->item = it;
    return FFTGAL_OK;
}

// Upload a captured iteration into the plan's iteration argument slots.
int upload_iteration(Plan *pl, const IterCfg &cfg) {
    if (cfg.passes.size() > (size_t)kMaxPasses) return fail(pl, FFTGAL_EINVAL, "too many passes");
    size_t mused = 0;
    for (const PassRec &r : cfg.passes) {
        if (r.np < 2) continue;
        if (pl->margs_host.size() < kMultiArgsBytes) pl->margs_host.assign(kMultiArgsBytes, 0);
        const size_t tb = (size_t)r.np * (r.type == 0 ? sizeof(PencilArgs) : sizeof(RowArgs));
        std::memcpy(pl->margs_host.data() + r.table_off, r.type == 0 ? (const void *)r.pas.data() : (const void *)r.ras.data(),
                    tb);
        std::memcpy(pl->margs_host.data() + r.woff_off, r.woff.data(), (size_t)r.np * sizeof(int));
        mused = std::max(mused, r.woff_off + (size_t)r.np * sizeof(int));
    }
    if (mused > 0)
        HIPCHECK(pl, hipMemcpyAsync(pl->ws + pl->Lo.margs, pl->margs_host.data(), mused, hipMemcpyHostToDevice,
                                    pl->stream));
    // every write to an iteration slot goes through its host image, so the
    // slots of the passes go up in one copy (slots of passes that take their
    // arguments elsewhere carry their previous, unread contents), and the
    // update and CG item in a second
    for (size_t i = 0; i < cfg.passes.size(); ++i) {
        const PassRec &r = cfg.passes[i];
        const bool fast = r.type == 0 ? r.pa.fast : r.ra.fast;
        if (!fast || r.np > 1) continue;
        const size_t sz = r.type == 0 ? sizeof(PencilArgs) : sizeof(RowArgs);
        std::memcpy(pl->iter_host[i], r.type == 0 ? (const void *)&r.pa : (const void *)&r.ra, sz);
    }
    if (!cfg.passes.empty())
        HIPCHECK(pl, hipMemcpyAsync(pl->iter_slot(0), pl->iter_host[0], cfg.passes.size() * kArgSlot,
                                    hipMemcpyHostToDevice, pl->stream));
    std::memcpy(pl->iter_host[kMaxPasses], &cfg.upd, sizeof(UpdArgs));
    std::memcpy(pl->iter_host[kMaxPasses + 1], &cfg.item, sizeof(CgItem));
    HIPCHECK(pl, hipMemcpyAsync(pl->iter_slot(kMaxPasses), pl->iter_host[kMaxPasses], 2 * kArgSlot,
                                hipMemcpyHostToDevice, pl->stream));
    return FFTGAL_OK;
}

// Launch one captured pass of a single plan (specialised passes read their
// arguments from `dev_args`).
int launch_pass(Plan *pl, const PassRec &r, const void *dev_args) {
    const int *woff0 = reinterpret_cast<const int *>(pl->arg_slot(0));
    if (r.np > 1) {  // several shifts in one launch: argument table and offsets
        const char *tab = pl->ws + pl->Lo.margs + r.table_off;
        const int *woff = reinterpret_cast<const int *>(pl->ws + pl->Lo.margs + r.woff_off);
        TimedLaunch t(pl, r.cls);
        if (r.type == 0)
            HIPCHECK(pl, launch_pencil_multi(r.pa, reinterpret_cast<const PencilArgs *>(tab), woff, r.np, r.grid, r.fp64,
                                             pl->stream, t.ev));
        else
            HIPCHECK(pl, launch_row_multi(r.ra, reinterpret_cast<const RowArgs *>(tab), woff, r.np, r.grid, r.fp64,
                                          pl->stream, t.ev));
        return FFTGAL_OK;
    }
    if (r.type == 0) {
        if (r.pa.fast) {
            TimedLaunch t(pl, r.cls);
            HIPCHECK(pl, launch_pencil_multi(r.pa, reinterpret_cast<const PencilArgs *>(dev_args), woff0, 1, r.grid,
                                             r.fp64, pl->stream, t.ev));
        } else {
            Timed t(pl, r.cls);
            HIPCHECK(pl, launch_pencil(r.pa, r.nouter, r.fp64, pl->stream));
        }
    } else {
        if (r.ra.fast) {
            TimedLaunch t(pl, r.cls);
            HIPCHECK(pl, launch_row_multi(r.ra, reinterpret_cast<const RowArgs *>(dev_args), woff0, 1, r.grid, r.fp64,
                                          pl->stream, t.ev));
        } else {
            Timed t(pl, r.cls);
            HIPCHECK(pl, launch_row(r.ra, r.fp64, pl->stream));
        }
    }
    return FFTGAL_OK;
}

int enqueue_iteration(Plan *pl, const IterCfg &cfg) {
    for (size_t i = 0; i < cfg.passes.size(); ++i) {
        const int rc = launch_pass(pl, cfg.passes[i], pl->iter_slot((int)i));
        if (rc) return rc;
    }
    const CgItem *item = reinterpret_cast<const CgItem *>(pl->iter_slot(kMaxPasses + 1));
    const UpdArgs *upd = reinterpret_cast<const UpdArgs *>(pl->iter_slot(kMaxPasses));
    const int *woff0 = reinterpret_cast<const int *>(pl->arg_slot(0));
    {
        TimedLaunch t(pl, FFTGAL_K_CG_UPDATE);
        HIPCHECK(pl, launch_cg_update_multi(upd, woff0, 1, cfg.upd.nblocks, cfg.fp64, pl->stream, t.ev));
    }
    TimedLaunch t(pl, FFTGAL_K_CG_SCALAR);
    HIPCHECK(pl, launch_cg_check_multi(item, 1, pl->stream, t.ev));
    return FFTGAL_OK;
}

// Update-grid arguments of a solve's vectors (CG update geometry).
UpdArgs solve_vectors(Plan *pl, int kind, int alpha) {
    UpdArgs u{};
    u.x = pl->xsol(kind, alpha);
    u.r = pl->ws + pl->so(pl->Lo.r);
    u.p = pl->ws + pl->so(pl->Lo.p);
    u.q = pl->ws + pl->so(pl->Lo.q);
    u.n_per_comp = pl->D.Ns;
    u.cs = pl->D.Ns;
    u.nc = pl->nc(kind);
    u.Nh = pl->D.Nh;
    u.nblocks = update_blocks((long)u.nc * pl->D.Ns);
    u.st = pl->status(kind, alpha);
    return u;
}

// Best-iterate checkpoint of an FP32 solve: K x with the partials of (x, K x)
// (the operator passes of an iteration, reading the iterate instead of
// forming p), then the energy test (see launch_cg_checkpoint).  Periodic
// checkpoints are skipped on the device once the solve is done; the final
// one runs after a solve that did not converge.
int checkpoint(Plan *pl, int kind, int alpha, bool final) {
    const Dims &D = pl->D;
    CgStatus *st = pl->status(kind, alpha);
    void *x = pl->xsol(kind, alpha);
    const CgStatus *gate = final ? nullptr : st;
    const int cls = FFTGAL_K_CHECKPOINT;
    int nq = 0;
    for (int s = 0; s < D.nshift; ++s) {  // reduced Ga: the shifts in turn, summed into q
        void *rows = nullptr;
        int rc = inverse_passes(pl, false, kind, x, 0, 1, false, gate, &rows, cls, cls, s);
        if (rc) return rc;
        RowArgs r = base_row(pl, false, ROW_OPER, rows, kind, s);
        r.status = gate;
        rc = run_row(pl, r, false, cls);
        if (rc) return rc;
        rc = forward_passes(pl, false, kind, rows, pl->ws + pl->so(pl->Lo.q), x, 1.0 / ((double)D.nshift * D.Mtot), gate,
                            pl->at<double>(pl->so(pl->Lo.part_a)), &nq, cls, cls, s, s > 0);
        if (rc) return rc;
    }
    const UpdArgs u = solve_vectors(pl, kind, alpha);
    Timed t(pl, cls);
    HIPCHECK(pl, launch_cg_checkpoint(u, pl->ws + pl->so(pl->Lo.bvec), pl->ws + pl->so(pl->Lo.xbest), pl->at<double>(pl->so(pl->Lo.part_a)),
                                      nq, pl->at<double>(pl->so(pl->Lo.part_b)), kCkptEvery, final ? 1 : 0, false,
                                      pl->stream));
    return FFTGAL_OK;
}

// Right-hand side r_0 = -P^* F_M (A_M E), ||A_M E||, status initialisation,
// x = p = 0 (stream ordered; no host synchronisation).
int start_solve(Plan *pl, int kind, int alpha, double rtol, int maxit) {
    const Dims &D = pl->D;
    const bool fp64 = pl->fp64_iter();
    CgStatus *st = pl->status(kind, alpha);
    void *x = pl->xsol(kind, alpha);
    pl->hist_on = maxit <= kMaxHist;
    pl->hist_valid[kind][alpha] = pl->hist_on;
    pl->cur_alpha = alpha;
    const size_t es = fp64 ? 16 : 8;
    const size_t vbytes = (size_t)pl->nc(kind) * D.Ns * es;
    void *rows = pl->ws + (D.d == 3 ? pl->so(pl->Lo.T2) : pl->so(pl->Lo.T1));
    // one pass per shifted grid (reduced Ga; one grid otherwise), the load
    // partials of shift s at offset s * nload, the projected loads summed in r
    const double npts = (double)D.nshift * D.Mtot;
    int nload = 0, nrr = 0, rc = FFTGAL_OK;
    for (int s = 0; s < D.nshift; ++s) {
        RowArgs r = base_row(pl, fp64, ROW_RHS, rows, kind, s);
        for (int a = 0; a < 3; ++a) r.E[a] = (a == alpha) ? 1.0 : 0.0;
        configure_row_spread(r, fp64);  // the work-group count fixes the partial offsets
        nload = row_grid(r);
        if ((size_t)D.nshift * nload > pl->Lo.part_len) return fail(pl, FFTGAL_EINVAL, "partial buffers too small");
        r.partial = pl->at<double>(pl->so(pl->Lo.part_b)) + (size_t)s * nload;
        r.partial2 = pl->at<double>(pl->so(pl->Lo.part_c)) + (size_t)s * nload;
        rc = run_row(pl, r, fp64, FFTGAL_K_RHS);
        if (rc) return rc;
        rc = forward_passes(pl, fp64, kind, rows, pl->ws + pl->so(pl->Lo.r), nullptr, -1.0 / npts, nullptr,
                            pl->at<double>(pl->so(pl->Lo.part_a)), &nrr, FFTGAL_K_RHS, FFTGAL_K_RHS, s, s > 0);
        if (rc) return rc;
    }
    nload *= D.nshift;
    // FP32 iterations keep b for the exact energies of the checkpoints
    if (!fp64) HIPCHECK(pl, launch_copy_vec(pl->ws + pl->so(pl->Lo.bvec), pl->ws + pl->so(pl->Lo.r), vbytes, pl->stream));
    // The load sums |A_M E|^2 over grid points; (., .)_{R^{d x M}} divides by |M|.
    const double floor_rel = (fp64 ? kFloor64 : kFloor32) / std::sqrt(npts);
    if (!pl->warm[kind][alpha]) {
        Timed t(pl, FFTGAL_K_CG_SCALAR);
        HIPCHECK(pl, launch_cg_init(st, pl->at<double>(pl->so(pl->Lo.part_a)), nrr, pl->at<double>(pl->so(pl->Lo.part_b)), nload,
                                    pl->at<double>(pl->so(pl->Lo.part_c)), 1.0 / npts, rtol, floor_rel, maxit, pl->btol,
                                    pl->hist(kind, alpha), pl->stream));
        HIPCHECK(pl, launch_fill_zero(x, vbytes, pl->stream));
        HIPCHECK(pl, launch_fill_zero(pl->ws + pl->so(pl->Lo.p), vbytes, pl->stream));
        if (!fp64) HIPCHECK(pl, launch_fill_zero(pl->ws + pl->so(pl->Lo.xbest), vbytes, pl->stream));
        return FFTGAL_OK;
    }
    // Warm start from the iterate x0 already in x: keep (b, b), |A_M E|^2 and
    // (A_M E).E as scalars, apply the operator to x0, then r_0 = b - K x0.
    pl->warm[kind][alpha] = false;
    if (pl->reduced) return fail(pl, FFTGAL_EINVAL, "warm starts are not supported by reduced plans");
    double *scal = pl->at<double>(pl->Lo.gram) + 32;
    {
        Timed t(pl, FFTGAL_K_CG_SCALAR);
        HIPCHECK(pl, launch_sum_partials(scal, pl->at<double>(pl->so(pl->Lo.part_a)), nrr, 1, pl->stream));
        HIPCHECK(pl, launch_sum_partials(scal + 1, pl->at<double>(pl->so(pl->Lo.part_b)), nload, 1, pl->stream));
        HIPCHECK(pl, launch_sum_partials(scal + 2, pl->at<double>(pl->so(pl->Lo.part_c)), nload, 1, pl->stream));
    }
    void *rows0 = nullptr;
    rc = inverse_passes(pl, fp64, kind, x, 0, 1, false, nullptr, &rows0, FFTGAL_K_RHS, FFTGAL_K_RHS);
    if (rc) return rc;
    RowArgs ro = base_row(pl, fp64, ROW_OPER, rows0, kind);
    rc = run_row(pl, ro, fp64, FFTGAL_K_RHS);
    if (rc) return rc;
    int nq = 0;
    rc = forward_passes(pl, fp64, kind, rows0, pl->ws + pl->so(pl->Lo.q), nullptr, 1.0 / (double)D.Mtot, nullptr,
                        pl->at<double>(pl->so(pl->Lo.part_a)), &nq, FFTGAL_K_RHS, FFTGAL_K_RHS);
    if (rc) return rc;
    UpdArgs u{};
    u.x = x;
    u.r = pl->ws + pl->so(pl->Lo.r);
    u.p = nullptr;
    u.q = pl->ws + pl->so(pl->Lo.q);
    u.n_per_comp = D.Ns;
    u.cs = D.Ns;
    u.nc = pl->nc(kind);
    u.Nh = D.Nh;
    u.nblocks = update_blocks((long)u.nc * D.Ns);
    Timed t(pl, FFTGAL_K_CG_SCALAR);
    HIPCHECK(pl, launch_warm_residual(u, pl->at<double>(pl->so(pl->Lo.part_a)), pl->at<double>(pl->so(pl->Lo.part_b)),
                                      pl->at<double>(pl->so(pl->Lo.part_c)), fp64, pl->stream));
    HIPCHECK(pl, launch_cg_init_warm(st, pl->at<double>(pl->so(pl->Lo.part_a)), pl->at<double>(pl->so(pl->Lo.part_b)),
                                     pl->at<double>(pl->so(pl->Lo.part_c)), u.nblocks, scal, (double)D.Mtot, rtol, floor_rel,
                                     maxit, pl->btol, pl->hist(kind, alpha), pl->stream));
    HIPCHECK(pl, launch_fill_zero(pl->ws + pl->so(pl->Lo.p), vbytes, pl->stream));
    if (!fp64) HIPCHECK(pl, launch_copy_vec(pl->ws + pl->so(pl->Lo.xbest), x, vbytes, pl->stream));
    return FFTGAL_OK;
}

int finish_solve(Plan *pl, int kind, int alpha, const CgStatus &h, fftgal_info *info) {
    fftgal_info inf{};
    inf.iters = h.iter;
    inf.converged = h.converged;
    inf.res0 = std::sqrt(std::max(0.0, h.rr0));
    inf.rel_res = h.rr0 > 0 ? std::sqrt(std::max(0.0, h.rr) / h.rr0) : 0.0;
    inf.stagnated = h.stagnated;
    inf.iterate = h.ck_restore ? h.best_it : h.iter;
    pl->last_info[kind][alpha] = inf;
    if (info) *info = inf;
    pl->solved[kind][alpha] = true;
    if (h.breakdown) return fail(pl, FFTGAL_EBREAKDOWN, "CG breakdown (non-SPD or non-finite material)");
    if (h.stagnated)
        return fail(pl, FFTGAL_ENOTCONV, "FP32 iterations stalled after %d iterations; the field of iteration %d "
                    "(lowest exact energy) is kept", h.iter, inf.iterate);
    if (!h.converged) return fail(pl, FFTGAL_ENOTCONV, "CG did not converge in %d iterations", h.maxit);
    return FFTGAL_OK;
}

// After an FP32 solve that stopped without converging (at maxit or on a stall
// not already handled by a checkpoint): keep the better of the last iterate
// and the kept copy, then read the status again.
int final_checkpoint(Plan *pl, int kind, int alpha, CgStatus *h) {
    if (pl->fp64_iter() || h->converged || h->breakdown || (h->stagnated && h->ck_restore)) return FFTGAL_OK;
    const int rc = checkpoint(pl, kind, alpha, true);
    if (rc) return rc;
    HIPCHECK(pl, hipMemcpyAsync(h, pl->status(kind, alpha), sizeof *h, hipMemcpyDeviceToHost, pl->stream));
    HIPCHECK(pl, hipStreamSynchronize(pl->stream));
    return FFTGAL_OK;
}

// Whether the CG iterations of this plan's solves run in the single
// work-group solver (2D Ga on a double grid it holds in LDS).
bool use_solo(const Plan *pl) {
    const Dims &D = pl->D;
    return pl->solo && D.d == 2 && !pl->gani && !pl->reduced && D.nshift == 1 && !pl->fM[0].blue &&
           !pl->fM[1].blue && solo_fits(D.M[0], D.M[1], pl->fp64_iter());
}

// Arguments of the single work-group solver for one solve (in the plan's
// current solve slot).
SoloArgs make_solo(Plan *pl, int kind, int alpha) {
    const Dims &D = pl->D;
    const bool fp64 = pl->fp64_iter();
    SoloArgs a{};
    a.x = pl->xsol(kind, alpha);
    a.r = pl->ws + pl->so(pl->Lo.r);
    a.p = pl->ws + pl->so(pl->Lo.p);
    a.st = pl->status(kind, alpha);
    a.mirror = nullptr;
    a.hist = pl->hist_on ? pl->hist(kind, alpha) : nullptr;
    a.hist_cap = kMaxHist + 1;
    const RowArgs r = base_row(pl, fp64, ROW_OPER, nullptr, kind, 0);
    a.g = r.g;
    a.gstride = r.gstride;
    a.nfield = r.nfield;
    for (int i = 0; i < 4; ++i) {
        a.A0[i] = r.A0[i];
        a.D[i] = r.D[i];
    }
    a.tw = pl->ws + (fp64 ? pl->Lo.tw64 : pl->Lo.tw32);
    a.tw0 = pl->fM[0].twoff[0];
    a.tw1 = pl->fM[1].twoff[0];
    a.M0 = D.M[0];
    a.M1 = D.M[1];
    a.N0 = D.N[0];
    a.Nh = D.Nh;
    a.kind = kind;
    a.scale = 1.0 / ((double)D.nshift * D.Mtot);
    return a;
}

// Iterations of a solve in the single work-group solver: one launch up to
// the next FP32 checkpoint (FP64: up to maxit; the kernel stops at
// convergence), then the status.
int run_solve_solo(Plan *pl, int kind, int alpha, int maxit, fftgal_info *info) {
    const bool fp64 = pl->fp64_iter();
    CgStatus *st = pl->status(kind, alpha);
    const SoloArgs sa = make_solo(pl, kind, alpha);
    static_assert(sizeof(SoloArgs) <= kArgSlot, "argument slot too small");
    std::memcpy(pl->iter_host[0], &sa, sizeof sa);
    HIPCHECK(pl, hipMemcpyAsync(pl->iter_slot(0), pl->iter_host[0], sizeof sa, hipMemcpyHostToDevice, pl->stream));
    const SoloArgs *dev = reinterpret_cast<const SoloArgs *>(pl->iter_slot(0));
    CgStatus h{};
    int enq = 0;
    int rc = FFTGAL_OK;
    for (;;) {
        const int n = fp64 ? maxit - enq : std::min(maxit - enq, kCkptEvery - enq % kCkptEvery);
        if (n > 0) {
            TimedLaunch t(pl, FFTGAL_K_SOLO);
            HIPCHECK(pl, launch_solo(sa, dev, 1, n, fp64, pl->stream, t.ev));
            enq += n;
            if (!fp64 && enq % kCkptEvery == 0 && (rc = checkpoint(pl, kind, alpha, false))) return rc;
        }
        HIPCHECK(pl, hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, pl->stream));
        HIPCHECK(pl, hipStreamSynchronize(pl->stream));
        if (h.done || enq >= maxit) break;
    }
    if ((rc = final_checkpoint(pl, kind, alpha, &h))) return rc;
    return finish_solve(pl, kind, alpha, h, info);
}

int run_solve(Plan *pl, int kind, int alpha, double rtol, int maxit, fftgal_info *info) {
    const bool fp64 = pl->fp64_iter();
    CgStatus *st = pl->status(kind, alpha);
    int rc = start_solve(pl, kind, alpha, rtol, maxit);
    if (rc) return rc;
    if (use_solo(pl)) return run_solve_solo(pl, kind, alpha, maxit, info);
    IterCfg cfg;
    rc = capture_iteration(pl, kind, alpha, fp64, &cfg);
    if (rc) return rc;
    rc = upload_iteration(pl, cfg);
    if (rc) return rc;
    // Iterations are enqueued in chunks without host synchronisation; after a
    // chunk the host reads the status and sizes the next chunk from the
    // observed per-iteration residual reduction, so that few no-op launches
    // (kernels return at once when `done` is set) follow convergence.
    CgStatus h{};
    int chunk = 8;
    int enq = 0;
    int it_prev = 0;
    double rr_prev = 0.0;
    bool first = true;
    for (;;) {
        const int todo = std::min(chunk, std::max(0, maxit - enq));
        for (int i = 0; i < todo; ++i) {
            rc = enqueue_iteration(pl, cfg);
            if (rc) return rc;
            ++enq;
            if (!fp64 && enq % kCkptEvery == 0 && (rc = checkpoint(pl, kind, alpha, false))) return rc;
        }
        HIPCHECK(pl, hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, pl->stream));
        HIPCHECK(pl, hipStreamSynchronize(pl->stream));
        if (h.done || enq >= maxit) break;
        const double target = std::max(h.tol2 * h.rr0, h.floor2);
        int next = 2 * chunk;
        // the rate since the previous read (at the first read: since the start,
        // from the initial residual); an iteration enqueued past convergence
        // costs its seven no-op launches, one too few a read of the status
        const int i0 = first ? 0 : it_prev;
        const double r0v = first ? h.rr0 : rr_prev;
        if (h.iter > i0 && h.rr < r0v && h.rr > 0.0 && target > 0.0) {
            const double rate = std::log(h.rr / r0v) / (h.iter - i0);  // < 0
            const double remain = std::log(target / h.rr) / rate;
            next = (int)std::ceil(remain) + 2;
        }
        first = false;
        chunk = std::max(2, std::min(next, 64));
        it_prev = h.iter;
        rr_prev = h.rr;
    }
    if ((rc = final_checkpoint(pl, kind, alpha, &h))) return rc;
    return finish_solve(pl, kind, alpha, h, info);
}

int solve_entry(Plan *pl, int kind, int alpha, double rtol, int maxit, fftgal_info *info) {
    if (!pl) return FFTGAL_EINVAL;
    if (!pl->have_mat) return fail(pl, FFTGAL_ESTATE, "no material set");
    if (pl->busy) return fail(pl, FFTGAL_ESTATE, "the plan has a solve in a batch");
    if (alpha < -1 || alpha >= pl->D.d) return fail(pl, FFTGAL_EINVAL, "alpha %d out of range", alpha);
    if (!(rtol >= 0.0) || maxit < 0) return fail(pl, FFTGAL_EINVAL, "rtol must be >= 0 and maxit >= 0");
    int worst = FFTGAL_OK;
    const int a0 = alpha < 0 ? 0 : alpha;
    const int a1 = alpha < 0 ? pl->D.d : alpha + 1;
    for (int a = a0; a < a1; ++a) {
        const int rc = run_solve(pl, kind, a, rtol, maxit, info ? info + (a - a0) : nullptr);
        if (rc == FFTGAL_EDEVICE || rc == FFTGAL_EINVAL) return rc;
        if (rc != FFTGAL_OK && worst == FFTGAL_OK) worst = rc;
    }
    return worst;
}

// Validate an inclusion description (eq. inclcomp: SPD phases, boxes with
// sides in (0, 1], discs of radius in (0, 1/2] in 2D, no overlaps under the
// periodic minimum image) and build its device table.
int parse_inclusions(Plan *pl, const fftgal_material *m, int d, std::vector<InclDev> *out) {
    if (!chol_spd(m->A0, d)) return fail(pl, FFTGAL_EINVAL, "A0 is not symmetric positive definite");
    const int n = m->n_incl;
    if (n < 0 || n > 100000) return fail(pl, FFTGAL_EINVAL, "n_incl out of range");
    if (n > 0 && (!m->shape || !m->center || !m->size || !m->A_in))
        return fail(pl, FFTGAL_EINVAL, "inclusion arrays must not be NULL");
    std::vector<InclDev> &inc = *out;
    inc.assign(n, InclDev{});
    for (int i = 0; i < n; ++i) {
        const int s = m->shape[i];
        if (s != FFTGAL_RECT && s != FFTGAL_CIRC) return fail(pl, FFTGAL_EINVAL, "inclusion %d: bad shape", i);
        if (s == FFTGAL_CIRC && d != 2) return fail(pl, FFTGAL_EINVAL, "inclusion %d: CIRC needs d = 2", i);
        inc[i].shape = s;
        for (int a = 0; a < 3; ++a) {
            inc[i].c[a] = a < d ? m->center[i * d + a] : 0.0;
            inc[i].h[a] = a < d ? m->size[i * d + a] : 0.0;
        }
        for (int a = 0; a < d; ++a)
            if (!std::isfinite(inc[i].c[a])) return fail(pl, FFTGAL_EINVAL, "inclusion %d: bad centre", i);
        if (s == FFTGAL_RECT) {
            for (int a = 0; a < d; ++a)
                if (!(inc[i].h[a] > 0.0 && inc[i].h[a] <= 1.0))
                    return fail(pl, FFTGAL_EINVAL, "inclusion %d: side must be in (0, 1]", i);
        } else if (!(inc[i].h[0] > 0.0 && inc[i].h[0] <= 0.5)) {
            return fail(pl, FFTGAL_EINVAL, "inclusion %d: radius must be in (0, 1/2]", i);
        }
        if (!chol_spd(m->A_in + (size_t)i * d * d, d))
            return fail(pl, FFTGAL_EINVAL, "inclusion %d: A_in is not symmetric positive definite", i);
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (overlap(d, inc[i].shape, inc[i].c, inc[i].h, inc[j].shape, inc[j].c, inc[j].h))
                return fail(pl, FFTGAL_EINVAL, "inclusions %d and %d overlap", i, j);
    return FFTGAL_OK;
}

// Extreme eigenvalues of a symmetric d x d matrix (cyclic Jacobi rotations in
// long double; d <= 3).
void sym_extremes(const double *A, int d, double *hi, double *lo) {
    long double a[3][3];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) a[i][j] = 0.5L * ((long double)A[i * d + j] + (long double)A[j * d + i]);
    for (int sweep = 0; sweep < 60; ++sweep) {
        long double off = 0.0L;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) off += a[p][q] * a[p][q];
        if (off == 0.0L) break;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                if (a[p][q] == 0.0L) continue;
                const long double th = (a[q][q] - a[p][p]) / (2.0L * a[p][q]);
                const long double t = (th >= 0 ? 1.0L : -1.0L) / (fabsl(th) + sqrtl(th * th + 1.0L));
                const long double c = 1.0L / sqrtl(t * t + 1.0L), sn = t * c;
                for (int k = 0; k < d; ++k) {  // columns p, q
                    const long double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - sn * akq;
                    a[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {  // rows p, q
                    const long double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - sn * aqk;
                    a[q][k] = sn * apk + c * aqk;
                }
            }
    }
    long double h = a[0][0], l = a[0][0];
    for (int i = 1; i < d; ++i) {
        h = std::max(h, a[i][i]);
        l = std::min(l, a[i][i]);
    }
    *hi = (double)h;
    *lo = (double)l;
}

}  // namespace

namespace {

// Device workspace of the internal batch that runs all 2d solves of a plan
// made with FFTGAL_CONCURRENT at once.
size_t bws_bytes(int d) { return align256(fftgal_batch_workspace_bytes(2 * d)); }

// Field f of the general material (entries 11, 12, [13,] 22, [23,] 33).
void field_entry(int f, int d, int *a, int *b) {
    int k = 0;
    for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) {
            if (k == f) {
                *a = i;
                *b = j;
                return;
            }
            ++k;
        }
}

// Inclusion composite with phases that need the general fields (eq.
// inclcomp_formula per matrix entry): for each side (A, then A^{-1}, whose
// inclusion values are the inverses of the phases because inclusions do not
// overlap) and each entry (a, b), the series w0 delta_k0 + sum_i w_i chi_i(k)
// with w0 = the matrix phase's entry and w_i = the entry of phase i minus it,
// transformed to the M-grid (eq. MBA_GA).
int general_inclusions(Plan *pl, const fftgal_material *m, std::vector<InclDev> &inc, InclDev *inc_dev) {
    const Dims &D = pl->D;
    const int d = D.d, n = (int)inc.size();
    double A0inv[9];
    if (!inv_small(m->A0, d, A0inv)) return fail(pl, FFTGAL_EINVAL, "A0 is singular");
    std::vector<double> inv_in((size_t)n * d * d);
    for (int i = 0; i < n; ++i)
        if (!inv_small(m->A_in + (size_t)i * d * d, d, &inv_in[(size_t)i * d * d]))
            return fail(pl, FFTGAL_EINVAL, "inclusion %d: A_in is singular", i);
    void *U = pl->ws + pl->so(pl->Lo.T2);
    for (int pass = 0; pass < 2; ++pass) {
        const double *base = pass == 0 ? m->A0 : A0inv;
        const double *ph = pass == 0 ? m->A_in : inv_in.data();
        double *field = pl->at<double>(pass == 0 ? pl->Lo.gA64 : pl->Lo.gB64);
        for (int f = 0; f < D.nfield; ++f) {
            int a, b;
            field_entry(f, d, &a, &b);
            for (int i = 0; i < n; ++i) inc[i].w = ph[(size_t)i * d * d + a * d + b] - base[a * d + b];
            if (n > 0)
                HIPCHECK(pl, hipMemcpyAsync(inc_dev, inc.data(), (size_t)n * sizeof(InclDev), hipMemcpyHostToDevice,
                                            pl->stream));
            {
                Timed t(pl, FFTGAL_K_SETUP);
                HIPCHECK(pl, launch_incl_coeff(U, d, D.L[0], D.L[1], D.Lh, inc_dev, n, base[a * d + b], pl->stream));
            }
            const int rc = series_to_field(pl, U, field + (size_t)f * D.Mtot);
            if (rc) return rc;
            HIPCHECK(pl, hipStreamSynchronize(pl->stream));  // host table reused
        }
    }
    pl->gen = true;
    pl->separate_gB = true;
    return FFTGAL_OK;
}

// Matrix voxel image (eq. gridcomp with C^p in R^{d x d}, Lemma grid_compos
// per entry): validation, then for each side (the image; the voxel-wise
// inverse of image_dual or of the image) and entry (a, b) the scalar image of
// that entry through the voxel series (sinc window) to the M-grid field.  A
// host image passes through the W scratch region in chunks.
int tensor_voxels(Plan *pl, const fftgal_material *m, long Ptot, size_t wbytes) {
    const Dims &D = pl->D;
    const int d = D.d;
    const size_t vb = (size_t)d * d * 8;  // bytes per voxel matrix
    double *staging = pl->at<double>(pl->vox_u);
    double *chunkbuf = pl->at<double>(pl->vox_w);
    const long cap = (long)(wbytes / vb);
    if (!m->image_device && cap < 1) return fail(pl, FFTGAL_ENOMEM, "no scratch for the matrix image");
    // run `body(device_matrices, first_voxel, count)` over the image, chunked for host images
    auto over = [&](const double *img, auto body) -> int {
        if (m->image_device) return body(img, 0L, Ptot);
        for (long v0 = 0; v0 < Ptot; v0 += cap) {
            const long cnt = std::min(cap, Ptot - v0);
            HIPCHECK(pl, hipMemcpyAsync(chunkbuf, img + (size_t)v0 * d * d, (size_t)cnt * vb, hipMemcpyHostToDevice,
                                        pl->stream));
            const int rc = body(chunkbuf, v0, cnt);
            if (rc) return rc;
            HIPCHECK(pl, hipStreamSynchronize(pl->stream));  // the chunk buffer is reused
        }
        return FFTGAL_OK;
    };
    const bool dual = m->image_dual != nullptr;
    for (int which = 0; which < (dual ? 2 : 1); ++which) {
        const double *img = which == 1 ? m->image_dual : m->image;
        double bad = 0.0;
        int rc = over(img, [&](const double *src, long, long cnt) -> int {
            int np = 0;
            HIPCHECK(pl, launch_tensor_check(src, cnt, d, pl->at<double>(pl->so(pl->Lo.part_a)), &np, pl->stream));
            HIPCHECK(pl, launch_sum_partials(pl->at<double>(pl->Lo.gram), pl->at<double>(pl->so(pl->Lo.part_a)), np, 1,
                                             pl->stream));
            double c = 0.0;
            HIPCHECK(pl, hipMemcpyAsync(&c, pl->at<double>(pl->Lo.gram), 8, hipMemcpyDeviceToHost, pl->stream));
            HIPCHECK(pl, hipStreamSynchronize(pl->stream));
            bad += c;
            return FFTGAL_OK;
        });
        if (rc) return rc;
        if (bad != 0.0)
            return fail(pl, FFTGAL_EINVAL, "%.0f voxels %sare not finite symmetric positive definite matrices", bad,
                        which == 1 ? "of the dual image " : "");
    }
    for (int pass = 0; pass < 2; ++pass) {
        const double *img = (pass == 1 && dual) ? m->image_dual : m->image;
        double *field = pl->at<double>(pass == 0 ? pl->Lo.gA64 : pl->Lo.gB64);
        for (int f = 0; f < D.nfield; ++f) {
            int a, b;
            field_entry(f, d, &a, &b);
            int rc = over(img, [&](const double *src, long v0, long cnt) -> int {
                Timed t(pl, FFTGAL_K_SETUP);
                HIPCHECK(pl, launch_tensor_component(src, cnt, d, a, b, pass, staging + v0, pl->stream));
                return FFTGAL_OK;
            });
            if (rc) return rc;
            void *coef = nullptr;
            if ((rc = voxel_series(pl, staging, 0, 0.0, &coef))) return rc;
            if ((rc = series_to_field(pl, coef, field + (size_t)f * D.Mtot))) return rc;
        }
    }
    pl->gen = true;
    pl->separate_gB = true;
    return FFTGAL_OK;
}

// Inclusion composite whose phases have the form A0 + g(x) D with one scalar
// field per side: all phases equal (two-phase, any SPD matrices; g is the
// indicator of the inclusions), or every phase isotropic (g is the conductivity
// itself, and 1/conductivity for the dual).
int scalar_inclusions(Plan *pl, const fftgal_material *m, std::vector<InclDev> &inc, bool same) {
    const Dims &D = pl->D;
    const int d = D.d, n = (int)inc.size();
    double *gA = pl->at<double>(pl->Lo.gA64);
    double *gB = pl->at<double>(pl->Lo.gB64);
    int rc = FFTGAL_OK;
    double A0inv[9];
    inv_small(m->A0, d, A0inv);
    double wA0 = 0.0, wB0 = 0.0;
    std::vector<double> wA(n), wB(n);
    if (same) {
        pl->separate_gB = false;
        std::memset(pl->DA, 0, sizeof pl->DA);
        std::memset(pl->DB, 0, sizeof pl->DB);
        for (int k = 0; k < d * d; ++k) {
            pl->A0[k] = m->A0[k];
            pl->B0[k] = A0inv[k];
        }
        if (n > 0) {
            double Ainv[9];
            inv_small(m->A_in, d, Ainv);
            for (int k = 0; k < d * d; ++k) {
                pl->DA[k] = m->A_in[k] - m->A0[k];
                pl->DB[k] = Ainv[k] - A0inv[k];
            }
        }
        for (int i = 0; i < n; ++i) wA[i] = wB[i] = 1.0;
    } else {
        double a0;
        if (!is_iso(m->A0, d, &a0))
            return fail(pl, FFTGAL_EINVAL, "different inclusion phases need isotropic A0 and A_in");
        pl->separate_gB = true;
        wA0 = a0;
        wB0 = 1.0 / a0;
        for (int i = 0; i < n; ++i) {
            double ai;
            if (!is_iso(m->A_in + (size_t)i * d * d, d, &ai))
                return fail(pl, FFTGAL_EINVAL, "different inclusion phases need isotropic A0 and A_in");
            wA[i] = ai - a0;
            wB[i] = 1.0 / ai - 1.0 / a0;
        }
        for (int k = 0; k < 9; ++k) pl->A0[k] = pl->B0[k] = pl->DA[k] = pl->DB[k] = 0.0;
        for (int a = 0; a < d; ++a) pl->DA[a * d + a] = pl->DB[a * d + a] = 1.0;
    }
    // device inclusion table lives at the end of the W scratch region
    void *U = pl->ws + pl->so(pl->Lo.T2);
    const size_t inc_bytes = (size_t)std::max(n, 1) * sizeof(InclDev);
    const size_t t1_bytes = pl->so(pl->Lo.T2) - pl->so(pl->Lo.T1);
    if (inc_bytes + 4096 > t1_bytes / 2) return fail(pl, FFTGAL_EINVAL, "too many inclusions for this plan");
    InclDev *inc_dev = reinterpret_cast<InclDev *>(pl->ws + pl->so(pl->Lo.T1) + (t1_bytes - inc_bytes - 256) / 256 * 256);
    for (int pass = 0; pass < (pl->separate_gB ? 2 : 1); ++pass) {
        for (int i = 0; i < n; ++i) inc[i].w = pass == 0 ? wA[i] : wB[i];
        HIPCHECK(pl, hipMemcpyAsync(inc_dev, inc.data(), (size_t)n * sizeof(InclDev), hipMemcpyHostToDevice,
                                    pl->stream));
        if (pl->gani) {
            // Def. GaNi: the material at the grid points, not a Fourier series
            Timed t(pl, FFTGAL_K_SETUP);
            HIPCHECK(pl, launch_sample_incl(pass == 0 ? gA : gB, d, D.M, inc_dev, n, pass == 0 ? wA0 : wB0,
                                            pl->stream));
        } else {
            {
                Timed t(pl, FFTGAL_K_SETUP);
                HIPCHECK(pl, launch_incl_coeff(U, d, D.L[0], D.L[1], D.Lh, inc_dev, n, pass == 0 ? wA0 : wB0,
                                               pl->stream));
            }
            rc = pl->reduced ? series_to_shifted_fields(pl, U, pass == 0 ? gA : gB)
                             : series_to_field(pl, U, pass == 0 ? gA : gB);
            if (rc) return rc;
        }
        HIPCHECK(pl, hipStreamSynchronize(pl->stream));  // host table reused
    }
    return FFTGAL_OK;
}

size_t workspace_bytes(int d, const int32_t *N, int precision, const int32_t *P, int scheme) {
    Dims D;
    const bool lean = (precision & FFTGAL_REDUCED_LEAN) != 0;
    const bool tensor = (precision & FFTGAL_TENSOR) != 0;
    const bool conc = (precision & FFTGAL_CONCURRENT) != 0;
    const bool fastg = (precision & FFTGAL_FAST_GRID) != 0;
    precision &= ~(FFTGAL_REDUCED_LEAN | FFTGAL_TENSOR | FFTGAL_CONCURRENT | FFTGAL_SEPARATE_PASSES |
                   FFTGAL_FAST_GRID);
    if (precision != FFTGAL_FP64 && precision != FFTGAL_FP32_ITER) return 0;
    if (lean && scheme != kSchemeReduced) return 0;
    if (tensor && scheme != kSchemeGa) return 0;
    if (conc && scheme == kSchemeReduced) return 0;
    if (fastg && scheme != kSchemeGa) return 0;
    if (!make_dims(d, N, nullptr, &D, scheme, tensor, fastg)) return 0;
    const size_t base = make_layout(D, precision, !lean, conc ? 2 * d : 1).total + (conc ? bws_bytes(d) : 0);
    if (P == nullptr) return base;
    Dims DP;
    if (!make_dims(d, N, P, &DP, scheme, tensor, fastg)) return 0;
    // a plan lays out its regions without P: an image that does not fit them
    // uses a tail of twiddles, U and W regions after the layout
    int Pv[3] = {1, 1, 1};
    size_t entry = 0;
    for (int a = 0; a < d; ++a) {
        Pv[a] = P[a];
        entry += fft_table_len(P[a]);
    }
    size_t need_u = 0, need_w = 0;
    voxel_scratch(D, Pv, &need_u, &need_w);
    return base + align256(entry * 16) + align256(entry * 8) + align256(need_u) + align256(need_w);
}

int make_plan(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *dev_workspace, size_t bytes,
              void *hip_stream, int scheme) {
    if (out == nullptr) return fail(nullptr, FFTGAL_EINVAL, "out is NULL");
    *out = nullptr;
    Dims D;
    const bool lean = (precision & FFTGAL_REDUCED_LEAN) != 0;
    const bool tensor = (precision & FFTGAL_TENSOR) != 0;
    const bool conc = (precision & FFTGAL_CONCURRENT) != 0;
    const bool sep = (precision & FFTGAL_SEPARATE_PASSES) != 0;
    const bool fastg = (precision & FFTGAL_FAST_GRID) != 0;
    precision &= ~(FFTGAL_REDUCED_LEAN | FFTGAL_TENSOR | FFTGAL_CONCURRENT | FFTGAL_SEPARATE_PASSES |
                   FFTGAL_FAST_GRID);
    if (precision != FFTGAL_FP64 && precision != FFTGAL_FP32_ITER)
        return fail(nullptr, FFTGAL_EINVAL, "unknown precision %d", precision);
    if (fastg && scheme != kSchemeGa)
        return fail(nullptr, FFTGAL_EINVAL, "FFTGAL_FAST_GRID applies to Ga plans only");
    if (lean && scheme != kSchemeReduced)
        return fail(nullptr, FFTGAL_EINVAL, "FFTGAL_REDUCED_LEAN applies to reduced plans only");
    if (tensor && scheme != kSchemeGa)
        return fail(nullptr, FFTGAL_EINVAL, "FFTGAL_TENSOR applies to Ga plans only");
    if (conc && scheme == kSchemeReduced)
        return fail(nullptr, FFTGAL_EINVAL, "FFTGAL_CONCURRENT applies to Ga and GaNi plans");
    if (!make_dims(d, N, nullptr, &D, scheme, tensor, fastg))
        return fail(nullptr, FFTGAL_EINVAL,
                    "d must be 2 or 3 and every N odd and >= 1");
    if (dev_workspace == nullptr || (reinterpret_cast<uintptr_t>(dev_workspace) & 255u))
        return fail(nullptr, FFTGAL_EINVAL, "workspace must be a 256-byte aligned device pointer");
    Layout Lo = make_layout(D, precision, !lean, conc ? 2 * d : 1);
    const size_t bws = conc ? bws_bytes(d) : 0;  // the internal batch of fftgal_solve_all
    if (bytes < Lo.total + bws)
        return fail(nullptr, FFTGAL_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, Lo.total + bws);
    // a larger workspace provisions voxel images up to the largest P that fits
    auto *pl = new Plan();
    pl->D = D;
    pl->Lo = Lo;
    pl->gani = scheme == kSchemeGani;
    pl->reduced = scheme == kSchemeReduced;
    pl->solo = !sep;
    pl->grouped = !lean && D.nshift > 1;
    pl->precision = precision;
    pl->slot_used.assign(Lo.nslots, 0);
    pl->bws_off = Lo.total;
    pl->bws_len = bws;
    pl->stream = reinterpret_cast<hipStream_t>(hip_stream);
    pl->ws = reinterpret_cast<char *>(dev_workspace);
    pl->ws_bytes = bytes;
    std::vector<double> tab;
    size_t entry = 0;
    for (int a = 0; a < d; ++a) {
        build_fft(D.M[a], entry, tab, &pl->fM[a]);
        entry = tab.size() / 2;
    }
    std::vector<float> tab32(tab.begin(), tab.end());
    hipError_t e = hipMemcpyAsync(pl->ws + Lo.tw64, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl->ws + Lo.tw32, tab32.data(), tab32.size() * 4, hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = launch_fill_zero(pl->ws + Lo.args, kArgsBytes, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) {
        delete pl;
        return fail(nullptr, FFTGAL_EDEVICE, "twiddle upload failed: %s", hipGetErrorString(e));
    }
    *out = pl;
    return FFTGAL_OK;
}

}  // namespace

// ---- the library's static workspace (fftgal_plan_static) -------------------
//
// A file-scope device array that every GPU the library runs on holds until
// the process ends.  Its name is a host-side stand-in in host code: the
// device address is taken once per device with hipGetSymbolAddress and only
// that address is used.  One plan at a time may hold a device's array.
constexpr size_t kStaticBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
struct StaticSlot {
    void *ptr = nullptr;           // device address of `scratch` on this device
    const Plan *owner = nullptr;   // the live plan holding it
};
std::mutex g_static_mu;
std::map<int, StaticSlot> g_static;
}  // namespace

extern "C" {


size_t fftgal_workspace_bytes_p(int d, const int32_t *N, int precision, const int32_t *P) {
    return workspace_bytes(d, N, precision, P, kSchemeGa);
}

size_t fftgal_workspace_bytes_gani(int d, const int32_t *N, int precision, const int32_t *P) {
    return workspace_bytes(d, N, precision, P, kSchemeGani);
}

size_t fftgal_workspace_bytes_reduced(int d, const int32_t *N, int precision, const int32_t *P) {
    return workspace_bytes(d, N, precision, P, kSchemeReduced);
}

size_t fftgal_workspace_bytes(int d, const int32_t *N, int precision) {
    return fftgal_workspace_bytes_p(d, N, precision, nullptr);
}

int fftgal_plan(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *dev_workspace, size_t bytes,
                void *hip_stream) {
    return make_plan(out, d, N, precision, dev_workspace, bytes, hip_stream, kSchemeGa);
}

int fftgal_plan_static(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *hip_stream) {
    if (out == nullptr) return fail(nullptr, FFTGAL_EINVAL, "out is NULL");
    *out = nullptr;
    const size_t need = fftgal_workspace_bytes(d, N, precision);
    if (need == 0) return fail(nullptr, FFTGAL_EINVAL, "d must be 2 or 3, every N odd and >= 1, precision known");
    if (need > kStaticBytes)
        return fail(nullptr, FFTGAL_ENOMEM, "the plan needs %zu bytes; the static workspace holds %zu", need,
                    kStaticBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, FFTGAL_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot &slot = g_static[dev];
    if (slot.owner != nullptr)
        return fail(nullptr, FFTGAL_ESTATE, "the static workspace of device %d is held by another plan", dev);
    if (slot.ptr == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(nullptr, FFTGAL_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        slot.ptr = p;
    }
    const int rc = make_plan(out, d, N, precision, slot.ptr, kStaticBytes, hip_stream, kSchemeGa);
    if (rc != FFTGAL_OK) return rc;
    (*out)->static_dev = dev;
    slot.owner = *out;
    return FFTGAL_OK;
}

size_t fftgal_static_workspace_bytes(void) { return kStaticBytes; }

int fftgal_plan_gani(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *dev_workspace,
                     size_t bytes, void *hip_stream) {
    return make_plan(out, d, N, precision, dev_workspace, bytes, hip_stream, kSchemeGani);
}

int fftgal_plan_reduced(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *dev_workspace,
                        size_t bytes, void *hip_stream) {
    return make_plan(out, d, N, precision, dev_workspace, bytes, hip_stream, kSchemeReduced);
}


int fftgal_set_material(struct fftgal_plan *pl, const fftgal_material *m) {
    if (!pl) return FFTGAL_EINVAL;
    if (!m) return fail(pl, FFTGAL_EINVAL, "material is NULL");
    if (pl->busy) return fail(pl, FFTGAL_ESTATE, "the plan has a solve in a batch");
    const Dims &D = pl->D;
    const int d = D.d;
    pl->have_mat = false;
    pl->gen = false;
    for (auto &row : pl->solved)
        for (bool &s : row) s = false;
    for (auto &row : pl->warm)
        for (bool &s : row) s = false;
    double *gA = pl->at<double>(pl->Lo.gA64);
    double *gB = pl->at<double>(pl->Lo.gB64);
    int rc = FFTGAL_OK;
    if (m->kind == FFTGAL_INCLUSIONS) {
        const int n = m->n_incl;
        std::vector<InclDev> inc;
        if ((rc = parse_inclusions(pl, m, d, &inc))) return rc;
        bool same = true;
        for (int i = 1; i < n && same; ++i)
            for (int k = 0; k < d * d; ++k)
                if (m->A_in[(size_t)i * d * d + k] != m->A_in[k]) same = false;
        bool all_iso = true;
        double tmp;
        all_iso = is_iso(m->A0, d, &tmp);
        for (int i = 0; i < n && all_iso; ++i) all_iso = is_iso(m->A_in + (size_t)i * d * d, d, &tmp);
        if (!same && !all_iso) {
            if (D.nfield < 2)
                return fail(pl, FFTGAL_EINVAL, "inclusion phases that differ and are not all isotropic need a plan "
                                               "made with FFTGAL_TENSOR");
            const size_t inc_bytes = (size_t)std::max(n, 1) * sizeof(InclDev);
            const size_t t1_bytes = pl->so(pl->Lo.T2) - pl->so(pl->Lo.T1);
            if (inc_bytes + 4096 > t1_bytes / 2) return fail(pl, FFTGAL_EINVAL, "too many inclusions for this plan");
            InclDev *inc_dev =
                reinterpret_cast<InclDev *>(pl->ws + pl->so(pl->Lo.T1) + (t1_bytes - inc_bytes - 256) / 256 * 256);
            if ((rc = general_inclusions(pl, m, inc, inc_dev))) return rc;
        } else {
            if ((rc = scalar_inclusions(pl, m, inc, same))) return rc;
        }
    } else if (m->kind == FFTGAL_VOXELS) {
        long Ptot = 1;
        for (int a = 0; a < d; ++a) {
            if (m->P[a] < 1 || m->P[a] % 2 == 0 || m->P[a] > 100000)
                return fail(pl, FFTGAL_EINVAL, "voxel resolution P[%d] = %d is not an odd integer", a, m->P[a]);
            Ptot *= m->P[a];
        }
        if (!m->image) return fail(pl, FFTGAL_EINVAL, "image is NULL");
        // the image, its R2C rows and the image twiddles must fit the scratch
        // regions of this plan, or else the workspace tail beyond its layout
        size_t need_u = 0, need_w = 0;
        voxel_scratch(D, m->P, &need_u, &need_w);
        std::vector<double> tab;
        size_t entry = 0;
        FftDesc fP[3];
        for (int a = 0; a < d; ++a) {
            build_fft(m->P[a], entry, tab, &fP[a]);
            entry = tab.size() / 2;
        }
        const size_t ubytes = pl->so(pl->Lo.r) - pl->so(pl->Lo.T2);
        const size_t wbytes = pl->so(pl->Lo.T2) - pl->so(pl->Lo.T1);
        if (need_u <= ubytes && need_w <= wbytes && entry <= pl->Lo.twP_len) {
            pl->vox_tw64 = pl->Lo.twP64;
            pl->vox_tw32 = pl->Lo.twP32;
            pl->vox_u = pl->so(pl->Lo.T2);
            pl->vox_w = pl->so(pl->Lo.T1);
        } else {
            const size_t t0 = pl->Lo.total;
            pl->vox_tw64 = t0;
            pl->vox_tw32 = pl->vox_tw64 + align256(entry * 16);
            pl->vox_u = pl->vox_tw32 + align256(entry * 8);
            pl->vox_w = pl->vox_u + align256(need_u);
            if (pl->vox_w + need_w > pl->ws_bytes)
                return fail(pl, FFTGAL_ENOMEM,
                            "voxel image too large for this workspace (size it with fftgal_workspace_bytes_p)");
        }
        for (int a = 0; a < d; ++a) {
            pl->Pcur[a] = m->P[a];
            pl->fP[a] = fP[a];
        }
        std::vector<float> tab32(tab.begin(), tab.end());
        HIPCHECK(pl, hipMemcpyAsync(pl->ws + pl->vox_tw64, tab.data(), tab.size() * 8, hipMemcpyHostToDevice,
                                    pl->stream));
        HIPCHECK(pl, hipMemcpyAsync(pl->ws + pl->vox_tw32, tab32.data(), tab32.size() * 4, hipMemcpyHostToDevice,
                                    pl->stream));
        if (m->image_tensor) {
            if (D.nfield < 2)
                return fail(pl, FFTGAL_EINVAL, "matrix voxel images need a plan made with FFTGAL_TENSOR");
            const size_t wb = pl->vox_w == pl->so(pl->Lo.T1) ? wbytes : need_w;
            if ((rc = tensor_voxels(pl, m, Ptot, wb))) return rc;
        } else {
        // the image is read from the caller's device buffer, or from a staging
        // copy at the start of the U scratch region (re-uploaded per pass,
        // since the transforms overwrite U)
        double *staging = pl->at<double>(pl->vox_u);
        // an optional dual image: the primal side uses `image`, the dual side
        // 1 / image_dual (Lemma bounds_bounds: upper and lower approximations)
        const bool dual = m->image_dual != nullptr;
        auto img_of = [&](int which) -> const double * {
            const double *src = (which == 1 && dual) ? m->image_dual : m->image;
            return m->image_device ? src : staging;
        };
        auto upload = [&](int which) -> int {
            if (!m->image_device) {
                const double *src = (which == 1 && dual) ? m->image_dual : m->image;
                HIPCHECK(pl, hipMemcpyAsync(staging, src, (size_t)Ptot * 8, hipMemcpyHostToDevice, pl->stream));
            }
            return FFTGAL_OK;
        };
        double stats[4];
        for (int which = dual ? 1 : 0; which >= 0; --which) {
            if ((rc = upload(which))) return rc;
            {
                Timed t(pl, FFTGAL_K_SETUP);
                HIPCHECK(pl, launch_image_stats(img_of(which), Ptot, pl->at<double>(pl->so(pl->Lo.part_a)),
                                                pl->at<double>(pl->Lo.gram), pl->stream));
            }
            HIPCHECK(pl, hipMemcpyAsync(stats, pl->at<double>(pl->Lo.gram), sizeof stats, hipMemcpyDeviceToHost,
                                        pl->stream));
            HIPCHECK(pl, hipStreamSynchronize(pl->stream));
            if (stats[2] != 0.0)
                return fail(pl, FFTGAL_EINVAL, "%.0f voxels %sare not positive finite conductivities", stats[2],
                            which == 1 ? "of the dual image " : "");
        }
        const double *img = img_of(0);
        const double vmin = stats[0], vmax = stats[1];
        const bool two = stats[3] == 0.0 && !dual;
        std::memset(pl->DA, 0, sizeof pl->DA);
        std::memset(pl->DB, 0, sizeof pl->DB);
        std::memset(pl->A0, 0, sizeof pl->A0);
        std::memset(pl->B0, 0, sizeof pl->B0);
        pl->separate_gB = !two;
        if (two) {
            for (int a = 0; a < d; ++a) {
                pl->A0[a * d + a] = vmin;
                pl->DA[a * d + a] = vmax - vmin;
                pl->B0[a * d + a] = 1.0 / vmin;
                pl->DB[a * d + a] = 1.0 / vmax - 1.0 / vmin;
            }
        } else {
            for (int a = 0; a < d; ++a) pl->DA[a * d + a] = pl->DB[a * d + a] = 1.0;
        }
        const int npass = two ? 1 : 2;
        for (int pass = 0; pass < npass; ++pass) {
            if (pass > 0 && (rc = upload(1))) return rc;
            if (pass > 0) img = img_of(1);
            const int map = two ? (vmax == vmin ? 3 : 1) : (pass == 0 ? 0 : 2);
            if (pl->gani) {
                Timed t(pl, FFTGAL_K_SETUP);
                HIPCHECK(pl, launch_sample_voxel(pass == 0 ? gA : gB, img, d, m->P, D.M, map, vmax, pl->stream));
                continue;
            }
            void *coef = nullptr;
            rc = voxel_series(pl, img, map, vmax, &coef);
            if (rc) return rc;
            rc = pl->reduced ? series_to_shifted_fields(pl, coef, pass == 0 ? gA : gB)
                             : series_to_field(pl, coef, pass == 0 ? gA : gB);
            if (rc) return rc;
        }
        }
    } else {
        return fail(pl, FFTGAL_EINVAL, "unknown material kind %d", m->kind);
    }
    if (!pl->fp64_iter()) {
        Timed t(pl, FFTGAL_K_SETUP);
        const size_t nv = (size_t)D.nshift * (pl->gen ? D.nfield : 1) * D.Mtot;
        HIPCHECK(pl, launch_convert_d2f(pl->at<float>(pl->Lo.gA32), gA, nv, pl->stream));
        if (pl->separate_gB) HIPCHECK(pl, launch_convert_d2f(pl->at<float>(pl->Lo.gB32), gB, nv, pl->stream));
    }
    HIPCHECK(pl, hipStreamSynchronize(pl->stream));
    pl->have_mat = true;
    return FFTGAL_OK;
}

int fftgal_solve_primal(struct fftgal_plan *pl, int alpha, double rtol, int maxit, fftgal_info *info) {
    return solve_entry(pl, KIND_E, alpha, rtol, maxit, info);
}

int fftgal_solve_dual(struct fftgal_plan *pl, int alpha, double rtol, int maxit, fftgal_info *info) {
    return solve_entry(pl, KIND_J, alpha, rtol, maxit, info);
}

int fftgal_bounds(struct fftgal_plan *pl, double *upper, double *lower, double *gap) {
    if (!pl) return FFTGAL_EINVAL;
    const Dims &D = pl->D;
    const int d = D.d;
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < d; ++a)
            if (!pl->solved[k][a]) return fail(pl, FFTGAL_ESTATE, "bounds need all %d primal and dual solves", d);
    double gram[2][9];
    for (int kind = 0; kind < 2; ++kind) {
        const int nc = pl->nc(kind);
        const void *xs = pl->xsol(kind, 0);
        long st_ss = (long)D.nc_max * D.Ns;
        if (!pl->fp64_iter()) {
            // FP64 copies of the FP32 iterates (component-wise exact)
            double *x64 = pl->at<double>(pl->Lo.xsol64);
            Timed t(pl, FFTGAL_K_BOUNDS);
            for (int a = 0; a < d; ++a)
                HIPCHECK(pl, launch_convert_f2d(x64 + (size_t)a * D.nc_max * D.Ns * 2,
                                                reinterpret_cast<const float *>(pl->xsol(kind, a)),
                                                (size_t)nc * D.Ns * 2, pl->stream));
            xs = x64;
        } else {
            st_ss = (long)(pl->vec_bytes() / 16);
        }
        // the energy quadrature on every shifted grid (reduced Ga: the
        // quadratic form of Lemma reduce_grid), the d^2 sums of shift s in
        // gram + 16 s, added on the host in shift order
        for (int i = 0; i < d * d; ++i) gram[kind][i] = 0.0;
        for (int s = 0; s < D.nshift; ++s) {
            void *rows = nullptr;
            int rc = inverse_passes(pl, true, kind, xs, st_ss, d, false, nullptr, &rows, FFTGAL_K_BOUNDS,
                                    FFTGAL_K_BOUNDS, s);
            if (rc) return rc;
            RowArgs r = base_row(pl, true, ROW_GRAM, rows, kind, s);
            r.ncomp = d * d;
            r.partial = pl->at<double>(pl->so(pl->Lo.part_b));
            rc = run_row(pl, r, true, FFTGAL_K_BOUNDS);
            if (rc) return rc;
            Timed t(pl, FFTGAL_K_BOUNDS);
            HIPCHECK(pl, launch_sum_partials(pl->at<double>(pl->Lo.gram), pl->at<double>(pl->so(pl->Lo.part_b)), row_grid(r),
                                             d * d, pl->stream));
            double gs[9];
            HIPCHECK(pl, hipMemcpyAsync(gs, pl->at<double>(pl->Lo.gram), d * d * 8, hipMemcpyDeviceToHost,
                                        pl->stream));
            HIPCHECK(pl, hipStreamSynchronize(pl->stream));
            for (int i = 0; i < d * d; ++i) gram[kind][i] += gs[i];
        }
        for (int i = 0; i < d * d; ++i) gram[kind][i] /= (double)D.nshift * D.Mtot;
    }
    double up[9], bh[9], lo[9];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            up[i * d + j] = 0.5 * (gram[0][i * d + j] + gram[0][j * d + i]);
            bh[i * d + j] = 0.5 * (gram[1][i * d + j] + gram[1][j * d + i]);
        }
    if (!inv_small(bh, d, lo)) return fail(pl, FFTGAL_EBREAKDOWN, "dual Gram matrix is singular");
    for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j) lo[i * d + j] = lo[j * d + i] = 0.5 * (lo[i * d + j] + lo[j * d + i]);
    if (upper) std::memcpy(upper, up, sizeof(double) * d * d);
    if (lower) std::memcpy(lower, lo, sizeof(double) * d * d);
    if (gap) {
        double g = 0;
        for (int i = 0; i < d; ++i) g += up[i * d + i] - lo[i * d + i];
        *gap = 0.5 * g;
    }
    return FFTGAL_OK;
}

int fftgal_set_timing(struct fftgal_plan *pl, int enable) {
    if (!pl) return FFTGAL_EINVAL;
    pl->timing_mask = enable != 0 ? (1u << FFTGAL_K_COUNT) - 1u : 0u;
    return FFTGAL_OK;
}

int fftgal_set_timing_classes(struct fftgal_plan *pl, uint32_t mask) {
    if (!pl) return FFTGAL_EINVAL;
    pl->timing_mask = mask & ((1u << FFTGAL_K_COUNT) - 1u);
    return FFTGAL_OK;
}

int fftgal_set_bound_tol(struct fftgal_plan *pl, double btol) {
    if (!pl) return FFTGAL_EINVAL;
    if (!(btol >= 0.0) || !std::isfinite(btol)) return fail(pl, FFTGAL_EINVAL, "bound tolerance must be >= 0");
    pl->btol = btol;
    return FFTGAL_OK;
}

int fftgal_read_timing(struct fftgal_plan *pl, double *ms, int32_t *count) {
    if (!pl) return FFTGAL_EINVAL;
    HIPCHECK(pl, hipStreamSynchronize(pl->stream));
    for (const auto &e : pl->evs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
            pl->t_ms[e.cls] += t;
            pl->t_cnt[e.cls] += 1;
        }
        pl->pool.push_back(e.a);
        pl->pool.push_back(e.b);
    }
    pl->evs.clear();
    for (int c = 0; c < FFTGAL_K_COUNT; ++c) {
        if (ms) ms[c] = pl->t_ms[c];
        if (count) count[c] = pl->t_cnt[c];
        pl->t_ms[c] = 0.0;
        pl->t_cnt[c] = 0;
    }
    return FFTGAL_OK;
}

int fftgal_warm_start(struct fftgal_plan *fine, struct fftgal_plan *coarse) {
    if (!fine) return FFTGAL_EINVAL;
    if (!coarse || coarse == fine) return fail(fine, FFTGAL_EINVAL, "coarse plan is NULL or the fine plan itself");
    if (!fine->have_mat) return fail(fine, FFTGAL_ESTATE, "no material set on the fine plan");
    if (fine->busy || coarse->busy) return fail(fine, FFTGAL_ESTATE, "a plan has a solve in a batch");
    if (fine->reduced) return fail(fine, FFTGAL_EINVAL, "warm starts are not supported by reduced plans");
    const int d = fine->D.d;
    if (coarse->D.d != d) return fail(fine, FFTGAL_EINVAL, "plans of different dimension");
    int n = 0;
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < d; ++a) n += coarse->solved[k][a] ? 1 : 0;
    if (n == 0) return fail(fine, FFTGAL_ESTATE, "the coarse plan has no finished solve");
    if (coarse->stream != fine->stream) HIPCHECK(fine, hipStreamSynchronize(coarse->stream));
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < d; ++a) {
            if (!coarse->solved[k][a]) continue;
            HIPCHECK(fine, launch_prolong(coarse->xsol(k, a), coarse->fp64_iter(), fine->xsol(k, a), fine->fp64_iter(),
                                          d, fine->nc(k), fine->D.N, coarse->D.N, fine->stream));
            fine->warm[k][a] = true;
        }
    return FFTGAL_OK;
}

int fftgal_envelope_images(struct fftgal_plan *pl, const fftgal_material *m, const int32_t *P, double *upper,
                           double *lower) {
    if (!pl) return FFTGAL_EINVAL;
    if (!m || !P || !upper || !lower) return fail(pl, FFTGAL_EINVAL, "NULL argument");
    if (m->kind != FFTGAL_INCLUSIONS) return fail(pl, FFTGAL_EINVAL, "envelopes are built from inclusions");
    if (pl->busy) return fail(pl, FFTGAL_ESTATE, "the plan has a solve in a batch");
    const int d = pl->D.d;
    for (int a = 0; a < d; ++a)
        if (P[a] < 1 || P[a] > 100000) return fail(pl, FFTGAL_EINVAL, "P[%d] out of range", a);
    std::vector<InclDev> inc;
    int rc = parse_inclusions(pl, m, d, &inc);
    if (rc) return rc;
    const int n = (int)inc.size();
    // table: inclusions, then the extreme eigenvalues of the matrix and of
    // every inclusion phase
    std::vector<double> ext(2 * (n + 1));
    sym_extremes(m->A0, d, &ext[0], &ext[1]);
    for (int i = 0; i < n; ++i) sym_extremes(m->A_in + (size_t)i * d * d, d, &ext[2 + 2 * i], &ext[3 + 2 * i]);
    const size_t inc_bytes = align256((size_t)std::max(n, 1) * sizeof(InclDev));
    if (inc_bytes + ext.size() * 8 > pl->so(pl->Lo.T2) - pl->so(pl->Lo.T1))
        return fail(pl, FFTGAL_ENOMEM, "too many inclusions for this plan's scratch");
    InclDev *inc_dev = reinterpret_cast<InclDev *>(pl->ws + pl->so(pl->Lo.T1));
    double *ext_dev = reinterpret_cast<double *>(pl->ws + pl->so(pl->Lo.T1) + inc_bytes);
    if (n > 0)
        HIPCHECK(pl, hipMemcpyAsync(inc_dev, inc.data(), (size_t)n * sizeof(InclDev), hipMemcpyHostToDevice,
                                    pl->stream));
    HIPCHECK(pl, hipMemcpyAsync(ext_dev, ext.data(), ext.size() * 8, hipMemcpyHostToDevice, pl->stream));
    {
        Timed t(pl, FFTGAL_K_SETUP);
        HIPCHECK(pl, launch_envelope(upper, lower, d, P, inc_dev, n, ext_dev, pl->stream));
    }
    HIPCHECK(pl, hipStreamSynchronize(pl->stream));  // host tables
    return FFTGAL_OK;
}

int fftgal_bounds_of(struct fftgal_plan *pl, struct fftgal_plan *src, double *upper, double *lower, double *gap) {
    if (!pl) return FFTGAL_EINVAL;
    if (!src || src == pl) return fail(pl, FFTGAL_EINVAL, "source plan is NULL or the plan itself");
    if (!pl->have_mat) return fail(pl, FFTGAL_ESTATE, "no material set");
    if (pl->busy || src->busy) return fail(pl, FFTGAL_ESTATE, "a plan has a solve in a batch");
    if (pl->reduced || src->reduced) return fail(pl, FFTGAL_EINVAL, "a-posteriori bounds take Ga and GaNi plans");
    const int d = pl->D.d;
    if (src->D.d != d) return fail(pl, FFTGAL_EINVAL, "plans of different dimension");
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < d; ++a)
            if (!src->solved[k][a])
                return fail(pl, FFTGAL_ESTATE, "the source plan needs all %d primal and dual solves", d);
    if (src->stream != pl->stream) HIPCHECK(pl, hipStreamSynchronize(src->stream));
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < d; ++a) {
            HIPCHECK(pl, launch_prolong(src->xsol(k, a), src->fp64_iter(), pl->xsol(k, a), pl->fp64_iter(), d,
                                        pl->nc(k), pl->D.N, src->D.N, pl->stream));
            pl->solved[k][a] = true;
            pl->warm[k][a] = false;
            pl->hist_valid[k][a] = false;
            pl->last_info[k][a] = src->last_info[k][a];
        }
    return fftgal_bounds(pl, upper, lower, gap);
}

int fftgal_history(struct fftgal_plan *pl, int kind, int alpha, double *energy, int cap, int *n) {
    if (!pl) return FFTGAL_EINVAL;
    if (kind < 0 || kind > 1 || alpha < 0 || alpha >= pl->D.d || cap < 0 || (cap > 0 && !energy) || !n)
        return fail(pl, FFTGAL_EINVAL, "bad kind, alpha or output arrays");
    if (!pl->solved[kind][alpha] || !pl->hist_valid[kind][alpha])
        return fail(pl, FFTGAL_ESTATE, "no recorded solve (maxit must be <= %d)", kMaxHist);
    const int iters = pl->last_info[kind][alpha].iters;
    std::vector<double> h((size_t)2 * (iters + 1));
    HIPCHECK(pl, hipMemcpyAsync(h.data(), pl->hist(kind, alpha), h.size() * 8, hipMemcpyDeviceToHost, pl->stream));
    HIPCHECK(pl, hipStreamSynchronize(pl->stream));
    // energy_k = energy_{k-1} - alpha_k (r_{k-1}, r_{k-1})  (CG on a quadratic
    // functional: phi(e_k) = phi(e_{k-1}) - alpha_k |r_{k-1}|^2 / 2)
    double e = h[1];
    *n = iters + 1;
    for (int k = 0; k <= iters; ++k) {
        if (k > 0) e -= h[2 * k + 1] * h[2 * (k - 1)];
        if (k < cap) energy[k] = e;
    }
    return FFTGAL_OK;
}

int fftgal_destroy(struct fftgal_plan *pl) {
    if (!pl) return FFTGAL_OK;
    if (pl->busy) return fail(pl, FFTGAL_ESTATE, "the plan has a solve in a batch");
    if (!pl->evs.empty()) (void)hipStreamSynchronize(pl->stream);
    for (const auto &e : pl->evs) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (hipEvent_t e : pl->pool) (void)hipEventDestroy(e);
    if (pl->static_dev >= 0) {
        // the static workspace is free for the next plan once this plan's work is done
        (void)hipStreamSynchronize(pl->stream);
        std::lock_guard<std::mutex> lock(g_static_mu);
        StaticSlot &slot = g_static[pl->static_dev];
        if (slot.owner == pl) slot.owner = nullptr;
    }
    delete pl;
    return FFTGAL_OK;
}

const char *fftgal_last_error(const struct fftgal_plan *pl) {
    return pl ? pl->err.c_str() : g_plan_error.c_str();
}

int fftgal_grid_size(const struct fftgal_plan *pl, int axis) {
    if (!pl || axis < 0 || axis >= pl->D.d) return 0;
    return pl->D.M[axis];
}

}  // extern "C"

// ---- batched CG ------------------------------------------------------------

struct fftgal_batch {
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t bytes = 0;
    int cap = 0;
    struct Member {
        Plan *pl;
        int kind, alpha, id;
        IterCfg cfg;
        int enq = 0;  // iterations enqueued (FP32 checkpoints every kCkptEvery)
        int slot = 0;  // the plan's solve slot
        bool solo = false;  // iterations in the single work-group solver
        SoloArgs sargs{};
    };
    std::vector<Member> members;
    struct Done {
        int id;
        fftgal_info info;
        int status;
    };
    std::deque<Done> done;
    bool dirty = true;
    struct Group {
        size_t pass;
        int np, total;
        size_t args_off, woff_off;
        PassRec proto;
    };
    std::vector<Group> groups;
    struct UGroup {
        bool fp64;
        int np, total;
        size_t args_off, woff_off;
    };
    std::vector<UGroup> ugroups;
    // members in the single work-group solver, one launch per grid and precision
    struct SGroup {
        bool fp64;
        int np;
        size_t args_off;
        SoloArgs proto;
    };
    std::vector<SGroup> sgroups;
    int n_items = 0;  // members in the per-pass kernels (CG items)
    // the single work-group solves run on a stream of the batch's own, beside
    // the per-pass kernels of the other members
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t items_off = 0;
    size_t blob_base = 0;  // device offset of the argument blob
    std::vector<unsigned char> blob;
    std::vector<CgStatus> mirror_host;
    int next_id = 0;
    std::string err = "no error";
};
typedef struct fftgal_batch Batch;

namespace {

int bfail(Batch *b, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    return code;
}

#define BHIPCHECK(b, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return bfail(b, FFTGAL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t blob_put(std::vector<unsigned char> &blob, const void *p, size_t n) {
    const size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + n);
    std::memcpy(blob.data() + off, p, n);
    return off;
}

bool pass_fast(const PassRec &r) { return r.type == 0 ? r.pa.fast != 0 : r.ra.fast != 0; }

// Group the members' specialised passes by (pass index, kernel, length,
// dimension, precision, kernel variant) and lay out their argument tables, work-group
// offsets, CG update arguments and CG items in one blob; upload it.
int batch_rebuild(Batch *b) {
    b->blob.clear();
    b->groups.clear();
    b->ugroups.clear();
    const size_t nm = b->members.size();
    for (size_t i = 0; i < 5; ++i) {
        std::map<std::tuple<int, int, int, int>, std::vector<size_t>> by;
        for (size_t m = 0; m < nm; ++m) {
            const auto &ps = b->members[m].cfg.passes;
            if (b->members[m].solo || i >= ps.size() || !pass_fast(ps[i])) continue;
            const PassRec &r = ps[i];
            const int n = r.type == 0 ? r.pa.f.n : r.ra.f.n;
            const int d = r.type == 0 ? r.pa.d : r.ra.d;
            const int fm = r.type == 0 ? r.pa.fast : r.ra.fast;
            by[std::make_tuple(r.type, n, d, (int)r.fp64 * 4 + fm)].push_back(m);
        }
        for (auto &kv : by) {
            const auto &ms = kv.second;
            const PassRec &proto = b->members[ms[0]].cfg.passes[i];
            const size_t sz = proto.type == 0 ? sizeof(PencilArgs) : sizeof(RowArgs);
            std::vector<unsigned char> tab(sz * ms.size());
            std::vector<int> woff(ms.size());
            int total = 0;
            for (size_t j = 0; j < ms.size(); ++j) {
                const PassRec &r = b->members[ms[j]].cfg.passes[i];
                std::memcpy(tab.data() + j * sz, r.type == 0 ? (const void *)&r.pa : (const void *)&r.ra, sz);
                woff[j] = total;
                total += r.grid;
            }
            Batch::Group g;
            g.pass = i;
            g.np = (int)ms.size();
            g.total = total;
            g.proto = proto;
            g.args_off = blob_put(b->blob, tab.data(), tab.size());
            g.woff_off = blob_put(b->blob, woff.data(), woff.size() * sizeof(int));
            b->groups.push_back(g);
        }
    }
    for (int f = 0; f < 2; ++f) {
        std::vector<UpdArgs> ua;
        std::vector<int> woff;
        int total = 0;
        for (size_t m = 0; m < nm; ++m) {
            const IterCfg &c = b->members[m].cfg;
            if (b->members[m].solo || (int)c.fp64 != f) continue;
            ua.push_back(c.upd);
            woff.push_back(total);
            total += c.upd.nblocks;
        }
        if (ua.empty()) continue;
        Batch::UGroup u;
        u.fp64 = f == 1;
        u.np = (int)ua.size();
        u.total = total;
        u.args_off = blob_put(b->blob, ua.data(), ua.size() * sizeof(UpdArgs));
        u.woff_off = blob_put(b->blob, woff.data(), woff.size() * sizeof(int));
        b->ugroups.push_back(u);
    }
    std::vector<CgItem> items;
    std::map<std::tuple<int, int, int>, std::vector<SoloArgs>> solo_by;
    for (size_t m = 0; m < nm; ++m) {
        CgStatus *mirror = reinterpret_cast<CgStatus *>(b->ws) + m;
        const Batch::Member &mem = b->members[m];
        if (mem.solo) {
            SoloArgs a = mem.sargs;
            a.mirror = mirror;
            solo_by[std::make_tuple((int)mem.cfg.fp64, a.M0, a.M1)].push_back(a);
            continue;
        }
        items.push_back(mem.cfg.item);
        items.back().mirror = mirror;
    }
    b->n_items = (int)items.size();
    b->items_off = items.empty() ? 0 : blob_put(b->blob, items.data(), items.size() * sizeof(CgItem));
    b->sgroups.clear();
    for (auto &kv : solo_by) {
        Batch::SGroup g;
        g.fp64 = std::get<0>(kv.first) != 0;
        g.np = (int)kv.second.size();
        g.proto = kv.second[0];
        g.args_off = blob_put(b->blob, kv.second.data(), kv.second.size() * sizeof(SoloArgs));
        b->sgroups.push_back(g);
    }
    if (b->blob_base + b->blob.size() > b->bytes) return bfail(b, FFTGAL_ENOMEM, "batch workspace too small");
    BHIPCHECK(b, hipMemcpyAsync(b->ws + b->blob_base, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice,
                                b->stream));
    b->dirty = false;
    return FFTGAL_OK;
}

}  // namespace

extern "C" {

size_t fftgal_batch_workspace_bytes(int capacity) {
    if (capacity < 1 || capacity > 65536) return 0;
    const size_t mirror = ((size_t)capacity * sizeof(CgStatus) + 255) & ~size_t(255);
    // per member: at most 5 pass argument structs, one update struct, one item,
    // and their offsets, each 256-byte aligned within its group
    return mirror + (size_t)capacity * (5 * kArgSlot + sizeof(UpdArgs) + sizeof(CgItem) + 64) + 64 * 1024;
}

int fftgal_batch_create(struct fftgal_batch **out, int capacity, void *dev_workspace, size_t bytes, void *hip_stream) {
    if (!out) return fail(nullptr, FFTGAL_EINVAL, "out is NULL");
    *out = nullptr;
    const size_t need = fftgal_batch_workspace_bytes(capacity);
    if (need == 0) return fail(nullptr, FFTGAL_EINVAL, "capacity out of range");
    if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 255u))
        return fail(nullptr, FFTGAL_EINVAL, "workspace must be a 256-byte aligned device pointer");
    if (bytes < need) return fail(nullptr, FFTGAL_ENOMEM, "batch workspace has %zu bytes, needs %zu", bytes, need);
    auto *b = new Batch();
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = reinterpret_cast<char *>(dev_workspace);
    b->bytes = bytes;
    b->cap = capacity;
    b->blob_base = ((size_t)capacity * sizeof(CgStatus) + 255) & ~size_t(255);
    *out = b;
    return FFTGAL_OK;
}

int fftgal_batch_add(struct fftgal_batch *b, struct fftgal_plan *pl, int kind, int alpha, double rtol, int maxit,
                     int *solve_id) {
    if (!b) return FFTGAL_EINVAL;
    if (!pl) return bfail(b, FFTGAL_EINVAL, "plan is NULL");
    if (pl->stream != b->stream) return bfail(b, FFTGAL_EINVAL, "the plan must use the batch's stream");
    if (kind != KIND_E && kind != KIND_J) return bfail(b, FFTGAL_EINVAL, "kind must be 0 (primal) or 1 (dual)");
    if (alpha < 0 || alpha >= pl->D.d) return bfail(b, FFTGAL_EINVAL, "alpha %d out of range", alpha);
    if (!(rtol >= 0.0) || maxit < 0) return bfail(b, FFTGAL_EINVAL, "rtol must be >= 0 and maxit >= 0");
    if (!pl->have_mat) return bfail(b, FFTGAL_ESTATE, "plan has no material");
    if (pl->reduced) return bfail(b, FFTGAL_EINVAL, "reduced plans do not join batches");
    if (pl->in_batch[kind][alpha]) return bfail(b, FFTGAL_ESTATE, "this solve of the plan is already in a batch");
    int slot = -1;
    for (int k = 0; k < (int)pl->slot_used.size() && slot < 0; ++k)
        if (!pl->slot_used[k]) slot = k;
    if (slot < 0)
        return bfail(b, FFTGAL_ESTATE, "the plan's %d solve slot(s) are in use (FFTGAL_CONCURRENT gives 2d)",
                     (int)pl->slot_used.size());
    if ((int)b->members.size() >= b->cap) return bfail(b, FFTGAL_ENOMEM, "batch is full");
    pl->slot = slot;
    int rc = start_solve(pl, kind, alpha, rtol, maxit);
    Batch::Member m;
    m.pl = pl;
    m.kind = kind;
    m.alpha = alpha;
    m.slot = slot;
    m.id = b->next_id++;
    if (!rc) rc = capture_iteration(pl, kind, alpha, pl->fp64_iter(), &m.cfg);
    if (!rc && use_solo(pl)) {
        m.solo = true;
        m.sargs = make_solo(pl, kind, alpha);
    }
    pl->slot = 0;
    if (rc) return bfail(b, rc, "start of solve failed: %s", pl->err.c_str());
    pl->busy += 1;
    pl->slot_used[slot] = 1;
    pl->in_batch[kind][alpha] = true;
    pl->solved[kind][alpha] = false;
    b->members.push_back(std::move(m));
    b->dirty = true;
    if (solve_id) *solve_id = b->members.back().id;
    return FFTGAL_OK;
}

int fftgal_batch_step(struct fftgal_batch *b, int iterations, int *n_active) {
    if (!b) return FFTGAL_EINVAL;
    if (iterations < 0) return bfail(b, FFTGAL_EINVAL, "iterations must be >= 0");
    const int nm = (int)b->members.size();
    if (nm == 0 || iterations == 0) {
        if (n_active) *n_active = nm;
        return FFTGAL_OK;
    }
    if (b->dirty) {
        const int rc = batch_rebuild(b);
        if (rc) return rc;
    }
    char *base = b->ws + b->blob_base;
    const CgItem *items = reinterpret_cast<const CgItem *>(base + b->items_off);
    if (!b->sgroups.empty()) {
        // single work-group solves: on the side stream, in launches up to the
        // next FP32 checkpoint of any of them (the checkpoints fall on the same
        // iteration counts as when solved alone)
        if (!b->side) {
            BHIPCHECK(b, hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
            BHIPCHECK(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
            BHIPCHECK(b, hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
        }
        BHIPCHECK(b, hipEventRecord(b->ev_fork, b->stream));
        BHIPCHECK(b, hipStreamWaitEvent(b->side, b->ev_fork, 0));
        int left = iterations;
        while (left > 0) {
            int n = left;
            for (const auto &m : b->members)
                if (m.solo && !m.cfg.fp64) n = std::min(n, kCkptEvery - m.enq % kCkptEvery);
            for (const auto &g : b->sgroups)
                BHIPCHECK(b, launch_solo(g.proto, reinterpret_cast<const SoloArgs *>(base + g.args_off), g.np, n,
                                         g.fp64, b->side));
            for (auto &m : b->members) {
                if (!m.solo) continue;
                m.enq += n;
                if (m.cfg.fp64 || m.enq % kCkptEvery) continue;
                m.pl->slot = m.slot;
                const hipStream_t own = m.pl->stream;
                m.pl->stream = b->side;
                const int rc = checkpoint(m.pl, m.kind, m.alpha, false);
                m.pl->stream = own;
                m.pl->slot = 0;
                if (rc) return bfail(b, rc, "checkpoint failed: %s", m.pl->err.c_str());
            }
            left -= n;
        }
        BHIPCHECK(b, hipEventRecord(b->ev_join, b->side));
    }
    for (int it = 0; it < iterations && b->n_items > 0; ++it) {
        for (size_t i = 0; i < 5; ++i) {
            for (const auto &g : b->groups) {
                if (g.pass != i) continue;
                const int *woff = reinterpret_cast<const int *>(base + g.woff_off);
                if (g.proto.type == 0)
                    BHIPCHECK(b, launch_pencil_multi(g.proto.pa, reinterpret_cast<const PencilArgs *>(base + g.args_off),
                                                     woff, g.np, g.total, g.proto.fp64, b->stream));
                else
                    BHIPCHECK(b, launch_row_multi(g.proto.ra, reinterpret_cast<const RowArgs *>(base + g.args_off),
                                                  woff, g.np, g.total, g.proto.fp64, b->stream));
            }
            for (auto &m : b->members) {
                if (m.solo || i >= m.cfg.passes.size() || pass_fast(m.cfg.passes[i])) continue;
                const PassRec &r = m.cfg.passes[i];
                if (r.type == 0)
                    BHIPCHECK(b, launch_pencil(r.pa, r.nouter, r.fp64, b->stream));
                else
                    BHIPCHECK(b, launch_row(r.ra, r.fp64, b->stream));
            }
        }
        for (const auto &u : b->ugroups)
            BHIPCHECK(b, launch_cg_update_multi(reinterpret_cast<const UpdArgs *>(base + u.args_off),
                                                reinterpret_cast<const int *>(base + u.woff_off), u.np, u.total,
                                                u.fp64, b->stream));
        BHIPCHECK(b, launch_cg_check_multi(items, b->n_items, b->stream));
        // FP32 members: best-iterate checkpoints at the same iteration counts
        // as when solved alone
        for (auto &m : b->members) {
            if (m.solo) continue;
            ++m.enq;
            if (m.cfg.fp64 || m.enq % kCkptEvery) continue;
            m.pl->slot = m.slot;
            const int rc = checkpoint(m.pl, m.kind, m.alpha, false);
            m.pl->slot = 0;
            if (rc) return bfail(b, rc, "checkpoint failed: %s", m.pl->err.c_str());
        }
    }
    if (!b->sgroups.empty()) BHIPCHECK(b, hipStreamWaitEvent(b->stream, b->ev_join, 0));
    b->mirror_host.resize(nm);
    BHIPCHECK(b, hipMemcpyAsync(b->mirror_host.data(), b->ws, nm * sizeof(CgStatus), hipMemcpyDeviceToHost,
                                b->stream));
    BHIPCHECK(b, hipStreamSynchronize(b->stream));
    std::vector<Batch::Member> keep;
    keep.reserve(nm);
    for (int m = 0; m < nm; ++m) {
        Batch::Member &mem = b->members[m];
        const CgStatus &h = b->mirror_host[m];
        if (!h.done) {
            keep.push_back(std::move(mem));
            continue;
        }
        Batch::Done d;
        d.id = mem.id;
        CgStatus hf = h;
        mem.pl->slot = mem.slot;
        const int rc = final_checkpoint(mem.pl, mem.kind, mem.alpha, &hf);
        mem.pl->slot = 0;
        if (rc) return bfail(b, rc, "checkpoint failed: %s", mem.pl->err.c_str());
        d.status = finish_solve(mem.pl, mem.kind, mem.alpha, hf, &d.info);
        mem.pl->busy -= 1;
        mem.pl->slot_used[mem.slot] = 0;
        mem.pl->in_batch[mem.kind][mem.alpha] = false;
        b->done.push_back(d);
        b->dirty = true;
    }
    b->members.swap(keep);
    if (n_active) *n_active = (int)b->members.size();
    return FFTGAL_OK;
}

int fftgal_batch_poll(struct fftgal_batch *b, int *solve_id, fftgal_info *info, int *status) {
    if (!b || b->done.empty()) return 0;
    const Batch::Done d = b->done.front();
    b->done.pop_front();
    if (solve_id) *solve_id = d.id;
    if (info) *info = d.info;
    if (status) *status = d.status;
    return 1;
}

int fftgal_batch_destroy(struct fftgal_batch *b) {
    if (!b) return FFTGAL_OK;
    if (!b->members.empty()) (void)hipStreamSynchronize(b->stream);
    if (b->side) {
        (void)hipStreamSynchronize(b->side);
        (void)hipStreamDestroy(b->side);
        (void)hipEventDestroy(b->ev_fork);
        (void)hipEventDestroy(b->ev_join);
    }
    for (auto &m : b->members) {
        m.pl->busy -= 1;
        m.pl->slot_used[m.slot] = 0;
        m.pl->in_batch[m.kind][m.alpha] = false;
    }
    delete b;
    return FFTGAL_OK;
}

const char *fftgal_batch_last_error(const struct fftgal_batch *b) { return b ? b->err.c_str() : "batch is NULL"; }

int fftgal_solve_all(struct fftgal_plan *pl, double rtol, int maxit, fftgal_info *info) {
    if (!pl) return FFTGAL_EINVAL;
    if (!pl->have_mat) return fail(pl, FFTGAL_ESTATE, "no material set");
    if (pl->busy) return fail(pl, FFTGAL_ESTATE, "the plan has a solve in a batch");
    if (!(rtol >= 0.0) || maxit < 0) return fail(pl, FFTGAL_EINVAL, "rtol must be >= 0 and maxit >= 0");
    const int d = pl->D.d;
    auto hard = [](int rc) { return rc == FFTGAL_EDEVICE || rc == FFTGAL_EINVAL || rc == FFTGAL_ESTATE; };
    if ((int)pl->slot_used.size() < 2 * d || pl->bws_len == 0) {
        // one solve slot: the d primal, then the d dual solves
        const int r1 = solve_entry(pl, KIND_E, -1, rtol, maxit, info);
        if (hard(r1)) return r1;
        const int r2 = solve_entry(pl, KIND_J, -1, rtol, maxit, info ? info + d : nullptr);
        if (hard(r2)) return r2;
        return r1 != FFTGAL_OK ? r1 : r2;
    }
    // all 2d solves as members of one batch: every launch of an iteration
    // covers all of them; each keeps its own reductions, so the results equal
    // those of the solves run one after another
    Batch *b = nullptr;
    int rc = fftgal_batch_create(&b, 2 * d, pl->ws + pl->bws_off, pl->bws_len, pl->stream);
    if (rc) return fail(pl, rc, "internal batch: %s", fftgal_last_error(nullptr));
    int ids[6];
    for (int k = 0; k < 2 && !rc; ++k)
        for (int a = 0; a < d && !rc; ++a) {
            rc = fftgal_batch_add(b, pl, k, a, rtol, maxit, &ids[k * d + a]);
            if (rc) fail(pl, rc, "internal batch: %s", b->err.c_str());
        }
    int active = rc ? 0 : 2 * d;
    while (!rc && active > 0) {
        rc = fftgal_batch_step(b, 16, &active);
        if (rc) fail(pl, rc, "internal batch: %s", b->err.c_str());
    }
    int worst = FFTGAL_OK;
    int sid = 0, st = 0;
    fftgal_info inf{};
    while (fftgal_batch_poll(b, &sid, &inf, &st)) {
        for (int j = 0; j < 2 * d; ++j)
            if (ids[j] == sid) {
                if (info) info[j] = inf;
                if (st != FFTGAL_OK && worst == FFTGAL_OK) worst = st;
            }
    }
    fftgal_batch_destroy(b);
    if (rc) return rc;
    if (worst == FFTGAL_EBREAKDOWN) return fail(pl, worst, "CG breakdown (non-SPD or non-finite material)");
    if (worst == FFTGAL_ENOTCONV) return fail(pl, worst, "a solve did not converge (see info)");
    return worst;
}

}  // extern "C"
