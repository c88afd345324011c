// Tile autotuner of the MFMA contraction kernel.
//
// The first time a contraction shape (precision, output kind, M, N, K, both batch levels, operand
// layouts) is met in an adaptive pass with tuning enabled, every admissible configuration is run on
// a scratch output (beta = 0, so the real output is untouched), timed with HIP events on the
// caller's stream (the least of three runs after a warm-up), and the fastest is kept in a
// process-wide table.  The configurations are the tiles {64 x 64, 128 x 128, and for bf16 planes
// 256 x 128, for outputs of at most 64 columns 64 x 64 on full-width waves, for K of at most 128
// the single-stage 128 x 128, and for K-contiguous operands of at least 256 rows and columns and K a
// multiple of 16 the three-stage 256 x 256 on 32 x 32 MFMA tiles} times the split-K counts {s0, then 2, 3, 4, 5, 6, 8, 12, 16, 24, 32
// above it}, s0 being the least count that keeps FP32 accumulation chains short (1 for FP64 and for
// short K).  Counts that are not powers of two bring a grid of a few hundred tiles closer to a whole
// number of rounds over the compute units (a 2304^3 FP64 contraction: 476 us at 3 splits, 525 us at
// 4, 671 us at 1).  Later contractions of that shape (including fixed passes that are being captured
// into a graph) take the table entry without timing anything.
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "plan.hpp"

namespace dtrg {

namespace {

typedef std::tuple<int, int, int, int, int, int, int, int, int, int> TuneKey;

std::mutex g_mu;
std::map<TuneKey, GemmCfg> g_table;

// the precision field also carries a symmetric output's kind (prec + 16 sym): such an output
// computes about half of its tiles, so it is tuned on its own
TuneKey key_of(Prec prec, Out out, const GemmOp& op) {
    return TuneKey((int)prec + 16 * op.sym, (int)out, op.M, op.N, op.K, op.batch, op.batch2, op.a_kmajor ? 1 : 0,
                   op.b_kmajor ? 1 : 0, prec == Prec::F64 ? 0 : op.max_chain);
}

// largest split-K workspace a trial may claim (elements)
constexpr i64 kMaxTrialPartials = 1LL << 26;
// contractions below this many flops are launch-bound: the heuristic is kept, nothing is timed
constexpr double kMinTunedFlops = 1e8;
// split-K is only tried up to this many blocks in the grid
constexpr i64 kMaxTrialBlocks = 2048;

// candidate split-K counts: the chain floor, then the listed counts above it (ascending)
std::vector<int> split_counts(int minsp) {
    static const int kCounts[] = {2, 3, 4, 5, 6, 8, 12, 16, 24, 32};
    std::vector<int> v{minsp};
    for (int c : kCounts)
        if (c > minsp) v.push_back(c);
    return v;
}

}  // namespace

int tuned_count() {
    std::lock_guard<std::mutex> g(g_mu);
    return (int)g_table.size();
}

// Persisted table: a text file, one shape per line, "dtrg-tune 1" first:
//   prec out M N K batch batch2 a_kmajor b_kmajor max_chain tile splits
// (prec + 16 sym for a symmetric output).  Loaded entries do not replace shapes the process has tuned already.
int tune_load(const std::string& path) {
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return 0;
    char head[32] = {0};
    int ver = 0, n = 0;
    if (std::fscanf(f, "%31s %d", head, &ver) != 2 || std::string(head) != "dtrg-tune" || ver != 1) {
        std::fclose(f);
        throw Error(DTRG_EINVAL, "tile_table " + path + ": not a dtrg-tune 1 file");
    }
    std::lock_guard<std::mutex> g(g_mu);
    for (;;) {
        int v[12];
        int got = 0;
        for (int i = 0; i < 12; ++i) got += std::fscanf(f, "%d", &v[i]) == 1;
        if (got == 0) break;
        // tile 0 and splits 0 are the heuristic's choice (kept for shapes too small to time)
        if (got != 12 || v[10] < 0 || v[10] > 6 || v[11] < 0 || v[11] > 256) {
            std::fclose(f);
            throw Error(DTRG_EINVAL, "tile_table " + path + ": malformed entry " + std::to_string(n + 1));
        }
        const TuneKey key(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9]);
        GemmCfg c;
        c.tile = v[10];
        c.splits = v[11];
        if (g_table.emplace(key, c).second) ++n;
    }
    std::fclose(f);
    return n;
}

void tune_save(const std::string& path) {
    std::map<TuneKey, GemmCfg> snap;
    {
        std::lock_guard<std::mutex> g(g_mu);
        snap = g_table;
    }
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) throw Error(DTRG_EINVAL, "tile_table " + path + ": cannot write");
    std::fprintf(f, "dtrg-tune 1\n");
    for (const auto& e : snap) {
        const TuneKey& k = e.first;
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                     std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k),
                     std::get<9>(k), e.second.tile, e.second.splits);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0)
        throw Error(DTRG_EINVAL, "tile_table " + path + ": cannot write");
}

GemmCfg tuned_cfg(Prec prec, Out out, const GemmOp& op, bool allow_tune, hipStream_t s, Scratch& ws,
                  DevBuf<double>& scratch) {
    const TuneKey key = key_of(prec, out, op);
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_table.find(key);
        if (it != g_table.end()) return it->second;
    }
    if (!allow_tune || op.M == 0 || op.N == 0 || op.K == 0) return op.cfg;
    if (2.0 * op.M * (double)op.N * op.K * op.batch * op.batch2 < kMinTunedFlops) {
        std::lock_guard<std::mutex> g(g_mu);
        g_table[key] = op.cfg;
        return op.cfg;
    }

    const int np = prec_planes(prec);
    const int BK = np > 1 ? 32 : 16;
    const i64 nz = (i64)op.batch * op.batch2;
    const int minsp = gemm_chain_splits(prec, op);
    std::vector<GemmCfg> cands;
    for (int tile = 1; tile <= (np > 1 ? 6 : 2); ++tile) {
        if ((tile == 2 || tile == 5) && std::max(op.M, op.N) < 128) continue;
        if (tile == 6 && (op.a_kmajor || op.b_kmajor || op.M < 256 || op.N < 256 || op.K % 16 != 0)) continue;
        if (tile == 5 && op.K > 128) continue;
        if (tile == 3 && op.M < 256) continue;
        if (tile == 4 && op.N > 64) continue;
        const int BMt = tile_rows(tile), BNt = tile_cols(tile);
        const i64 tm = (op.M + BMt - 1) / BMt, tn = (op.N + BNt - 1) / BNt;
        const i64 tiles = (op.sym == 1 ? tm * (tm + 1) / 2 : tm * tn) * nz;
        // the chain floor is always a candidate (the untuned path would take it too); larger
        // split counts only within the trial limits
        for (int sp : split_counts(minsp)) {
            if (sp > minsp) {
                if (op.K < sp * BK * 2) break;
                if (nz * sp >= 65536) break;
                if (tiles * sp > kMaxTrialBlocks) break;
                if (nz * sp * op.M * op.N > kMaxTrialPartials) break;
            }
            GemmCfg c;
            c.tile = tile;
            c.splits = sp;
            cands.push_back(c);
        }
    }
    // trial output: the real output's extent (all planes) in the scratch buffer
    const int eout = out == Out::F64 ? 8 : (out == Out::F32 ? 4 : 2);
    const int onp = out == Out::Split ? np : 1;
    const i64 ext1 = gemm_c_extent(op);
    const i64 ext = ext1 * onp;
    scratch.ensure((size_t)((ext * eout + 7) / 8));
    hipEvent_t e0, e1;
    DTRG_HIP(hipEventCreate(&e0));
    DTRG_HIP(hipEventCreate(&e1));
    GemmCfg best = gemm_resolve(prec, op);
    float best_ms = 1e30f;
    try {
        for (const GemmCfg& c : cands) {
            GemmOp t = op;
            t.cfg = c;
            t.C = scratch.p;
            t.c_ps = ext1;
            t.c_cap = (i64)scratch.bytes() / eout;
            t.beta = 0.0;
            t.tag = 0;
            gemm(prec, out, t, s, ws);   // warm-up (and workspace growth)
            float ms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                DTRG_HIP(hipEventRecord(e0, s));
                gemm(prec, out, t, s, ws);
                DTRG_HIP(hipEventRecord(e1, s));
                DTRG_HIP(hipEventSynchronize(e1));
                float m = 0.f;
                DTRG_HIP(hipEventElapsedTime(&m, e0, e1));
                ms = std::min(ms, m);
            }
            if (ms < best_ms) { best_ms = ms; best = c; }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> g(g_mu);
    g_table[key] = best;
    return best;
}

}  // namespace dtrg
