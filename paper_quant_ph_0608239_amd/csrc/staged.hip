// LDS-staged passes: several gates per read and write of the state.
//
// The paper distributes the state over processors and calls the qubits held in one processor's
// memory "local": gates on local qubits need no communication (Sec. III.B). Here the same idea is
// applied to one workgroup's LDS. A pass picks m resident qubits R (always the lowest L index bits,
// so that every block is a set of contiguous runs of >= 256 bytes, plus the targets of the next
// pending gates). Block b of the pass holds the 2^m amplitudes whose index bits outside R equal b.
// A workgroup loads its block into LDS, applies, in circuit order, every pending gate whose target
// is resident and that no skipped earlier gate blocks (controls and diagonal gates may sit on any
// qubit: outside R they are constants of the block), then writes the block back once.
//
// Inside a block, gates run in stages. In a stage each thread holds E = 2^LOG_E amplitudes in
// registers: the amplitudes whose local index has the thread's bits at the "thread bits" TB and
// any value at the stage's "register bits" RB (|RB| = LOG_E). Gates whose target is a register
// bit are register-only (no LDS, no barrier); diagonal gates run in any stage. Between stages the
// block goes through LDS once to change RB. LDS slots are padded (one slot per 2^P) so that the
// usual RB/TB splits are free of bank conflicts.
#include <algorithm>
#include <functional>
#include <set>
#include <utility>
#include <array>
#include <cstring>
#include <cmath>
#include <complex>

#include "qsim_internal.h"

#include "staged_device.h"

namespace qsim {

using namespace staged;

namespace staged {
// factors of angle-defined diagonal operations, evaluated once per plan in FP64 on the device, and
// the FP32 copy of every op's coefficients
__global__ void k_op_angles(SOp *ops, int nops)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nops) return;
    SOp &op = ops[i];
    if (op.angles == 1 || op.angles == 3) {
        // 3: theta = s 2 pi / 2^k with s = theta[0], k = theta[1], an exact scaling of FP64 2 pi
        const double th = op.angles == 3 ? op.theta[0] * ldexp(kTwoPi, -int(op.theta[1])) : op.theta[0];
        op.m[0] = 1.0;
        op.m[1] = 0.0;
        sincos(th, &op.m[3], &op.m[2]);
    } else if (op.angles == 2) {
        sincos(op.theta[0], &op.m[1], &op.m[0]);
        sincos(op.theta[1], &op.m[3], &op.m[2]);
    }
    for (int k = 0; k < 8; ++k) op.mf[k] = float(op.m[k]);
}
}  // namespace staged

// ------------------------------------------------------------------------------------------------
// host side: scheduling
// ------------------------------------------------------------------------------------------------
struct StagedPlan;
void staged_free(StagedPlan *p);

// One launch of a staged plan: a pass, or a renormalisation sweep that no pass can take.
enum { kActPass = 0, kActNorm = 1, kActScale = 2 };
struct StagedAct {
    int type;
    int index;  // the pass, or the renormalisation point whose squared norm the sweep writes or applies
};

struct StagedPlan {
    int n = 0, dtype = 0, m = 0, log_e = 0, log_t = 0;
    std::vector<SPass> passes;
    // renormalisation points folded into the passes: per pass, the point whose squared norm scales its
    // loads and the point its stores' norm goes to (-1: none)
    std::vector<int> scale_of, norm_of;
    std::vector<StagedAct> acts;  // launch order
    int renorms = 0;
    SPass *d_passes = nullptr;
    SStage *d_stages = nullptr;
    SRound *d_rounds = nullptr;
    SOp *d_ops = nullptr;
    SBlk *d_blks = nullptr;
    // renormalisation buffer: [0, renorms) squared norms, then kAuxLevel2 level-2 partial sums at
    // aux_l2, then one partial sum per block at aux_part
    double *d_aux = nullptr;
    size_t aux_l2 = 0, aux_part = 0;
};

namespace {

enum GKind { G_DENSE, G_X, G_PHASE, G_DIAG, G_SWAP };

struct GInfo {
    GKind kind;
    int target, target2;
    uint64_t controls;
    uint64_t qmask;   // every qubit the gate touches
    double m[8];
    double theta[2];
    int angles;
};

GInfo describe(const qsim_gate &g)
{
    GInfo d{};
    d.target = g.target;
    d.target2 = g.op == QSIM_OP_SWAP ? g.target2 : -1;
    d.controls = g.controls;
    d.qmask = g.controls | (uint64_t(1) << g.target) | (g.op == QSIM_OP_SWAP ? (uint64_t(1) << g.target2) : 0);
    if (g.op == QSIM_OP_SWAP) {
        d.kind = G_SWAP;
        return d;
    }
    if (g.op == QSIM_OP_PHASE) {
        d.kind = G_PHASE;
        d.angles = 1;
        d.theta[0] = g.theta;
        return d;
    }
    if (g.op == QSIM_OP_RK || g.op == QSIM_OP_RKDG) {  // the angle s 2 pi / 2^k is formed on the device
        d.kind = G_PHASE;
        d.angles = 3;
        d.theta[0] = g.op == QSIM_OP_RK ? 1.0 : -1.0;
        d.theta[1] = double(g.target2);
        return d;
    }
    if (g.op == QSIM_OP_RZ) {
        d.kind = G_DIAG;
        d.angles = 2;
        d.theta[0] = -0.5 * g.theta;
        d.theta[1] = 0.5 * g.theta;
        return d;
    }
    double u[8];
    gate_matrix(g, u);
    switch (classify(u)) {
    case Kind::Phase1: d.kind = G_PHASE; d.m[0] = u[6]; d.m[1] = u[7]; break;
    case Kind::Diag: d.kind = G_DIAG; d.m[0] = u[0]; d.m[1] = u[1]; d.m[2] = u[6]; d.m[3] = u[7]; break;
    case Kind::Swap: d.kind = G_X; memcpy(d.m, u, sizeof(u)); break;
    default: d.kind = G_DENSE; memcpy(d.m, u, sizeof(u)); break;
    }
    return d;
}

inline bool diagonal(const GInfo &g) { return g.kind == G_PHASE || g.kind == G_DIAG; }

// (ar + i ai) <- (ar + i ai)(br + i bi)
inline void cmul_host(double &ar, double &ai, double br, double bi)
{
    const double r = ar * br - ai * bi;
    ai = ar * bi + ai * br;
    ar = r;
}

// Row phases of dense single-qubit gates are carried forward instead of applied. A dense U is
// written U = D U' with D = diag(e0, e1) unitary and U' with a real first column (U'00 = |U00|,
// U'10 = |U10|); U' is applied in U's place and D is carried along the qubit's timeline: diagonal
// gates and gates that use the qubit only as a control commute with it, an uncontrolled quantum
// swap moves it to the other qubit, and X exchanges its two entries (X D = D' X). The next
// uncontrolled dense gate on the qubit absorbs it as a column scaling (U_next D). Where a gate
// that does not commute with it comes (a gate with controls that targets the qubit), or at the end
// of the circuit, D goes back into the gate that split it off: that gate keeps its unsplit matrix
// (every gate between it and here commutes with D). The circuit's unitary is unchanged, no gate is
// added, and a 2x2 with a real first column costs 12 multiply-adds per amplitude pair instead of 16.
void carry_row_phases(int n, std::vector<GInfo> &g)
{
    struct Ph {
        double r0 = 1.0, i0 = 0.0, r1 = 1.0, i1 = 0.0;
        long src = -1;  // index in the output of the gate D was split off, -1: D = identity
    };
    std::vector<Ph> pend(static_cast<size_t>(n), Ph{});
    std::vector<std::array<double, 8>> unsplit;  // matrix of each output gate before the split
    std::vector<GInfo> out;
    out.reserve(g.size());
    unsplit.reserve(g.size());
    auto emit = [&](const GInfo &x) {
        out.push_back(x);
        std::array<double, 8> m;
        memcpy(m.data(), x.m, sizeof(x.m));
        unsplit.push_back(m);
    };
    auto flush = [&](int q) {
        Ph &p = pend[size_t(q)];
        if (p.src >= 0) memcpy(out[size_t(p.src)].m, unsplit[size_t(p.src)].data(), sizeof(out[0].m));
        p = Ph{};
    };
    for (const GInfo &x : g) {
        if (diagonal(x)) {
            emit(x);
            continue;
        }
        if (x.kind == G_SWAP) {
            if (x.controls == 0) {
                std::swap(pend[size_t(x.target)], pend[size_t(x.target2)]);
            } else {
                flush(x.target);
                flush(x.target2);
            }
            emit(x);
            continue;
        }
        const int q = x.target;
        Ph &p = pend[size_t(q)];
        if (x.controls != 0) {
            flush(q);
            emit(x);
            continue;
        }
        if (x.kind == G_X) {
            std::swap(p.r0, p.r1);
            std::swap(p.i0, p.i1);
            emit(x);
            continue;
        }
        GInfo y = x;
        cmul_host(y.m[0], y.m[1], p.r0, p.i0);  // column 0 times e0
        cmul_host(y.m[4], y.m[5], p.r0, p.i0);
        cmul_host(y.m[2], y.m[3], p.r1, p.i1);  // column 1 times e1
        cmul_host(y.m[6], y.m[7], p.r1, p.i1);
        emit(y);  // records the unsplit matrix U D
        GInfo &z = out.back();
        Ph e;
        for (int k = 0; k < 2; ++k) {  // row k divided by the phase of its first entry
            double &ar = z.m[4 * k], &ai = z.m[4 * k + 1];
            const double a = std::hypot(ar, ai);
            double er = 1.0, ei = 0.0;
            if (a > 0.0) {
                er = ar / a;
                ei = ai / a;
            }
            ar = a;
            ai = 0.0;
            cmul_host(z.m[4 * k + 2], z.m[4 * k + 3], er, -ei);
            (k == 0 ? e.r0 : e.r1) = er;
            (k == 0 ? e.i0 : e.i1) = ei;
        }
        const bool trivial = e.r0 == 1.0 && e.i0 == 0.0 && e.r1 == 1.0 && e.i1 == 0.0;
        e.src = trivial ? -1 : long(out.size() - 1);
        p = e;
    }
    for (int q = 0; q < n; ++q) flush(q);
    g.swap(out);
}

}  // namespace

// kernel variants: (amplitudes per thread, threads) per dtype; see launch_pass
// block shapes that have a half-buffer kernel
static bool half_variant(int dtype, int log_e, int log_t)
{
    if (dtype == QSIM_C128) return log_e == 4 && log_t >= 6 && log_t <= 8;
    return log_e == 5 && log_t >= 6 && log_t <= 8;  // with 16 amplitudes per thread the full buffer measured faster
}

bool staged::staged_variant_ok(int dtype, int log_e, int log_t)
{
    if (log_t < 6 || log_t > 10) return false;
    if (dtype == QSIM_C128) return (log_e == 3 && log_t >= 7 && log_t <= 9) || (log_e == 4 && log_t <= 9);
    return (log_e == 4 && log_t >= 7) || (log_e == 5 && log_t <= 9);
}

namespace {

// an op of the stage being built, with what the round placement needs
struct HOp {
    bool dense;
    int lb;             // dense: local bit of the target
    int target;         // physical target qubit
    uint64_t controls;  // physical control qubits
    uint64_t qmask;     // every qubit the gate touches
    uint64_t gcm;       // condition on non-resident bits
    uint32_t lcm;       // condition on resident bits (local positions)
    double m[8];        // dense 2x2, or diag d0 = m[0..1], d1 = m[2..3]
    double theta[2];
    int angles;
    int pair = -1;      // a two-qubit block: its index in the stage's block list (dense is false)
    int lb2 = -1;       // a two-qubit block: local bit of its higher-ranked register bit (lb: the lower)
};

// ordering key of the flip list: after the register-bit lists and the pair lists (the diagonal list
// follows it)
constexpr int flip_key_of(int log_e) { return kLists * log_e + npairs(log_e); }

// two ops of a stage may run in either order
bool commute(const HOp &a, const HOp &b)
{
    if (a.pair >= 0 || b.pair >= 0) return (a.qmask & b.qmask) == 0;
    if (!a.dense && !b.dense) return true;
    if (a.dense && !b.dense) return !((b.qmask >> a.target) & 1);
    if (!a.dense && b.dense) return !((a.qmask >> b.target) & 1);
    return a.target != b.target && !((b.controls >> a.target) & 1) && !((a.controls >> b.target) & 1);
}

}  // namespace

// Thread bits of a stage, lowest lane first. LDS slot s(e) = e + (e >> P) (one pad slot per 2^P)
// puts a lane bit at local position b < 2P on the bank group of b mod P (and higher positions on
// none), so the first P lanes take one position from each residue class where the register bits
// leave one: then the 2^P lanes of a wide LDS access hit distinct bank groups. The low run keeps its
// order (0, 1, ... are their own classes), so stages that read memory directly stay coalesced.
// nfix local bits fb[i] are pinned at thread positions fj[i] (the split bits of the half-buffer
// exchanges: either at a position >= P, or a low-run bit at its own position); the bank-class picks
// and then the remaining bits in ascending order take the free positions.
static void order_threads(SStage &cur, uint32_t rbset, int m, int log_e, int dtype, const uint8_t *R, int nfix,
                          const int *fj, const int *fb)
{
    const int P = dtype == QSIM_C128 ? 4 : 5;
    const int lt = m - log_e;
    uint32_t left = ((1u << m) - 1) & ~rbset;
    uint32_t taken_pos = 0, done_class = 0;
    for (int i = 0; i < nfix; ++i) {
        cur.tbits[fj[i]] = uint8_t(fb[i]);
        left &= ~(1u << fb[i]);
        taken_pos |= 1u << fj[i];
        if (fb[i] < 2 * P) done_class |= 1u << (fb[i] % P);
    }
    int jt = 0;
    for (int c = 0; c < P; ++c) {
        if ((done_class >> c) & 1) continue;
        for (int b = c; b < 2 * P && b < m; b += P)
            if ((left >> b) & 1) {
                while ((taken_pos >> jt) & 1) ++jt;
                if (jt >= lt) break;
                cur.tbits[jt++] = uint8_t(b);
                left &= ~(1u << b);
                break;
            }
    }
    for (int b = 0; b < m; ++b)
        if ((left >> b) & 1) {
            while ((taken_pos >> jt) & 1) ++jt;
            cur.tbits[jt++] = uint8_t(b);
        }
    for (int j = 0; j < lt; ++j) cur.ptb[j] = R[cur.tbits[j]];
}

// Close a stage: fix its register bits, turn every op's condition into its register part (pair or
// element masks) and its thread part, and order the ops into rounds. An op goes to the earliest
// round in which it runs after every earlier op of the stage it does not commute with (within a
// round: bit 0 ops, ..., bit LOG_E-1 ops, unconditional before conditional, then diagonal ops).
// Two-qubit blocks of a stage. Walking the ops in circuit order, each register bit may belong to one
// open block: a single-qubit block (the ops on that bit alone so far) or a pair block (ops on that bit
// and one other register bit). An unconditional single-qubit op joins its bit's block or opens one; a
// two-qubit diagonal op (CZ, a controlled phase with a given factor) on two register bits joins their
// common pair block, or opens a pair block that takes in both bits' single-qubit blocks; if either bit
// is in a pair block with a third bit, it closes both bits' blocks and stays a separate op. Any other
// op closes the blocks of every register bit it touches. A closed block is placed where it closes: every op between one of its members and that
// place touches neither of its bits (it would have joined or closed the block), so it commutes with
// the members. A pair block with at least three dense members is multiplied into one 4x4 (FP64, in
// member order); any other block keeps its members as separate ops.
static std::vector<HOp> form_pair_blocks(const std::vector<HOp> &sops, uint32_t rbset, int m, const int *localof,
                                         const std::function<int(int)> &rank_of,
                                         std::vector<std::array<std::complex<double>, 16>> &mats)
{
    using cd = std::complex<double>;
    const size_t N = sops.size();
    auto regbits_of = [&](const HOp &h) {  // local register bits the op touches, or ~0u if it touches
        uint32_t lb = 0;                  // a non-resident qubit or a thread bit
        for (int q = 0; q < 64; ++q)
            if ((h.qmask >> q) & 1) {
                const int l = localof[q];
                if (l < 0 || !((rbset >> l) & 1)) return ~0u;
                lb |= 1u << l;
            }
        return lb;
    };
    auto blockable = [&](const HOp &h, uint32_t lb) {
        if (lb == ~0u || h.gcm != 0) return false;
        if (h.dense) return h.controls == 0 && __builtin_popcount(lb) == 1;
        return h.angles == 0 && __builtin_popcount(lb) <= 2;
    };
    struct Blk {
        uint32_t bits;
        std::vector<size_t> members;
        bool merged = false;
    };
    std::vector<Blk> blks;
    std::vector<int> owner(size_t(m), -1);
    std::vector<std::pair<long, int>> order;  // (op index, -1) or (-1, block index)
    auto close = [&](int id) {
        order.push_back({-1, id});
        for (int l = 0; l < m; ++l)
            if (owner[size_t(l)] == id) owner[size_t(l)] = -1;
    };
    for (size_t xi = 0; xi < N; ++xi) {
        const HOp &h = sops[xi];
        const uint32_t lb = regbits_of(h);
        if (!blockable(h, lb)) {
            for (int q = 0; q < 64; ++q)
                if ((h.qmask >> q) & 1) {
                    const int l = localof[q];
                    if (l >= 0 && owner[size_t(l)] >= 0) close(owner[size_t(l)]);
                }
            order.push_back({long(xi), -1});
            continue;
        }
        if (__builtin_popcount(lb) == 1) {
            const int l = __builtin_ctz(lb);
            if (owner[size_t(l)] < 0) {
                blks.push_back(Blk{lb, {}});
                owner[size_t(l)] = int(blks.size()) - 1;
            }
            blks[size_t(owner[size_t(l)])].members.push_back(xi);
            continue;
        }
        const int a = __builtin_ctz(lb), b = 31 - __builtin_clz(lb);
        int oa = owner[size_t(a)], ob = owner[size_t(b)];
        if (oa >= 0 && oa == ob) {
            blks[size_t(oa)].members.push_back(xi);
            continue;
        }
        auto is_pair = [&](int o) { return o >= 0 && __builtin_popcount(blks[size_t(o)].bits) == 2; };
        if (is_pair(oa) || is_pair(ob)) {
            // a two-qubit op across two blocks ends them both and runs on its own (on a layered circuit
            // each pair block then spans two single-qubit layers around its own two-qubit op)
            if (oa >= 0) close(oa);
            if (ob >= 0) close(ob);
            order.push_back({long(xi), -1});
            continue;
        }
        Blk nb{lb, {}};
        for (int o : {oa, ob})
            if (o >= 0) {
                nb.members.insert(nb.members.end(), blks[size_t(o)].members.begin(), blks[size_t(o)].members.end());
                blks[size_t(o)].merged = true;
            }
        std::sort(nb.members.begin(), nb.members.end());
        nb.members.push_back(xi);
        blks.push_back(nb);
        owner[size_t(a)] = owner[size_t(b)] = int(blks.size()) - 1;
    }
    for (int l = 0; l < m; ++l)
        if (owner[size_t(l)] >= 0) close(owner[size_t(l)]);

    std::vector<HOp> out;
    for (const auto &o : order) {
        if (o.first >= 0) {
            out.push_back(sops[size_t(o.first)]);
            continue;
        }
        const Blk &bk = blks[size_t(o.second)];
        if (bk.merged) continue;
        int ndense = 0;
        for (size_t xi : bk.members) ndense += sops[xi].dense;
        if (__builtin_popcount(bk.bits) != 2 || ndense < 3) {
            for (size_t xi : bk.members) out.push_back(sops[xi]);
            continue;
        }
        // the block's 4x4: p = bit of the lower-ranked register bit + 2 * bit of the higher one
        const int la = __builtin_ctz(bk.bits), lb2 = 31 - __builtin_clz(bk.bits);
        const int lo_l = rank_of(la) < rank_of(lb2) ? la : lb2, hi_l = lo_l == la ? lb2 : la;
        std::array<cd, 16> M{};
        for (int p = 0; p < 4; ++p) M[size_t(5 * p)] = 1.0;
        uint64_t qm = 0;
        for (size_t xi : bk.members) {
            const HOp &h = sops[xi];
            qm |= h.qmask;
            std::array<cd, 16> G{};
            auto bitof = [&](int p, int l) { return l == lo_l ? (p & 1) : ((p >> 1) & 1); };
            if (h.dense) {
                const int t = localof[h.target];
                const cd u[2][2] = {{cd(h.m[0], h.m[1]), cd(h.m[2], h.m[3])}, {cd(h.m[4], h.m[5]), cd(h.m[6], h.m[7])}};
                const int o = t == lo_l ? hi_l : lo_l;
                for (int po = 0; po < 4; ++po)
                    for (int pi = 0; pi < 4; ++pi)
                        if (bitof(po, o) == bitof(pi, o)) G[size_t(4 * po + pi)] = u[bitof(po, t)][bitof(pi, t)];
            } else {
                const int t = localof[h.target];
                const cd d0(h.m[0], h.m[1]), d1(h.m[2], h.m[3]);
                for (int p = 0; p < 4; ++p) {
                    bool cond = true;  // controls of a diagonal op are register bits of this pair
                    for (int q = 0; q < 64; ++q)
                        if (((h.controls >> q) & 1) && !bitof(p, localof[q])) cond = false;
                    G[size_t(5 * p)] = cond ? (bitof(p, t) ? d1 : d0) : cd(1.0);
                }
            }
            std::array<cd, 16> P{};
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    cd acc = 0.0;
                    for (int k = 0; k < 4; ++k) acc += G[size_t(4 * r + k)] * M[size_t(4 * k + c)];
                    P[size_t(4 * r + c)] = acc;
                }
            M = P;
        }
        HOp hb{};
        hb.dense = false;
        hb.pair = int(mats.size());
        hb.lb = lo_l;
        hb.target = -1;
        hb.qmask = qm;
        hb.lb2 = hi_l;
        mats.push_back(M);
        out.push_back(hb);
    }
    return out;
}

static void emit_stage(SStage cur, uint32_t rbset, int log_e, int m, int dtype, const int *localof, const uint8_t *R,
                       const std::vector<HOp> &sops_in, std::vector<SStage> &stages, std::vector<SRound> &rounds,
                       std::vector<SOp> &ops, std::vector<SBlk> &blks_out)
{
    const int E = 1 << log_e;
    int nrb = __builtin_popcount(rbset);
    // fill the register bits from the top local bits so the thread bits keep the low ones
    for (int s = m - 1; s >= 0 && nrb < log_e; --s)
        if (!((rbset >> s) & 1)) {
            rbset |= 1u << s;
            ++nrb;
        }
    for (int s = 0, j = 0; s < m; ++s)
        if ((rbset >> s) & 1) cur.rb[j++] = uint8_t(s);
    order_threads(cur, rbset, m, log_e, dtype, R, 0, nullptr, nullptr);
    for (int j = 0; j < log_e; ++j) cur.prb[j] = R[cur.rb[j]];
    auto rank_of = [&](int lb) { return __builtin_popcount(rbset & ((1u << lb) - 1)); };
    std::vector<std::array<std::complex<double>, 16>> mats;
    const std::vector<HOp> sops = form_pair_blocks(sops_in, rbset, m, localof, rank_of, mats);
    const size_t N = sops.size();
    std::vector<SOp> rec(N);
    std::vector<int> key(N), round(N);
    int nrounds = 0;
    for (size_t xi = 0; xi < N; ++xi) {
        const HOp &h = sops[xi];
        SOp o{};
        o.lt = -1;
        o.alt_rank = -1;
        o.gcm = h.gcm;
        uint32_t rsel = 0;  // register part of the condition, over the register index r
        for (int s = 0; s < m; ++s)
            if (((h.lcm >> s) & 1) && ((rbset >> s) & 1)) rsel |= 1u << rank_of(s);
        o.lcm_t = h.lcm & ~rbset;
        o.angles = h.angles;
        o.theta[0] = h.theta[0];
        o.theta[1] = h.theta[1];
        memcpy(o.m, h.m, sizeof(o.m));
        if (h.pair >= 0) {
            key[xi] = kLists * log_e + pair_index(log_e, rank_of(h.lb), rank_of(h.lb2));
        } else if (h.dense) {
            const int j = rank_of(h.lb);
            for (int p = 0; p < E / 2; ++p) {
                const int r = (p & ((1 << j) - 1)) | ((p >> j) << (j + 1));
                if ((uint32_t(r) & rsel) == rsel) o.pmask |= 1u << p;
            }
            // the unconditional lists take 2x2s with a real first column only; any other runs
            // through the conditional list (with an always-true condition)
            const bool rc = h.m[1] == 0.0 && h.m[5] == 0.0;
            const bool cond = o.lcm_t != 0 || rsel != 0 || o.gcm != 0 || !rc;
            key[xi] = kLists * j + (cond ? kListCond : 0);
        } else {
            const bool d0_one = h.angles == 1 || h.angles == 3 || (h.angles == 0 && h.m[0] == 1.0 && h.m[1] == 0.0);
            const int lt = localof[h.target];
            if (lt >= 0 && ((rbset >> lt) & 1)) {
                const int jt = rank_of(lt);
                for (int r = 0; r < E; ++r) {
                    if ((uint32_t(r) & rsel) != rsel) continue;
                    if ((r >> jt) & 1) o.m1 |= 1u << r;
                    else if (!d0_one) o.m0 |= 1u << r;
                }
            } else {
                for (int r = 0; r < E; ++r)
                    if ((uint32_t(r) & rsel) == rsel) o.m1 |= 1u << r;
                if (lt >= 0) {
                    if (d0_one) o.lcm_t |= 1u << lt;  // only lanes with the target bit set change
                    else o.lt = lt;
                } else {
                    const uint64_t tb = uint64_t(1) << h.target;
                    if (d0_one) o.gcm |= tb;  // only blocks with the target bit set change
                    else o.gtb = tb;
                }
            }
            // a sign flip: d0 = 1 and d1 = -1 exactly, with the target folded into the condition
            const bool flip = d0_one && h.angles == 0 && h.m[2] == -1.0 && h.m[3] == 0.0 && o.m0 == 0 && o.lt < 0 &&
                              o.gtb == 0;
            key[xi] = flip_key_of(log_e) + (flip ? 0 : 1);
        }
        int k = 0;
        for (size_t y = 0; y < xi; ++y)
            if (!commute(h, sops[y])) k = std::max(k, key[y] <= key[xi] ? round[y] : round[y] + 1);
        round[xi] = k;
        nrounds = std::max(nrounds, k + 1);
        rec[xi] = o;
    }
    // Fuse two-qubit sign flips (CZ) into the dense op that runs last before them in their round on
    // one of their qubits: the flip then acts as a row negation of that op's 2x2, chosen per pair
    // (other qubit a register bit), per lane (a thread bit) or per block (a non-resident bit). Every
    // op executed between the dense op and the flip's place commutes with the flip, so the order
    // of non-commuting operations is unchanged.
    const int flip_key = flip_key_of(log_e);
    std::vector<char> gone(N, 0);
    auto bit_of_key = [&](int kk) { return kk / kLists; };
    // condition of a fused flip on the qubit other than the dense op's target
    auto set_alt = [&](size_t d, uint64_t q2, int j, bool col) {
        const uint64_t other = q2 & ~(uint64_t(1) << sops[d].target);
        const int qo = __builtin_ctzll(other);
        const int lo = localof[qo];
        SOp &o = rec[d];
        o.alt_col = col ? 1u : 0u;
        o.alt_rank = -1;
        if (lo >= 0 && ((rbset >> lo) & 1)) {
            const int jo = rank_of(lo);
            o.alt_rank = jo;
            for (int p = 0; p < E / 2; ++p) {
                const int r = (p & ((1 << j) - 1)) | ((p >> j) << (j + 1));
                if ((r >> jo) & 1) o.amask |= 1u << p;
            }
            key[d] = kLists * j + kListPairFlip + (jo < j ? jo : jo - 1);
        } else if (lo >= 0) {
            o.amask = (1u << (E / 2)) - 1;
            o.alt_lcm = 1u << lo;
            key[d] = kLists * j + kListLaneFlip;
        } else {
            o.amask = (1u << (E / 2)) - 1;
            o.galt = other;
            key[d] = kLists * j + kListBlockFlip;
        }
    };
    // a two-qubit block on one of the qubits q2 in rounds [r0, r1)
    auto pair_between = [&](int r0, int r1, uint64_t q2) {
        for (size_t yi = 0; yi < N; ++yi)
            if (sops[yi].pair >= 0 && round[yi] >= r0 && round[yi] < r1 && (sops[yi].qmask & q2)) return true;
        return false;
    };
    // the only dense op of its round on its register bit
    auto alone = [&](size_t d) {
        const int j = bit_of_key(key[d]);
        for (size_t yi = 0; yi < N; ++yi)
            if (yi != d && !gone[yi] && round[yi] == round[d] && sops[yi].dense && bit_of_key(key[yi]) == j && key[yi] < flip_key)
                return false;
        return true;
    };
    for (size_t xi = 0; xi < N; ++xi) {
        if (key[xi] != flip_key || __builtin_popcountll(sops[xi].controls) != 1) continue;
        const uint64_t q2 = (uint64_t(1) << sops[xi].target) | sops[xi].controls;
        // the dense op of this round on one of the flip's qubits that executes last
        long best = -1;
        for (size_t yi = 0; yi < N; ++yi) {
            if (gone[yi] || round[yi] != round[xi] || !sops[yi].dense || !((q2 >> sops[yi].target) & 1)) continue;
            if (best < 0 || key[yi] > key[size_t(best)] || (key[yi] == key[size_t(best)] && yi > size_t(best))) best = long(yi);
        }
        if (best < 0) continue;
        const size_t d = size_t(best);
        if (key[d] % kLists != 0 || !alone(d)) continue;  // only a plain unconditional op takes a flip
        // the round's two-qubit blocks run after its single-bit lists and before its flips
        if (pair_between(round[xi], round[xi] + 1, q2)) continue;
        set_alt(d, q2, bit_of_key(key[d]), false);
        gone[xi] = 1;
    }
    // the flips left: fuse each into the first dense op executed after it (later rounds of the stage)
    // on one of its qubits, as a column negation
    for (size_t xi = 0; xi < N; ++xi) {
        if (gone[xi] || key[xi] != flip_key || __builtin_popcountll(sops[xi].controls) != 1) continue;
        const uint64_t q2 = (uint64_t(1) << sops[xi].target) | sops[xi].controls;
        long best = -1;
        for (size_t yi = 0; yi < N; ++yi) {
            if (gone[yi] || round[yi] <= round[xi] || !sops[yi].dense || !((q2 >> sops[yi].target) & 1)) continue;
            if (best < 0 || round[yi] < round[size_t(best)] ||
                (round[yi] == round[size_t(best)] && (key[yi] < key[size_t(best)] || (key[yi] == key[size_t(best)] && yi < size_t(best)))))
                best = long(yi);
        }
        if (best < 0) continue;
        const size_t d = size_t(best);
        if (key[d] % kLists != 0 || !alone(d)) continue;
        if (pair_between(round[xi] + 1, round[d], q2)) continue;
        set_alt(d, q2, bit_of_key(key[d]), true);
        gone[xi] = 1;
    }
    cur.round_begin = int(rounds.size());
    // keys: register-bit lists, then pair lists, then flips and diagonal ops; the pair lists go to
    // pseg (block table), everything else to seg (op table)
    const int fk = flip_key_of(log_e);
    for (int k = 0; k < nrounds; ++k) {
        SRound rd{};
        for (int list = 0; list <= fk + 1; ++list) {
            const bool pl = list >= kLists * log_e && list < fk;
            if (pl) rd.pseg[list - kLists * log_e] = int(blks_out.size());
            else rd.seg[list < fk ? list : list - npairs(log_e)] = int(ops.size());
            for (size_t xi = 0; xi < N; ++xi) {
                if (gone[xi] || round[xi] != k || key[xi] != list) continue;
                if (pl) {
                    SBlk b{};
                    const auto &M = mats[size_t(sops[xi].pair)];
                    for (int e = 0; e < 16; ++e) {
                        b.m[2 * e] = M[size_t(e)].real();
                        b.m[2 * e + 1] = M[size_t(e)].imag();
                        b.mf[2 * e] = float(b.m[2 * e]);
                        b.mf[2 * e + 1] = float(b.m[2 * e + 1]);
                    }
                    blks_out.push_back(b);
                } else {
                    ops.push_back(rec[xi]);
                }
            }
        }
        rd.pseg[npairs(log_e)] = int(blks_out.size());
        rd.seg[kLists * log_e + 2] = int(ops.size());
        rounds.push_back(rd);
    }
    cur.round_end = int(rounds.size());
    stages.push_back(cur);
}

// Schedule `gates` for an n-qubit state into passes of m resident qubits with 2^log_e amplitudes per
// thread; passes, stages, rounds and ops are appended to the given tables (indices are absolute).
// Half-buffer form of a pass: for every LDS round trip (load layout -> first stage, stage -> next
// stage, last stage -> store layout) pick a split bit that sits at the same thread position in both
// layouts (in the load/store layout, local bit j is at thread position j), then pin those positions in
// each stage's thread order. Splits that are all at wave positions (>= 6: whole wavefronts per half)
// select the wave-split kernel (SPass::direct bit 3); otherwise a split bit >= 2P, which leaves the bank
// groups of the other bits unchanged, is preferred. Returns false (the pass keeps the full buffer) if a
// round trip has no such bit or the pass ends a stage with a quantum swap.
static bool assign_half(SPass &ps, std::vector<SStage> &stages, int m, int log_e, int dtype)
{
    const int lt = m - log_e, P = dtype == QSIM_C128 ? 4 : 5;
    if (lt <= P) return false;
    const int s0 = ps.stage_begin, ns = ps.stage_end - ps.stage_begin;
    std::vector<uint32_t> T(static_cast<size_t>(ns)), rbs(static_cast<size_t>(ns));
    for (int s = 0; s < ns; ++s) {
        const SStage &st = stages[size_t(s0 + s)];
        if (st.swap_p >= 0) return false;
        uint32_t rb = 0;
        for (int j = 0; j < log_e; ++j) rb |= 1u << st.rb[j];
        rbs[size_t(s)] = rb;
        T[size_t(s)] = ((1u << m) - 1) & ~rb;
    }
    std::vector<int> bi(size_t(ns), -1), ji(size_t(ns), -1), bo(size_t(ns), -1), jo(size_t(ns), -1);
    // Round trip s leaves stage s (s = -1: the load into stage 0; s = ns - 1: the store). Its split
    // (b, j) has b in cand_of(s); in the load/store layout b == j. A position below P holds a low-run
    // bit at its own position only, and a low-run bit elsewhere only between stages that do not touch
    // memory directly (those keep the low run on their first lanes in order), except the top one at a
    // wave position. Within the stage it shares with the previous round trip, one bit per position.
    auto needed = [&](int s) { return s < 0 ? !(ps.direct & 1) : s == ns - 1 ? !(ps.direct & 2) : true; };
    auto cand_of = [&](int s) { return s < 0 ? T[0] : s == ns - 1 ? T[size_t(s)] : T[size_t(s)] & T[size_t(s + 1)]; };
    auto valid = [&](int s, int b, int j, int in_b, int in_j) {
        if (!((cand_of(s) >> b) & 1)) return false;
        if ((s < 0 || s == ns - 1) && b != j) return false;
        if ((j < P || b < P) && b != j) {
            if (j < P) return false;
            // next to a stage that touches memory directly, only the top low-run bit may move (to a
            // wave position): its lanes then still cover 2^(P-1) consecutive amplitudes (128 bytes)
            if (((s == 0 && (ps.direct & 1)) || (s + 1 == ns - 1 && (ps.direct & 2))) && (b != P - 1 || j < 6))
                return false;
        }
        return in_j < 0 || ((j == in_j) == (b == in_b));
    };
    // First look for splits that are all at wave positions (uniform halves: the 128-VGPR kernel), by a
    // depth-first search along the chain of round trips, remembering failed states.
    std::vector<int> wb(size_t(ns + 1), -1), wj(size_t(ns + 1), -1);
    std::vector<char> failed(size_t((ns + 1) * (m + 1) * (lt + 1)), 0);
    std::function<bool(int, int, int)> dfs = [&](int s, int in_b, int in_j) -> bool {
        if (s == ns) return true;
        char &f = failed[size_t(((s + 1) * (m + 1) + (in_b + 1)) * (lt + 1) + (in_j + 1))];
        if (f) return false;
        if (!needed(s)) {
            wb[size_t(s + 1)] = wj[size_t(s + 1)] = -1;
            if (dfs(s + 1, -1, -1)) return true;
        } else {
            for (int j = lt - 1; j >= 6; --j)
                for (int b = m - 1; b >= 0; --b) {
                    if (!valid(s, b, j, in_b, in_j)) continue;
                    wb[size_t(s + 1)] = b;
                    wj[size_t(s + 1)] = j;
                    if (dfs(s + 1, b, j)) return true;
                }
        }
        f = 1;
        return false;
    };
    const bool wave = lt > 6 && dfs(-1, -1, -1);
    if (wave) {
        for (int s = -1; s < ns; ++s) {
            if (s >= 0) {
                bo[size_t(s)] = wb[size_t(s + 1)];
                jo[size_t(s)] = wj[size_t(s + 1)];
            }
            if (s + 1 < ns) {
                bi[size_t(s + 1)] = wb[size_t(s + 1)];
                ji[size_t(s + 1)] = wj[size_t(s + 1)];
            }
        }
    } else {
        // otherwise the best split per round trip in order (a position >= 6 and a bit >= 2P preferred)
        auto pick = [&](int s, int &b_out, int &j_out) {
            const int in_b = s >= 0 ? bi[size_t(s)] : -1, in_j = s >= 0 ? ji[size_t(s)] : -1;
            int best = -1;
            for (int j = 0; j < lt; ++j)
                for (int b = 0; b < m; ++b) {
                    if (!valid(s, b, j, in_b, in_j)) continue;
                    const int sc = (j >= 6 ? 10000 : 0) + (b >= 2 * P ? 1000 : 0) + (b >= P ? 500 : 0) + 32 * j + b;
                    if (sc > best) {
                        best = sc;
                        b_out = b;
                        j_out = j;
                    }
                }
            return best >= 0;
        };
        if (needed(-1) && !pick(-1, bi[0], ji[0])) return false;
        for (int s = 0; s + 1 < ns; ++s) {
            if (!pick(s, bo[size_t(s)], jo[size_t(s)])) return false;
            bi[size_t(s + 1)] = bo[size_t(s)];
            ji[size_t(s + 1)] = jo[size_t(s)];
        }
        if (needed(ns - 1) && !pick(ns - 1, bo[size_t(ns - 1)], jo[size_t(ns - 1)])) return false;
    }
    for (int s = 0; s < ns; ++s) {
        SStage &st = stages[size_t(s0 + s)];
        int fj[2], fb[2], nf = 0;
        if (ji[size_t(s)] >= 0) {
            fj[nf] = ji[size_t(s)];
            fb[nf++] = bi[size_t(s)];
        }
        if (jo[size_t(s)] >= 0 && jo[size_t(s)] != ji[size_t(s)]) {
            fj[nf] = jo[size_t(s)];
            fb[nf++] = bo[size_t(s)];
        }
        order_threads(st, rbs[size_t(s)], m, log_e, dtype, ps.R, nf, fj, fb);
        st.hb_in = uint8_t(std::max(bi[size_t(s)], 0));
        st.hj_in = uint8_t(std::max(ji[size_t(s)], 0));
        st.hb_out = uint8_t(std::max(bo[size_t(s)], 0));
        st.hj_out = uint8_t(std::max(jo[size_t(s)], 0));
    }
    ps.direct |= wave ? 12 : 4;
    return true;
}

int staged::staged_schedule(int n, int dtype, int m, int log_e, const std::vector<qsim_gate> &gates,
                            std::vector<SPass> &passes, std::vector<SStage> &stages, std::vector<SRound> &rounds,
                            std::vector<SOp> &ops, std::vector<SBlk> &blks, int search_width)
{
    if (m > kMaxM || log_e < 1 || log_e > kMaxLogE || m - log_e > kMaxLogT || m - log_e < 0)
        return set_error(QSIM_EINVAL, "staged: block shape outside the kernel tables");
    const int L = dtype == QSIM_C128 ? 4 : 5;  // low run: 2^L amplitudes = 256 bytes
    std::vector<GInfo> gi(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) gi[i] = describe(gates[i]);
    carry_row_phases(n, gi);
    const size_t G = gi.size();
    std::vector<char> done(G, 0);
    size_t ndone = 0;

    // gates that a pass with resident set R executes after the gates marked in dn, in circuit order:
    // a gate runs when none of its qubits is held back by an earlier gate that does not run, and it is
    // diagonal or its target(s) are resident
    auto executable = [&](const std::vector<char> &dn, uint64_t R, std::vector<size_t> *take) {
        int dense = 0, all = 0;
        uint64_t blocked = 0;
        for (size_t i = 0; i < G; ++i) {
            if (dn[i]) continue;
            const GInfo &g = gi[i];
            if (g.qmask & blocked) {
                blocked |= g.qmask;
                continue;
            }
            bool ok = diagonal(g) || ((R >> g.target) & 1);
            if (g.kind == G_SWAP) ok = ((R >> g.target) & 1) && ((R >> g.target2) & 1);
            if (ok) {
                ++all;
                if (!diagonal(g)) ++dense;
                if (take) take->push_back(i);
            } else {
                blocked |= g.qmask;
            }
        }
        return std::make_pair(dense, all);
    };
    // Resident-set candidates of the next pass: the low run plus the targets of the earliest pending
    // non-diagonal gates, and the low run plus every window of m - L consecutive qubits above it (a
    // window lets a pass run the light cone of neighbouring-qubit circuits several layers deep).
    auto candidates = [&](const std::vector<char> &dn) {
        std::vector<uint64_t> c;
        uint64_t R = (uint64_t(1) << L) - 1;
        int cnt = L;
        for (size_t i = 0; i < G && cnt < m; ++i) {
            if (dn[i] || diagonal(gi[i])) continue;
            const int tg[2] = {gi[i].target, gi[i].target2};
            const int need = (gi[i].kind == G_SWAP) ? 2 : 1;
            int missing = 0;
            for (int k = 0; k < need; ++k)
                if (!((R >> tg[k]) & 1)) ++missing;
            if (cnt + missing > m) break;
            for (int k = 0; k < need; ++k)
                if (!((R >> tg[k]) & 1)) {
                    R |= uint64_t(1) << tg[k];
                    ++cnt;
                }
        }
        for (int q = 0; q < n && cnt < m; ++q)
            if (!((R >> q) & 1)) {
                R |= uint64_t(1) << q;
                ++cnt;
            }
        c.push_back(R);
        const int w = m - L;
        for (int a = L; a + w <= n; ++a) {
            const uint64_t Rw = ((uint64_t(1) << L) - 1) | (((uint64_t(1) << w) - 1) << a);
            if (Rw != R) c.push_back(Rw);
        }
        return c;
    };
    // the greedy rule: the candidate that executes the most non-diagonal gates (then the most gates)
    auto greedy = [&](const std::vector<char> &dn) {
        const std::vector<uint64_t> c = candidates(dn);
        uint64_t R = c[0];
        std::pair<int, int> best = executable(dn, R, nullptr);
        for (size_t k = 1; k < c.size(); ++k) {
            const std::pair<int, int> e = executable(dn, c[k], nullptr);
            if (e > best) {
                best = e;
                R = c[k];
            }
        }
        return R;
    };
    // Passes are costed mostly per pass (each moves the whole state through HBM once), so the schedule
    // wants few of them. The greedy rule fills each pass, but a pass that leaves the frontier of
    // neighbouring-qubit circuits ragged costs later passes. A beam search over the candidate sequences
    // (states ranked by the non-diagonal gates run so far, the best `width` kept per depth, equal gate
    // sets merged) replaces the greedy sequence where it finishes in fewer passes. Its work is bounded
    // by a budget of gate visits; a circuit too large for it keeps the greedy sequence.
    std::vector<uint64_t> chosen;  // resident set of each pass, empty: decide greedily pass by pass
    if (search_width > 1 && G > 0) {
        std::vector<char> dn(G, 0);
        std::vector<uint64_t> gseq;
        size_t left = G;
        while (left > 0) {
            const uint64_t R = greedy(dn);
            std::vector<size_t> take;
            executable(dn, R, &take);
            if (take.empty()) break;
            for (size_t i : take) dn[i] = 1;
            left -= take.size();
            gseq.push_back(R);
        }
        const double ncand = double(std::max(1, n - (m - L) - L + 2));
        const double per_width = double(gseq.size()) * ncand * double(G);
        const int width = int(std::min<double>(search_width, 4.0e8 / std::max(1.0, per_width)));
        if (left == 0 && gseq.size() > 1 && width > 1) {
            struct St {
                std::vector<char> dn;
                int dense, all;
                std::vector<uint64_t> seq;
            };
            std::vector<St> level(1, St{std::vector<char>(G, 0), 0, 0, {}});
            std::vector<uint64_t> found;
            for (size_t depth = 1; depth < gseq.size() && found.empty(); ++depth) {
                std::set<std::vector<char>> seen;
                std::vector<St> next;
                for (const St &s : level) {
                    for (uint64_t R : candidates(s.dn)) {
                        std::vector<size_t> take;
                        const std::pair<int, int> e = executable(s.dn, R, &take);
                        if (take.empty()) continue;
                        St t{s.dn, s.dense + e.first, s.all + e.second, s.seq};
                        for (size_t i : take) t.dn[i] = 1;
                        t.seq.push_back(R);
                        if (!seen.insert(t.dn).second) continue;  // the same gates done: the first sequence stays
                        if (size_t(t.all) == G && found.empty()) found = t.seq;
                        next.push_back(std::move(t));
                    }
                }
                std::stable_sort(next.begin(), next.end(), [](const St &a, const St &b) {
                    return a.dense != b.dense ? a.dense > b.dense : a.all > b.all;
                });
                if (next.size() > size_t(width)) next.resize(size_t(width));
                level.swap(next);
            }
            if (!found.empty() && found.size() < gseq.size()) chosen = found;
        }
    }
    size_t npass = 0;
    while (ndone < G) {
        uint64_t R = npass < chosen.size() ? chosen[npass] : greedy(done);
        ++npass;
        SPass ps{};
        ps.m = m;
        int localof[64];
        for (int q = 0, s = 0; q < 64; ++q) {
            localof[q] = -1;
            if (q < n && ((R >> q) & 1)) {
                ps.R[s] = uint8_t(q);
                localof[q] = s++;
            }
        }
        auto local_mask = [&](uint64_t phys) {
            uint32_t lm = 0;
            for (int q = 0; q < n; ++q)
                if (((phys >> q) & 1) && localof[q] >= 0) lm |= 1u << localof[q];
            return lm;
        };
        // --- executable gates, in circuit order
        std::vector<size_t> take;
        executable(done, R, &take);
        // --- stages: a stage holds dense ops on at most log_e distinct resident targets (its
        // register bits) and diagonal ops on any qubits; a quantum swap ends it
        ps.stage_begin = int(stages.size());
        auto make_hop = [&](const GInfo &g) {
            HOp h{};
            h.target = g.target;
            h.controls = g.controls;
            h.qmask = g.qmask;
            h.gcm = g.controls & ~R;
            h.lcm = local_mask(g.controls);
            h.angles = g.angles;
            h.theta[0] = g.theta[0];
            h.theta[1] = g.theta[1];
            if (diagonal(g)) {
                h.dense = false;
                if (g.kind == G_PHASE) {  // diag(1, c)
                    h.m[0] = 1.0;
                    h.m[1] = 0.0;
                    h.m[2] = g.m[0];
                    h.m[3] = g.m[1];
                } else {
                    memcpy(h.m, g.m, 4 * sizeof(double));
                }
            } else {
                // dense or X on a resident target (X runs as the 2x2 [[0,1],[1,0]]: products with
                // exact 0/1 coefficients)
                h.dense = true;
                h.lb = localof[g.target];
                memcpy(h.m, g.m, sizeof(h.m));
            }
            return h;
        };
        bool has_swap = false;
        for (size_t i : take) has_swap = has_swap || gi[i].kind == G_SWAP;
        if (has_swap) {
            // circuit order: a stage closes at a fifth register bit or at a quantum swap
            std::vector<HOp> sops;
            SStage cur{};
            cur.swap_p = cur.swap_q = -1;
            uint32_t rbset = 0;
            int nrb = 0;
            auto close_stage = [&]() {
                emit_stage(cur, rbset, log_e, m, dtype, localof, ps.R, sops, stages, rounds, ops, blks);
                sops.clear();
                cur = SStage{};
                cur.swap_p = cur.swap_q = -1;
                rbset = 0;
                nrb = 0;
            };
            for (size_t i : take) {
                const GInfo &g = gi[i];
                if (g.kind == G_SWAP) {
                    cur.swap_p = localof[g.target];
                    cur.swap_q = localof[g.target2];
                    cur.swap_lcm = local_mask(g.controls);
                    cur.swap_gcm = g.controls & ~R;
                    close_stage();
                    continue;
                }
                const HOp h = make_hop(g);
                if (h.dense && !((rbset >> h.lb) & 1)) {
                    if (nrb == log_e) close_stage();
                    rbset |= 1u << h.lb;
                    ++nrb;
                }
                sops.push_back(h);
            }
            if (!sops.empty() || int(stages.size()) == ps.stage_begin) close_stage();
        } else {
            // Stages in dependency order, each on the register-bit set S that runs the most dense ops:
            // the first log_e distinct targets in circuit order, or a window of log_e consecutive
            // local bits (on neighbour-coupled circuits a stage then runs a light cone of several
            // layers on its qubits, and the block goes through LDS fewer times). Within the pass the
            // same rule as for passes holds: an op runs when no earlier op left behind holds one of
            // its qubits, and it is diagonal or its target is in S.
            std::vector<size_t> rem(take);
            auto stage_take = [&](uint32_t S, std::vector<size_t> *sel, std::vector<size_t> *rest) {
                int dense = 0, all = 0;
                uint64_t blocked = 0;
                for (size_t i : rem) {
                    const GInfo &g = gi[i];
                    bool ok = !(g.qmask & blocked) && (diagonal(g) || ((S >> localof[g.target]) & 1));
                    if (ok) {
                        ++all;
                        if (!diagonal(g)) ++dense;
                        if (sel) sel->push_back(i);
                    } else {
                        blocked |= g.qmask;
                        if (rest) rest->push_back(i);
                    }
                }
                return std::make_pair(dense, all);
            };
            while (!rem.empty()) {
                uint32_t S = 0;
                int ns = 0;
                for (size_t i : rem) {
                    const GInfo &g = gi[i];
                    if (diagonal(g) || ((S >> localof[g.target]) & 1)) continue;
                    if (ns == log_e) break;
                    S |= 1u << localof[g.target];
                    ++ns;
                }
                std::pair<int, int> best = stage_take(S, nullptr, nullptr);
                for (int a = 0; a + log_e <= m; ++a) {
                    const uint32_t Sw = ((1u << log_e) - 1) << a;
                    const std::pair<int, int> c = stage_take(Sw, nullptr, nullptr);
                    if (c.first > best.first || (c.first == best.first && c.second > best.second)) {
                        best = c;
                        S = Sw;
                    }
                }
                std::vector<size_t> sel, rest;
                stage_take(S, &sel, &rest);
                if (sel.empty()) return set_error(QSIM_EINVAL, "staged: stage scheduler made no progress");
                std::vector<HOp> sops;
                uint32_t rbset = 0;
                for (size_t i : sel) {
                    const HOp h = make_hop(gi[i]);
                    if (h.dense) rbset |= 1u << h.lb;
                    sops.push_back(h);
                }
                SStage cur{};
                cur.swap_p = cur.swap_q = -1;
                emit_stage(cur, rbset, log_e, m, dtype, localof, ps.R, sops, stages, rounds, ops, blks);
                rem.swap(rest);
            }
        }
        ps.stage_end = int(stages.size());
        // direct memory access for the first / last stage when its register bits avoid the low run
        auto low_free = [&](const SStage &st) {
            for (int j = 0; j < log_e; ++j)
                if (st.rb[j] < L) return false;
            return true;
        };
        ps.direct = 0;
        if (low_free(stages[size_t(ps.stage_begin)])) ps.direct |= 1;
        if (low_free(stages[size_t(ps.stage_end - 1)]) && stages[size_t(ps.stage_end - 1)].swap_p < 0) ps.direct |= 2;
        if (half_variant(dtype, log_e, m - log_e)) assign_half(ps, stages, m, log_e, dtype);
        passes.push_back(ps);
        for (size_t i : take) done[i] = 1;
        ndone += take.size();
        if (take.empty()) return set_error(QSIM_EINVAL, "staged: scheduler made no progress");
    }

    return QSIM_OK;
}

int staged_build(int n, int dtype, const std::vector<qsim_gate> &gates, int lds_qubits, int lds_regs, StagedPlan **out,
                 qsim_plan_info *info)
{
    *out = nullptr;
    // defaults measured on the 30-qubit brickwork: 4096 amplitudes per block, 16 per thread
    const int log_e = lds_regs ? lds_regs : 4;
    int m = lds_qubits ? lds_qubits : 12;
    if (!staged_variant_ok(dtype, log_e, m - log_e))
        return set_error(QSIM_EINVAL, "staged: lds_qubits / lds_regs combination not available for this dtype");
    if (n < m) return set_error(QSIM_EUNSUPPORTED, "staged: the state is smaller than one LDS block");
    const int log_t = m - log_e;

    std::vector<SPass> passes;
    std::vector<SStage> stages;
    std::vector<SRound> rounds;
    std::vector<SOp> ops;
    std::vector<SBlk> blks;
    // renormalisation points cut the gate list into segments, each scheduled on its own (a point is a
    // pass boundary); the segments' passes follow each other in the tables
    std::vector<std::vector<qsim_gate>> segs(1);
    for (const qsim_gate &g : gates) {
        if (g.op == QSIM_OP_RENORM) segs.emplace_back();
        else segs.back().push_back(g);
    }
    const int R = int(segs.size()) - 1;
    std::vector<int> seg_first(segs.size()), seg_end(segs.size());
    for (size_t k = 0; k < segs.size(); ++k) {
        seg_first[k] = int(passes.size());
        if (!segs[k].empty())
            if (int rc = staged_schedule(n, dtype, m, log_e, segs[k], passes, stages, rounds, ops, blks, kPassSearchWidth)) return rc;
        seg_end[k] = int(passes.size());
    }
    StagedPlan *p = new StagedPlan();
    p->n = n;
    p->dtype = dtype;
    p->m = m;
    p->log_e = log_e;
    p->log_t = log_t;
    p->passes = passes;
    p->renorms = R;
    // Launch order. Point k takes its norm from the last pass of the segment before it and gives its
    // factor to the first pass of the segment after it; an empty segment before it means a norm sweep
    // (after any factor still owed), and a point with no pass after it ends in a scaling sweep.
    p->scale_of.assign(passes.size(), -1);
    p->norm_of.assign(passes.size(), -1);
    int owed = -1;  // the point whose factor the state has not received yet
    bool norm_in_pass = false;
    for (size_t k = 0; k < segs.size(); ++k) {
        const bool point_after = int(k) < R;
        if (seg_end[k] > seg_first[k]) {
            if (owed >= 0) p->scale_of[size_t(seg_first[k])] = owed;
            owed = -1;
            for (int i = seg_first[k]; i < seg_end[k]; ++i) p->acts.push_back(StagedAct{kActPass, i});
            if (point_after) {
                p->norm_of[size_t(seg_end[k] - 1)] = int(k);
                norm_in_pass = true;
                owed = int(k);
            }
        } else if (point_after) {
            if (owed >= 0) p->acts.push_back(StagedAct{kActScale, owed});
            p->acts.push_back(StagedAct{kActNorm, int(k)});
            owed = int(k);
        }
    }
    if (owed >= 0) p->acts.push_back(StagedAct{kActScale, owed});
    // one device copy of each pass record, of the stage table and of the op table
    hipError_t e = hipMalloc(&p->d_passes, sizeof(SPass) * std::max<size_t>(1, passes.size()));
    if (e == hipSuccess && R > 0) {
        p->aux_l2 = (size_t(R) + 31) / 32 * 32;
        p->aux_part = p->aux_l2 + kAuxLevel2;
        const size_t words = p->aux_part + (norm_in_pass ? size_t(dim(n - m)) : 0);
        e = hipMalloc(&p->d_aux, sizeof(double) * words);
        if (e == hipSuccess) e = hipMemset(p->d_aux, 0, sizeof(double) * words);
        if (e == hipSuccess) e = hipDeviceSynchronize();  // zeroed before any stream can use the plan
    }
    if (e == hipSuccess) e = hipMalloc(&p->d_stages, sizeof(SStage) * std::max<size_t>(1, stages.size()));
    if (e == hipSuccess) e = hipMalloc(&p->d_rounds, sizeof(SRound) * std::max<size_t>(1, rounds.size()));
    if (e == hipSuccess) e = hipMalloc(&p->d_ops, sizeof(SOp) * std::max<size_t>(1, ops.size()));
    if (e == hipSuccess) e = hipMalloc(&p->d_blks, sizeof(SBlk) * std::max<size_t>(1, blks.size()));
    if (e == hipSuccess && !blks.empty()) e = hipMemcpy(p->d_blks, blks.data(), sizeof(SBlk) * blks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !passes.empty())
        e = hipMemcpy(p->d_passes, passes.data(), sizeof(SPass) * passes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !stages.empty())
        e = hipMemcpy(p->d_stages, stages.data(), sizeof(SStage) * stages.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !rounds.empty())
        e = hipMemcpy(p->d_rounds, rounds.data(), sizeof(SRound) * rounds.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ops.empty()) e = hipMemcpy(p->d_ops, ops.data(), sizeof(SOp) * ops.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ops.empty()) {
        hipLaunchKernelGGL(k_op_angles, dim3(unsigned((ops.size() + 255) / 256)), dim3(256), 0, nullptr, p->d_ops, int(ops.size()));
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        staged_free(p);
        return hip_error(e, "staged plan upload");
    }
    info->method = QSIM_PLAN_STAGED;
    info->lds_qubits = m;
    info->lds_regs = log_e;
    // a norm sweep reads the state once, a scaling sweep reads and writes it
    int64_t norm_sweeps = 0, scale_sweeps = 0;
    for (const StagedAct &a : p->acts) {
        norm_sweeps += a.type == kActNorm;
        scale_sweeps += a.type == kActScale;
    }
    info->launches = int64_t(p->acts.size());
    info->passes = int64_t(passes.size()) + scale_sweeps;
    info->alg_bytes = (double(info->passes) * 2.0 + double(norm_sweeps)) * std::ldexp(1.0, n) * amp_bytes(dtype);
    info->alg_flops = 0.0;
    info->renorms = R;
    // vector flops the kernels issue (a multiply counts 1, a multiply-add 2), per thread and block of E
    // amplitudes, times the 2^n / E threads of all blocks: a dense 2x2 with a real first column 20 per
    // pair, a general one 28 per pair it runs on, a two-qubit block 120 per group of four, a phase factor
    // 6 per element it multiplies, a sign flip 0
    {
        const int E = 1 << log_e;
        double per_thread = 0.0;
        for (const SRound &rd : rounds) {
            for (int j = 0; j < log_e; ++j)
                for (int l = 0; l < kLists; ++l)
                    for (int oi = rd.seg[kLists * j + l]; oi < rd.seg[kLists * j + l + 1]; ++oi)
                        per_thread += l == kListCond ? 28.0 * __builtin_popcount(ops[size_t(oi)].pmask) : 20.0 * (E / 2);
            per_thread += 120.0 * (E / 4) * (rd.pseg[npairs(log_e)] - rd.pseg[0]);
            for (int oi = rd.seg[kLists * log_e + 1]; oi < rd.seg[kLists * log_e + 2]; ++oi)
                per_thread += 6.0 * (__builtin_popcount(ops[size_t(oi)].m1) + __builtin_popcount(ops[size_t(oi)].m0));
        }
        info->issued_flops = per_thread * std::ldexp(1.0, n - log_e);
    }
    *out = p;
    return QSIM_OK;
}

// the kernel that runs pass i: the wave-split kernel where every round trip splits at a wave position
// and the block shape has one, the half-buffer kernel where every round trip splits, else the full one
static int pass_variant(const StagedPlan *p, size_t i)
{
    const int v = p->log_e * 16 + p->log_t;
    const int d = p->passes[i].direct;
    if ((d & 12) == 12 && p->dtype == QSIM_C128 && (v == 4 * 16 + 7 || v == 4 * 16 + 8)) return QSIM_STAGED_WAVE;
    if ((d & 12) == 12 && p->dtype == QSIM_C64 && (v == 5 * 16 + 7 || v == 5 * 16 + 8)) return QSIM_STAGED_WAVE;
    return (d & 4) ? QSIM_STAGED_HALF : QSIM_STAGED_FULL;
}

static int launch_pass(StagedPlan *p, qsim_state *s, size_t i, int init_zero, const double *scale, double *norm)
{
    PassLaunch a{};
    a.data = s->data;
    a.pass = p->d_passes + i;
    a.stages = p->d_stages;
    a.rounds = p->d_rounds;
    a.ops = p->d_ops;
    a.blks = p->d_blks;
    a.scale = scale;
    a.norm = norm;
    a.grid = unsigned(dim(p->n - p->m));
    a.stream = s->stream;
    a.mode = init_zero ? 2 : (scale || norm) ? 1 : 0;
    const int form = pass_variant(p, i);
    int rc;
    if (p->dtype == QSIM_C128)
        rc = form == QSIM_STAGED_WAVE ? launch_wave_c128(p->log_e, p->log_t, a) : launch_pass_c128(form, p->log_e, p->log_t, a);
    else
        rc = form == QSIM_STAGED_WAVE ? launch_wave_c64(p->log_e, p->log_t, a) : launch_pass_c64(form, p->log_e, p->log_t, a);
    if (rc) return rc;
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

void staged_launch_list(const StagedPlan *p, int32_t *kind, int32_t *variant)
{
    for (size_t i = 0; i < p->acts.size(); ++i) {
        const StagedAct &a = p->acts[i];
        if (kind) kind[i] = a.type == kActPass ? QSIM_KERNEL_STAGED : QSIM_KERNEL_RENORM;
        if (variant) variant[i] = a.type == kActPass ? pass_variant(p, size_t(a.index)) : 0;
    }
}

double *staged_norms(StagedPlan *p) { return p->d_aux; }

// One launch of the plan. A pass that ends before a renormalisation point also sums its per-block
// partials into the point's squared norm (part of the same launch step).
static int run_act(StagedPlan *p, qsim_state *s, const StagedAct &a, bool init_zero)
{
    if (a.type == kActNorm) return launch_norm_into(s, p->d_aux + p->aux_l2, p->d_aux + a.index);
    if (a.type == kActScale) return launch_renorm_scale(s, p->d_aux + a.index);
    const size_t i = size_t(a.index);
    const double *scale = p->scale_of[i] >= 0 ? p->d_aux + p->scale_of[i] : nullptr;
    double *norm = p->norm_of[i] >= 0 ? p->d_aux + p->aux_part : nullptr;
    if (int rc = launch_pass(p, s, i, init_zero, scale, norm)) return rc;
    if (norm) return launch_sum_array(norm, dim(p->n - p->m), p->d_aux + p->aux_l2, p->d_aux + p->norm_of[i], s->stream);
    return QSIM_OK;
}

// from_zero: the first pass generates |0...0> in its loads instead of reading the state (a plan that
// does not start with a pass writes |0...0> first)
static bool zero_in_first_pass(const StagedPlan *p, bool from_zero)
{
    return from_zero && !p->acts.empty() && p->acts[0].type == kActPass;
}

int staged_execute(StagedPlan *p, qsim_state *s, bool from_zero)
{
    const bool zf = zero_in_first_pass(p, from_zero);
    if (from_zero && !zf)
        if (int rc = launch_set_basis(s, 0)) return rc;
    for (size_t i = 0; i < p->acts.size(); ++i)
        if (int rc = run_act(p, s, p->acts[i], zf && i == 0)) return rc;
    return QSIM_OK;
}

int staged_execute_timed(StagedPlan *p, qsim_state *s, bool from_zero, double *ms, int32_t *kind, int32_t *fk)
{
    const bool zf = zero_in_first_pass(p, from_zero);
    if (from_zero && !zf)
        if (int rc = launch_set_basis(s, 0)) return rc;
    const size_t L = p->acts.size();
    std::vector<hipEvent_t> ev(2 * L, nullptr);
    for (auto &e : ev) QSIM_HIP(hipEventCreate(&e));
    int rc = QSIM_OK;
    for (size_t i = 0; i < L && !rc; ++i) {
        QSIM_HIP(hipEventRecord(ev[2 * i], s->stream));
        rc = run_act(p, s, p->acts[i], zf && i == 0);
        QSIM_HIP(hipEventRecord(ev[2 * i + 1], s->stream));
    }
    if (!rc) {
        QSIM_HIP(hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < L; ++i) {
            float tms = 0.f;
            QSIM_HIP(hipEventElapsedTime(&tms, ev[2 * i], ev[2 * i + 1]));
            if (ms) ms[i] = tms;
            if (fk) fk[i] = 0;
        }
        staged_launch_list(p, kind, nullptr);
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return rc;
}

void staged_free(StagedPlan *p)
{
    if (!p) return;
    if (p->d_passes) (void)hipFree(p->d_passes);
    if (p->d_stages) (void)hipFree(p->d_stages);
    if (p->d_rounds) (void)hipFree(p->d_rounds);
    if (p->d_ops) (void)hipFree(p->d_ops);
    if (p->d_blks) (void)hipFree(p->d_blks);
    if (p->d_aux) (void)hipFree(p->d_aux);
    delete p;
}

}  // namespace qsim
