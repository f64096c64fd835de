// Program-specialised free-run and lockstep replay kernels.
//
// A KC-IR program is translated into HIP source in which every basic block is
// straight-line code: the simulated registers are variables (real VGPRs, no
// indexed register file), operands and special-register numbers are
// constants, and a converged wave moves between blocks with direct jumps.
// Only a divergent wave goes back to the smallest-pc dispatch.  Everything
// else -- block set-up, access logging, the epoch-local check, barrier
// episodes, deadlock and divergence findings, block publication -- is the
// interpreter's own device code (kc_device.h), compiled into the same kernel,
// so a specialised kernel produces exactly the records, findings and memory
// of the interpreter's free run.
//
// Fuel: each basic block of length n runs without per-instruction checks when
// every live lane of the wave holds at least n units (a wave-uniform lower
// bound is kept); otherwise its instructions check and spend fuel one by one.
//
// The source is compiled with hiprtc for gfx950 by the first launch that needs
// it (the programs of one stage in parallel, on threads joined before the
// launch: no compilation outlives the call, so none can be cut short by the
// process exiting); the code is cached per process by program text and the
// module loaded once per device.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "kc_internal.h"
#include "kc_jit.h"

namespace kc {

namespace {
#include "kc_jit_src.inc"   // kc_jit_internal_h, kc_jit_device_h: text of the two device headers

struct Instr {
    uint32_t op, d, a, b;
    int32_t imm;
};

Instr decode(uint64_t w) {
    return Instr{(uint32_t)(w & 0xFF), (uint32_t)((w >> 8) & 0xFF), (uint32_t)((w >> 16) & 0xFF),
                 (uint32_t)((w >> 24) & 0xFF), (int32_t)(uint32_t)(w >> 32)};
}

std::string reg(uint32_t r) { return "r" + std::to_string(r); }
std::string lit(int32_t v) {
    if (v == INT32_MIN) return "(-2147483647 - 1)";
    return "(" + std::to_string(v) + ")";
}

// Spend fuel one instruction at a time (slow copy of a block).
const char *kSlowFuel =
    "        {\n"
    "            const bool nofuel = act && t.fuel == 0u;\n"
    "            if (__ballot(nofuel)) {\n"
    "                emit_fault(nofuel, A, B, F_FUEL, epoch, 0, B.tid, 0, 0);\n"
    "                if (nofuel) { t.st = ST_EXIT; act = false; }\n"
    "                if (__ballot(act) == 0) continue;\n"
    "            }\n"
    "            if (act) t.fuel--;\n"
    "        }\n";

void gen_alu(std::ostringstream &o, const Instr &I, uint32_t pc) {
    const uint32_t base = I.op & ~uint32_t(OP_IMM);
    const std::string x = reg(I.a);
    const std::string y = (I.op & OP_IMM) ? lit(I.imm) : reg(I.b);
    const std::string d = reg(I.d);
    o << "        {\n            const int32_t x = " << x << ", y = " << y << ";\n";
    o << "            const uint32_t ux = (uint32_t)x, uy = (uint32_t)y;\n            (void)ux; (void)uy;\n";
    std::string v;
    switch (base) {
    case OP_ADD: v = "(int32_t)(ux + uy)"; break;
    case OP_SUB: v = "(int32_t)(ux - uy)"; break;
    case OP_MUL: v = "(int32_t)(ux * uy)"; break;
    case OP_DIV:
    case OP_REM:
        o << "            emit_fault(act && y == 0, A, B, F_ARITH, epoch, 0, B.tid, " << pc << "u, 0);\n";
        o << "            const int32_t ys = (y == 0 || y == -1) ? 1 : y;\n";
        v = base == OP_DIV ? "(y == 0 ? 0 : (y == -1 ? (int32_t)(0u - ux) : x / ys))"
                           : "((y == 0 || y == -1) ? 0 : x % ys)";
        break;
    case OP_AND: v = "(x & y)"; break;
    case OP_OR: v = "(x | y)"; break;
    case OP_XOR: v = "(x ^ y)"; break;
    case OP_SHL: v = "(int32_t)(ux << (uy & 31u))"; break;
    case OP_SHRA: v = "(x >> (int)(uy & 31u))"; break;
    case OP_SHRL: v = "(int32_t)(ux >> (uy & 31u))"; break;
    case OP_MIN: v = "min(x, y)"; break;
    case OP_MAX: v = "max(x, y)"; break;
    case OP_SLT: v = "(x < y ? 1 : 0)"; break;
    case OP_SLE: v = "(x <= y ? 1 : 0)"; break;
    case OP_SEQ: v = "(x == y ? 1 : 0)"; break;
    case OP_SNE: v = "(x != y ? 1 : 0)"; break;
    case OP_SLTU: v = "(ux < uy ? 1 : 0)"; break;
    default: v = "0"; break;
    }
    o << "            const int32_t v = " << v << ";\n            if (act) " << d << " = v;\n        }\n";
}

// A load or store; in lockstep mode a store is held in P until the step's
// stores land.
void gen_mem(std::ostringstream &o, const Instr &I, uint32_t pc, bool lockstep = false) {
    const bool sh = (I.op & 2u) == 0, st = (I.op & 1u) != 0;
    const char *lim = sh ? "B.sh_words" : "B.n_words";
    const char *arr = sh ? "S.sh" : "B.mem";
    o << "        {\n            const int32_t addr = (int32_t)((uint32_t)" << reg(I.a) << " + (uint32_t)" << lit(I.imm)
      << ");\n";
    o << "            const bool inb = act && (uint32_t)addr < " << lim << ";\n";
    if (st && lockstep) {
        o << "            if (inb) {\n                P.on = true;\n                P.shared = " << (sh ? "true" : "false")
          << ";\n                P.addr = addr;\n                P.val = " << reg(I.b) << ";\n            }\n";
    } else if (st) {
        o << "            if (inb) " << arr << "[addr] = " << reg(I.b) << ";\n";
    } else {
        o << "            int32_t v = 0;\n            if (inb) v = " << arr << "[addr];\n";
        o << "            if (act) " << reg(I.d) << " = v;\n";
    }
    if (sh && !st)
        o << "            if (A.uninit) emit_fault(inb && !shared_stored(S, (uint32_t)addr), A, B, F_UNINIT, epoch, 0u, "
             "B.tid, (uint32_t)addr, " << pc << "u);\n";
    if (sh && st && !lockstep) o << "            if (A.uninit && inb) mark_stored(S, (uint32_t)addr);\n";
    if (lockstep)
        o << "            if (A.wlog) wlog_append(A, B, inb, " << (sh ? "0u" : "1u") << ", (uint32_t)addr, "
          << (st ? "true" : "false") << ");\n";
    if (sh) {
        o << "            if (LOCAL) {\n";
        if (lockstep)
            o << "                if (inb) shadow_update(S.shadow, (uint32_t)addr, B.tid, " << (st ? "true" : "false")
              << ");\n";
        else
            o << "                if (inb) shadow_mark(S, (uint32_t)addr, B.tid, " << (st ? "true" : "false") << ");\n";
        o << "                L.total += (uint32_t)__popcll(__ballot(inb));\n            } else {\n    ";
    }
    const std::string key = std::string("B.kep | ((uint64_t)") + (sh ? "0" : "1") + "u << A.kp.s_sp) | " +
                            (st ? "1ull" : "0ull") + " | ((uint64_t)(uint32_t)addr << A.kp.s_addr)";
    if (sh) {
        o << "            log_rec(A, S.stage, L, inb, " << key << ");\n            }\n";
    } else {
        o << "            L.gtotal += (uint32_t)__popcll(__ballot(inb));\n";
        o << "            if (LOCAL) global_access(A, B, S, L, inb, (uint32_t)addr, " << (st ? "true" : "false") << ", "
          << key << ");\n";
        o << "            else log_rec(A, S.stage, L, inb, " << key << ");\n";
    }
    o << "            emit_fault(act && !inb, A, B, F_OOB, epoch, " << ((sh ? 0 : 2) + (st ? 1 : 0))
      << "u, B.tid, (uint32_t)addr, 0);\n        }\n";
}

}  // namespace

// A thread arriving at the barrier at `pc` (plain or with a predicate).
std::string arrive(const Instr &I, uint32_t pc, const char *indent) {
    std::ostringstream o;
    o << indent << "if (act) {\n" << indent << "    t.st = ST_WAIT;\n" << indent << "    t.bar_pc = " << pc << ";\n";
    if (I.op == OP_BARP)
        o << indent << "    t.bpred = " << ((I.imm + 1) << 1) << " | (" << reg(I.a) << " != 0 ? 1 : 0);\n";
    else
        o << indent << "    t.bpred = 0;\n";
    o << indent << "}\n";
    return o.str();
}

// After a release: the result of each barrier with a predicate goes to its
// destination register, for the lanes released from that barrier.
std::string barrier_results(const uint64_t *words, uint32_t n, const char *indent) {
    std::ostringstream o;
    bool any = false;
    for (uint32_t pc = 0; pc < n; pc++) any = any || decode(words[pc]).op == OP_BARP;
    if (!any) return "";
    o << indent << "if (__ballot(t.bpred != 0)) {\n";
    for (uint32_t pc = 0; pc < n; pc++) {
        const Instr I = decode(words[pc]);
        if (I.op == OP_BARP)
            o << indent << "    if (t.bpred != 0 && t.bar_pc == " << pc << ") " << reg(I.d) << " = t.bres;\n";
    }
    o << indent << "    t.bpred = 0;\n" << indent << "}\n";
    return o.str();
}

std::string jit_source(const uint64_t *words, uint32_t n, int waves) {
    std::vector<char> lead(n + 1, 0);
    lead[0] = 1;
    lead[n] = 1;
    for (uint32_t pc = 0; pc < n; pc++) {
        const Instr I = decode(words[pc]);
        if (I.op == OP_JMP || I.op == OP_BZ || I.op == OP_BNZ) {
            lead[(uint32_t)I.imm] = 1;
            lead[pc + 1] = 1;
        } else if (I.op == OP_BAR || I.op == OP_BARP || I.op == OP_EXIT) {
            lead[pc + 1] = 1;
        }
    }
    std::vector<uint32_t> starts;
    for (uint32_t pc = 0; pc < n; pc++)
        if (lead[pc]) starts.push_back(pc);

    std::ostringstream o;
    o << "#include \"kc_internal.h\"\n#include \"kc_device.h\"\n\nnamespace kc {\nnamespace {\n\n";
    o << "template <bool LOCAL>\n__device__ __forceinline__ uint32_t jit_run(const InterpArgs &A, BlockCtx &B, "
         "const Shared &S, Lane &t, LogState &L) {\n";
    o << "    uint32_t epoch = 0;\n";
    for (uint32_t r = 0; r < 16; r++) o << "    int32_t r" << r << " = 0;\n";
    o << "    bool conv = true;\n    int upc = 0;\n    uint32_t guard = B.u->fuel;\n";
    o << "    for (;;) {\n      for (;;) {\n";
    // the scheduling state is wave-uniform: reading it through lane 0 keeps
    // the branches on it scalar
    o << "        conv = uni(conv ? 1 : 0) != 0;\n        upc = uni(upc);\n        guard = uniu(guard);\n";
    o << "        const uint64_t runm = __ballot(t.st == ST_RUN);\n        if (runm == 0) break;\n";
    o << "        int cur;\n        bool act;\n";
    o << "        if (conv) {\n            cur = upc;\n            act = t.st == ST_RUN;\n        } else {\n";
    o << "            cur = uni(wave_min(t.st == ST_RUN ? t.pc : INT_MAX));\n";
    o << "            act = t.st == ST_RUN && t.pc == cur;\n";
    o << "            if (__ballot(act) == runm) { conv = true; upc = cur; }\n        }\n";
    // One case per basic block; every block ends by naming the next pc
    // (upc when converged, t.pc per lane otherwise) and returning to the
    // dispatch, so the control flow stays reducible.
    o << "        switch (cur) {\n";
    auto next = [&](const std::string &pc) {
        o << "            if (conv) upc = " << pc << ";\n            else if (act) t.pc = " << pc << ";\n"
          << "            break;\n";
    };
    for (size_t bi = 0; bi < starts.size(); bi++) {
        const uint32_t s = starts[bi];
        uint32_t e = s + 1;
        while (e < n && !lead[e]) e++;
        const uint32_t len = e - s;
        o << "        case " << s << ": {\n";
        auto body = [&](bool checks) {
            for (uint32_t pc = s; pc < e; pc++) {
                const Instr I = decode(words[pc]);
                o << "        // pc " << pc << "\n";
                if (checks) o << kSlowFuel;
                const uint32_t base = I.op & ~uint32_t(OP_IMM);
                if (base >= OP_ADD && base <= OP_SLTU) {
                    gen_alu(o, I, pc);
                } else if ((I.op >> 4) == 5) {
                    gen_mem(o, I, pc);
                } else if (I.op == OP_MOV) {
                    o << "        if (act) " << reg(I.d) << " = " << reg(I.a) << ";\n";
                } else if (I.op == OP_MOVI) {
                    o << "        if (act) " << reg(I.d) << " = " << lit(I.imm) << ";\n";
                } else if (I.op == OP_SREG) {
                    o << "        if (act) " << reg(I.d) << " = special(B, " << (uint32_t)I.imm << "u);\n";
                }
            }
        };
        // fast copy: every live lane holds fuel for the whole block; slow
        // copy: fuel checked and spent per instruction
        o << "        const bool fast = guard >= " << len << "u;\n";
        o << "        if (fast) {\n            guard -= " << len << "u;\n            if (act) t.fuel -= " << len << "u;\n";
        body(false);
        o << "        } else {\n";
        body(true);
        o << "            guard = uniu(wave_min_u((t.st == ST_RUN || t.st == ST_WAIT) ? t.fuel : 0xFFFFFFFFu));\n";
        o << "        }\n";
        const Instr T = decode(words[e - 1]);
        if (T.op == OP_JMP) {
            next(std::to_string(T.imm));
        } else if (T.op == OP_BZ || T.op == OP_BNZ) {
            o << "            const bool c = act && (" << reg(T.a) << (T.op == OP_BZ ? " == 0" : " != 0") << ");\n";
            o << "            const uint64_t am = __ballot(act), tk = __ballot(c);\n";
            o << "            if (conv && tk != 0 && tk != am) conv = false;\n";
            o << "            if (conv) upc = tk ? " << T.imm << " : " << e << ";\n";
            o << "            else if (act) t.pc = c ? " << T.imm << " : " << e << ";\n            break;\n";
        } else if (T.op == OP_BAR || T.op == OP_BARP) {
            o << arrive(T, e - 1, "            ") << "            break;\n";
        } else if (T.op == OP_EXIT) {
            o << "            if (act) t.st = ST_EXIT;\n            break;\n";
        } else {
            next(std::to_string(e));
        }
        o << "        }\n";
    }
    o << "        default:\n            if (act) t.st = ST_EXIT;\n            break;\n        }\n";
    o << "      }\n";
    o << "      if (free_episode<LOCAL>(A, B, S, t, L, epoch) == EP_DONE) break;\n";
    o << barrier_results(words, n, "      ");
    o << "      free_reconverge(t, conv, upc);\n    }\n    return epoch;\n}\n\n";
    // Lockstep replay: the interpreter's round protocol with one specialised
    // case per instruction.
    o << "template <bool LOCAL>\n__device__ __forceinline__ uint32_t jit_lock_run(const InterpArgs &A, BlockCtx &B, "
         "const Shared &S, const StoreTables &T, Lane &t, LogState &L) {\n";
    for (uint32_t r = 0; r < 16; r++) o << "    int32_t r" << r << " = 0;\n";
    o << "    auto exec = [&](int cur, uint64_t, bool act, Pending &P, uint32_t epoch, int &ctl, int &target, "
         "bool &cond) {\n";
    o << "        ctl = 0;\n        target = cur + 1;\n        cond = false;\n        (void)P;\n";
    o << "        switch (cur) {\n";
    for (uint32_t pc = 0; pc < n; pc++) {
        const Instr I = decode(words[pc]);
        const uint32_t base = I.op & ~uint32_t(OP_IMM);
        o << "        case " << pc << ": {\n";
        if (base >= OP_ADD && base <= OP_SLTU) {
            gen_alu(o, I, pc);
        } else if ((I.op >> 4) == 5) {
            gen_mem(o, I, pc, true);
        } else if (I.op == OP_MOV) {
            o << "        if (act) " << reg(I.d) << " = " << reg(I.a) << ";\n";
        } else if (I.op == OP_MOVI) {
            o << "        if (act) " << reg(I.d) << " = " << lit(I.imm) << ";\n";
        } else if (I.op == OP_SREG) {
            o << "        if (act) " << reg(I.d) << " = special(B, " << (uint32_t)I.imm << "u);\n";
        } else if (I.op == OP_JMP) {
            o << "        ctl = 1;\n        target = " << I.imm << ";\n";
        } else if (I.op == OP_BZ || I.op == OP_BNZ) {
            o << "        ctl = 2;\n        target = " << I.imm << ";\n        cond = " << reg(I.a)
              << (I.op == OP_BZ ? " == 0" : " != 0") << ";\n";
        } else if (I.op == OP_BAR || I.op == OP_BARP) {
            o << "        ctl = 3;\n" << arrive(I, pc, "        ");
        } else if (I.op == OP_EXIT) {
            o << "        ctl = 3;\n        if (act) t.st = ST_EXIT;\n";
        }
        o << "        } break;\n";
    }
    o << "        default: break;\n        }\n    };\n";
    // Converged memory-free runs: straight-line segments between loads and
    // stores, one step per instruction.
    std::vector<char> lead2(lead);
    for (uint32_t pc = 0; pc < n; pc++)
        if ((decode(words[pc]).op >> 4) == 5) lead2[pc] = lead2[pc + 1] = 1;
    o << "    auto run = [&](uint64_t todo, uint32_t epoch) -> uint32_t {\n";
    o << "        const bool act = (todo >> lane_id()) & 1ull;\n";
    o << "        int upc = uni(__builtin_amdgcn_readlane(t.pc, (int)((uint32_t)__ffsll((long long)todo) - 1u)));\n";
    o << "        if (__ballot(act && t.pc != upc)) return 0u;\n";
    o << "        uint32_t fmin = uniu(wave_min_u(act ? t.fuel : 0xFFFFFFFFu));\n";
    o << "        uint32_t steps = 0;\n        (void)epoch;\n";
    o << "        for (;;) {\n            upc = uni(upc);\n            fmin = uniu(fmin);\n            switch (upc) {\n";
    for (uint32_t s0 = 0; s0 < n; s0++) {
        if (!lead2[s0] || (decode(words[s0]).op >> 4) == 5) continue;
        uint32_t e = s0 + 1;
        while (e < n && !lead2[e]) e++;
        const uint32_t len = e - s0;
        o << "            case " << s0 << ": {\n";
        o << "                if (fmin < " << len << "u) goto out;\n";
        o << "                fmin -= " << len << "u;\n                if (act) t.fuel -= " << len << "u;\n";
        o << "                steps += " << len << "u;\n";
        for (uint32_t pc = s0; pc < e; pc++) {
            const Instr I = decode(words[pc]);
            const uint32_t base = I.op & ~uint32_t(OP_IMM);
            if (base >= OP_ADD && base <= OP_SLTU) {
                gen_alu(o, I, pc);
            } else if (I.op == OP_MOV) {
                o << "        if (act) " << reg(I.d) << " = " << reg(I.a) << ";\n";
            } else if (I.op == OP_MOVI) {
                o << "        if (act) " << reg(I.d) << " = " << lit(I.imm) << ";\n";
            } else if (I.op == OP_SREG) {
                o << "        if (act) " << reg(I.d) << " = special(B, " << (uint32_t)I.imm << "u);\n";
            }
        }
        const Instr T = decode(words[e - 1]);
        if (T.op == OP_JMP) {
            o << "                upc = " << T.imm << ";\n                continue;\n";
        } else if (T.op == OP_BZ || T.op == OP_BNZ) {
            o << "                const bool c = act && (" << reg(T.a) << (T.op == OP_BZ ? " == 0" : " != 0") << ");\n";
            o << "                const uint64_t am = __ballot(act), tk = __ballot(c);\n";
            o << "                if (tk == 0) { upc = " << e << "; continue; }\n";
            o << "                if (tk == am) { upc = " << T.imm << "; continue; }\n";
            o << "                if (act) t.pc = c ? " << T.imm << " : " << e << ";\n                return steps;\n";
        } else if (T.op == OP_BAR || T.op == OP_BARP) {
            o << arrive(T, e - 1, "                ") << "                return steps;\n";
        } else if (T.op == OP_EXIT) {
            o << "                if (act) t.st = ST_EXIT;\n                return steps;\n";
        } else {
            o << "                upc = " << e << ";\n                continue;\n";
        }
        o << "            }\n";
    }
    o << "            default: goto out;\n            }\n        }\n";
    o << "    out:\n        if (act) t.pc = upc;\n        return steps;\n    };\n";
    o << "    auto release = [&] {\n" << barrier_results(words, n, "        ") << "    };\n";
    // loads and stores as bit masks per 64 pcs (no program fetch)
    {
        const uint32_t chunks = (n + 63) / 64;
        o << "    auto kind = [](int p) -> uint32_t {\n        const uint32_t q = (uint32_t)p;\n";
        for (uint32_t c = 0; c < chunks; c++) {
            uint64_t mem = 0, st = 0;
            for (uint32_t pc = c * 64; pc < std::min(n, c * 64 + 64); pc++) {
                const Instr I = decode(words[pc]);
                if ((I.op >> 4) == 5) {
                    mem |= 1ull << (pc - c * 64);
                    if (I.op & 1u) st |= 1ull << (pc - c * 64);
                }
            }
            o << "        if (q < " << (c + 1) * 64 << "u) { const uint32_t b = q - " << c * 64
              << "u; return ((" << mem << "ull >> b) & 1ull) ? 1u + (uint32_t)((" << st << "ull >> b) & 1ull) : 0u; }\n";
        }
        o << "        return 0u;\n    };\n";
        o << "    auto word = [](int) -> uint64_t { return 0ull; };\n";
    }
    o << "    return run_block_lockstep<LOCAL>(A, B, S, T, t, L, exec, run, release, kind, word);\n}\n\n";
    o << "}  // namespace\n}  // namespace kc\n\n";
    // workgroups of up to 256 threads get the whole register file; larger ones
    // are bounded to 128 VGPRs
    const struct { const char *name; int bound; bool local; } kernels[] = {
        {"kc_jit_free_local_256", 256, true}, {"kc_jit_free_local_1024", 1024, true}, {"kc_jit_free_1024", 1024, false}};
    // the replay's blocks run one per CU, latency bound: workgroups of up to
    // 256 threads get a kernel with the whole register file (no spills)
    for (const char *name : {"kc_jit_lock_local_256", "kc_jit_lock_local", "kc_jit_lock"}) {
        const bool local = std::string(name) != "kc_jit_lock";
        const int bound = std::string(name) == "kc_jit_lock_local_256" ? 256 : 1024;
        o << "extern \"C\" __global__ void __launch_bounds__(" << bound << ") " << name << "(kc::InterpArgs A) {\n";
        o << "    kc::lockstep_body(A, [](const kc::InterpArgs &a, kc::BlockCtx &b, const kc::Shared &s, "
             "const kc::StoreTables &tb, kc::Lane &t, kc::LogState &l) {\n";
        o << "        return kc::jit_lock_run<" << (local ? "true" : "false") << ">(a, b, s, tb, t, l);\n    });\n}\n";
    }
    for (const auto &k : kernels) {
        o << "extern \"C\" __global__ void __launch_bounds__(" << k.bound << ") ";
        if (waves > 0) o << "__attribute__((amdgpu_waves_per_eu(" << waves << ", " << waves << "))) ";
        o << k.name << "(kc::InterpArgs A) {\n";
        o << "    kc::free_block(A, [](const kc::InterpArgs &a, kc::BlockCtx &b, const kc::Shared &s, kc::Lane &t, "
             "kc::LogState &l) {\n";
        o << "        return kc::jit_run<" << (k.local ? "true" : "false") << ">(a, b, s, t, l);\n    });\n}\n";
    }
    return o.str();
}

// ---- compilation and cache -------------------------------------------------------

struct JitEntry {
    std::string words;              // the program
    int waves = 0;                  // occupancy target of the kernels (0: the compiler's choice)
    std::mutex mu;
    std::condition_variable cv;
    int state = 0;                  // 0 not compiled, 2 being compiled, 1 code ready, -1 failed
    std::vector<char> code;
    std::string log;
    double compile_ms = 0.0;
    bool reported = false;          // a failure was printed
    std::map<int, std::pair<hipModule_t, JitFunctions>> loaded;   // per device
};

namespace {

// Process-wide cache, never freed.
struct Globals {
    std::mutex mu;
    std::map<std::string, std::shared_ptr<JitEntry>> cache;
};
Globals &G() {
    static Globals *g = new Globals;
    return *g;
}

}  // namespace

static void jit_compile_body(const std::shared_ptr<JitEntry> &e);

// Compile an entry claimed with jit_claim.  Never throws: a failure of any
// kind leaves the entry failed (state -1) and wakes its waiters.
void jit_compile(const std::shared_ptr<JitEntry> &e) {
    try {
        jit_compile_body(e);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(e->mu);
            e->state = -1;
            e->log = "compilation of the specialised kernels failed (host exception)";
        }
        e->cv.notify_all();
    }
}

static void jit_compile_body(const std::shared_ptr<JitEntry> &e) {
    const auto t0 = std::chrono::steady_clock::now();
    const std::string src = jit_source((const uint64_t *)e->words.data(), (uint32_t)(e->words.size() / 8), e->waves);
    std::vector<char> code;
    std::string log;
    bool ok = false;
    hiprtcProgram prog = nullptr;
    const char *headers[] = {kc_jit_internal_h, kc_jit_device_h};
    const char *names[] = {"kc_internal.h", "kc_device.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "kc_jit.hip", 2, headers, names) == HIPRTC_SUCCESS) {
        const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                              "-Xclang", "-packed-fp32-ops"};
        const hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
        size_t ls = 0;
        if (hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
            log.resize(ls);
            hiprtcGetProgramLog(prog, &log[0]);
        }
        size_t cs = 0;
        if (r == HIPRTC_SUCCESS && hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0) {
            code.resize(cs);
            ok = hiprtcGetCode(prog, code.data()) == HIPRTC_SUCCESS;
        }
        hiprtcDestroyProgram(&prog);
    } else {
        log = "hiprtcCreateProgram failed";
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->code = std::move(code);
        e->log = std::move(log);
        e->compile_ms = ms;
        e->state = ok ? 1 : -1;
    }
    e->cv.notify_all();
}

std::shared_ptr<JitEntry> jit_request(const uint64_t *words, uint32_t n, int waves) {
    std::string key((const char *)words, (size_t)n * 8);
    key.push_back((char)waves);
    std::lock_guard<std::mutex> g(G().mu);
    auto it = G().cache.find(key);
    if (it != G().cache.end()) return it->second;
    auto e = std::make_shared<JitEntry>();
    e->words.assign((const char *)words, (size_t)n * 8);
    e->waves = waves;
    G().cache[key] = e;
    return e;
}

bool jit_claim(const std::shared_ptr<JitEntry> &e) {
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->state != 0) return false;
    e->state = 2;
    return true;
}

bool jit_functions(const std::shared_ptr<JitEntry> &e, int device, bool wait, JitFunctions &out, double *compile_ms) {
    if (!e) return false;
    std::unique_lock<std::mutex> lk(e->mu);
    if (wait) e->cv.wait(lk, [&] { return e->state != 2; });
    if (e->state < 0 && !e->reported) {
        e->reported = true;
        std::fprintf(stderr, "libkc: specialised kernels unavailable, the interpreter runs instead:\n%s\n",
                     e->log.c_str());
    }
    if (e->state != 1) return false;
    auto it = e->loaded.find(device);
    if (it == e->loaded.end()) {
        JitFunctions f{};
        hipModule_t mod = nullptr;
        if (hipModuleLoadData(&mod, e->code.data()) != hipSuccess) {
            (void)hipGetLastError();
            e->state = -1;
            e->log += "\nhipModuleLoadData failed";
            return false;
        }
        if (hipModuleGetFunction(&f.local_256, mod, "kc_jit_free_local_256") != hipSuccess ||
            hipModuleGetFunction(&f.local_1024, mod, "kc_jit_free_local_1024") != hipSuccess ||
            hipModuleGetFunction(&f.free_1024, mod, "kc_jit_free_1024") != hipSuccess ||
            hipModuleGetFunction(&f.lock_local, mod, "kc_jit_lock_local") != hipSuccess ||
            hipModuleGetFunction(&f.lock_local_256, mod, "kc_jit_lock_local_256") != hipSuccess ||
            hipModuleGetFunction(&f.lock, mod, "kc_jit_lock") != hipSuccess) {
            (void)hipGetLastError();
            e->state = -1;
            e->log += "\nhipModuleGetFunction failed";
            return false;
        }
        it = e->loaded.emplace(device, std::make_pair(mod, f)).first;
        if (compile_ms) *compile_ms = e->compile_ms;
    }
    out = it->second.second;
    return true;
}

int jit_state(const std::shared_ptr<JitEntry> &e) {
    if (!e) return -1;
    std::lock_guard<std::mutex> lk(e->mu);
    return e->state;
}

std::string jit_log(const std::shared_ptr<JitEntry> &e) {
    if (!e) return "";
    std::lock_guard<std::mutex> lk(e->mu);
    return e->log;
}

hipError_t launch_jit(const JitFunctions &f, const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads,
                      hipStream_t s) {
    if (n_wg == 0) return hipSuccess;
    InterpArgs args = a;
    args.rep_hold = rep_hold_for(wg_threads);
    if (!args.local) args.gst_bits = 0;
    auto bytes = [&] {
        return interp_lds_bytes(args.sh_words_max, wg_threads, args.stage, false, args.local != 0, args.gst_bits);
    };
    size_t lds = bytes();
    while (lds > 64 * 1024 && args.stage > 64) {
        args.stage = (args.stage / 2 + 63) / 64 * 64;
        lds = bytes();
    }
    if (lds > 64 * 1024 && args.gst_bits) {
        args.gst_bits = 0;
        lds = bytes();
    }
    if (lds > 64 * 1024 && args.local) {
        args.local = 0;
        lds = bytes();
    }
    if (lds > 64 * 1024) return hipErrorInvalidValue;    // the caller falls back to the interpreter
    void *params[] = {&args};
    hipFunction_t fn = !args.local ? f.free_1024 : (wg_threads <= 256 ? f.local_256 : f.local_1024);
    return hipModuleLaunchKernel(fn, n_wg, 1, 1, wg_threads, 1, 1, (unsigned)lds, s, params, nullptr);
}

hipError_t launch_jit_lockstep(const JitFunctions &f, const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads,
                               hipStream_t s) {
    if (n_wg == 0) return hipSuccess;
    InterpArgs args = a;
    args.rep_hold = rep_hold_for(wg_threads);
    if (!args.local) args.gst_bits = 0;
    auto bytes = [&] {
        return interp_lds_bytes(args.sh_words_max, wg_threads, args.stage, true, args.local != 0, args.gst_bits);
    };
    size_t lds = bytes();
    while (lds > 64 * 1024 && args.stage > 64) {
        args.stage = (args.stage / 2 + 63) / 64 * 64;
        lds = bytes();
    }
    if (lds > 64 * 1024 && args.gst_bits) {
        args.gst_bits = 0;
        lds = bytes();
    }
    if (lds > 64 * 1024 && args.local) {
        args.local = 0;
        lds = bytes();
    }
    if (lds > 64 * 1024) return hipErrorInvalidValue;    // the caller falls back to the interpreter
    void *params[] = {&args};
    hipFunction_t k = args.local ? (wg_threads <= 256 ? f.lock_local_256 : f.lock_local) : f.lock;
    return hipModuleLaunchKernel(k, n_wg, 1, 1, wg_threads, 1, 1, (unsigned)lds, s, params, nullptr);
}

bool jit_fits(uint32_t sh_words_max, uint32_t wg_threads) {
    return interp_lds_bytes(sh_words_max, wg_threads, 64, false, false, 0) <= 64 * 1024;
}

}  // namespace kc
