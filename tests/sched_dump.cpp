// Test helper (host only): run the staged scheduler of libqsim on a gate list and write its tables, so
// that a CPU test can check them. Usage: sched_dump <gates.bin> <n> <dtype> <m> <log_e> <out.bin>.
// An optional seventh argument sets the width of the pass search (default: the one plans use; 1: the
// greedy rule alone). gates.bin holds qsim_gate records; out.bin holds the five record sizes, the five table lengths and
// the pass, stage, round, op and two-qubit block tables.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "staged_device.h"

using namespace qsim::staged;

int main(int argc, char **argv)
{
    if (argc != 7 && argc != 8) {
        std::fprintf(stderr, "usage: sched_dump gates.bin n dtype m log_e out.bin [search_width]\n");
        return 2;
    }
    std::FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<qsim_gate> gates;
    qsim_gate g;
    while (std::fread(&g, sizeof g, 1, f) == 1) gates.push_back(g);
    std::fclose(f);
    std::vector<SPass> passes;
    std::vector<SStage> stages;
    std::vector<SRound> rounds;
    std::vector<SOp> ops;
    std::vector<SBlk> blks;
    const int rc = staged_schedule(std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), std::atoi(argv[5]), gates,
                                   passes, stages, rounds, ops, blks,
                                   argc == 8 ? std::atoi(argv[7]) : kPassSearchWidth);
    if (rc) {
        std::printf("rc=%d\n", rc);
        return 1;
    }
    std::FILE *o = std::fopen(argv[6], "wb");
    if (!o) return 2;
    const uint64_t head[10] = {sizeof(SPass), sizeof(SStage), sizeof(SRound), sizeof(SOp), sizeof(SBlk),
                               passes.size(), stages.size(), rounds.size(), ops.size(), blks.size()};
    std::fwrite(head, sizeof head, 1, o);
    std::fwrite(passes.data(), sizeof(SPass), passes.size(), o);
    std::fwrite(stages.data(), sizeof(SStage), stages.size(), o);
    std::fwrite(rounds.data(), sizeof(SRound), rounds.size(), o);
    std::fwrite(ops.data(), sizeof(SOp), ops.size(), o);
    std::fwrite(blks.data(), sizeof(SBlk), blks.size(), o);
    std::fclose(o);
    return 0;
}
