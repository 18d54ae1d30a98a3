// Host-only driver of the planner for the sanitizer build (AddressSanitizer +
// UndefinedBehaviorSanitizer, compiled with g++ from the planner sources).
// Reads a circuit and a list of option sets from a text file, builds every
// plan and prints, per option set, the status, the plan JSON (detail 2) and the
// workspace of 64 and 1000 bitstrings, for comparison with the library build.
//
// Input: "rows cols n_slots n_gates", n_gates lines "kind cycle q0 q1 slot",
// then lines "ordering min_sliced_vars max_rank tree_exec mem_budget
// checkpoint_budget n_open q...".
#include <cstdio>
#include <fstream>
#include <iostream>
#include <string>
#include <vector>

#include "plan.hpp"

int main(int argc, char** argv) {
    if (argc != 2) { std::fprintf(stderr, "usage: planner_driver FILE\n"); return 2; }
    std::ifstream in(argv[1]);
    int rows = 0, cols = 0, n_slots = 0, n_gates = 0;
    if (!(in >> rows >> cols >> n_slots >> n_gates)) return 2;
    std::vector<qgm_gate> gates(static_cast<size_t>(n_gates));
    for (auto& g : gates)
        if (!(in >> g.kind >> g.cycle >> g.q0 >> g.q1 >> g.slot)) return 2;
    qgm_circuit c{rows, cols, n_gates, n_slots, gates.data()};
    int ordering, msv, max_rank, tree_exec, n_open;
    unsigned long long mem_budget, ckpt_budget;
    while (in >> ordering >> msv >> max_rank >> tree_exec >> mem_budget >> ckpt_budget >> n_open) {
        std::vector<int32_t> open(static_cast<size_t>(n_open));
        for (auto& q : open) in >> q;
        qgm_plan_opts o{};
        o.ordering = ordering;
        o.min_sliced_vars = msv;
        o.max_rank = max_rank;
        o.tree_exec = tree_exec;
        o.mem_budget = mem_budget;
        o.checkpoint_budget = ckpt_budget;
        qgm::Plan p;
        std::string err;
        const qgm_status st = qgm::build_plan(&c, open.data(), n_open, o, p, &err);
        std::cout << "status " << int(st) << "\n";
        if (st == QGM_OK) {
            std::cout << qgm::plan_json(p, 2) << "\n";
            std::cout << "ws " << qgm::workspace_layout(p, 64).total << " " << qgm::workspace_layout(p, 1000).total << "\n";
        }
    }
    return 0;
}
