// Host-only driver for the server's scheduling core (no GPU): reads commands
// from stdin and prints the scheduler's decisions, so the policy can be
// tested on a machine without a GPU.
//   submit <id> <bytes>   -> "ok" | "reject"
//   admit                 -> admitted slot ids and request ids
//   quantum               -> plan + complete one quantum; prints finished
//   retire <slot>
//   stats                 -> queued active bytes_in_use largest_free
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>

#include "../paper_1811_04384_amd/csrc/ising_sched.hpp"

int main(int argc, char** argv) {
    size_t budget = argc > 1 ? std::stoull(argv[1]) : 1 << 20;
    int slots = argc > 2 ? std::stoi(argv[2]) : 4;
    int quantum = argc > 3 ? std::stoi(argv[3]) : 10;
    ising::Scheduler s(budget, slots, quantum);
    ising::ArenaAllocator probe(budget);
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string cmd;
        in >> cmd;
        if (cmd == "submit") {
            ising::Request r;
            in >> r.id >> r.bytes >> r.sweeps;
            std::cout << (s.submit(r) ? "ok" : "reject") << "\n";
        } else if (cmd == "admit") {
            auto a = s.admit(0.0);
            std::cout << "admitted";
            for (int i : a) std::cout << " " << i << ":" << s.slots()[i].req.id << "@" << s.slots()[i].off;
            std::cout << "\n";
        } else if (cmd == "quantum") {
            s.plan_quantum();
            s.complete_quantum();
            auto f = s.finished();
            std::cout << "finished";
            for (int i : f) std::cout << " " << i << ":" << s.slots()[i].req.id;
            std::cout << "\n";
        } else if (cmd == "retire") {
            int i;
            in >> i;
            s.retire(i);
            std::cout << "retired " << i << "\n";
        } else if (cmd == "stats") {
            std::cout << "stats " << s.queued() << " " << s.active() << " " << s.bytes_in_use() << "\n";
        }
    }
    return 0;
}
