// Host driver of the float64 plan builder for sanitizer runs (AddressSanitizer and
// UndefinedBehaviorSanitizer): builds the plan of every geometry given on stdin, one per
// line, with the builder's worker threads, and prints its counts.
//
// Line: R D feed lambda0 z0 lambda_first dalpha col_offset dw row_offset n_views
//       views_per_turn cols rows  dx dy dz x_first y_first z_first nx ny nz
//       n_psi n_threads flags bp_slices
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>

#include "../../paper_2201_02309_amd/csrc/plan.hpp"

int main() {
    std::string line;
    int n = 0;
    while (std::getline(std::cin, line)) {
        if (line.empty()) continue;
        std::istringstream in(line);
        katsevich_geometry g{};
        katsevich_grid gr{};
        katsevich_options o{};
        long long nv = 0;
        in >> g.R >> g.D >> g.feed_per_turn >> g.lambda0 >> g.z0 >> g.lambda_first >> g.dalpha >>
            g.col_offset >> g.dw >> g.row_offset >> nv >> g.views_per_turn >> g.det_cols >> g.det_rows;
        g.n_views = nv;
        in >> gr.dx >> gr.dy >> gr.dz >> gr.x_first >> gr.y_first >> gr.z_first >> gr.nx >> gr.ny >> gr.nz;
        in >> o.n_psi >> o.n_threads >> o.flags >> o.bp_slices;
        if (!in) {
            std::fprintf(stderr, "bad line %d\n", n);
            return 2;
        }
        kats::PlanHost P;
        std::string err;
        const int st = kats::build_plan(g, gr, o, P, err);
        if (st != KATS_OK) {
            std::printf("plan %d: status %d (%s)\n", n, st, err.c_str());
        } else {
            std::printf("plan %d: W %d n_vv %lld valid %lld views %lld..%lld boxes %dx%d table %llu\n", n,
                        P.W, (long long)P.n_vv, (long long)P.n_valid, (long long)P.first_view,
                        (long long)P.last_view, P.bp_box_rows, P.bp_box_cols,
                        (unsigned long long)P.layout.total);
        }
        ++n;
    }
    std::printf("plans %d ok\n", n);
    return 0;
}
