// Controller state of adaptive graphlet sampling (Sec. 4.1, Algorithm AGS),
// advanced one round at a time: a round draws samples of the current shape j,
// and its class histogram updates the hit counts c_i, the per-shape sample
// counts n_j, the covered set and the next shape.
#pragma once

#include <vector>

#include "table.hpp"

struct AgsState {
    int k = 0, S = 0, NS = 0;             // classes and unrooted shapes at this k
    int64_t cbar = 0;
    std::vector<uint32_t> codes;          // canonical code of each class
    std::vector<int64_t> c, nj;
    std::vector<double> w, tjd;
    std::vector<char> cov, sig_ok;
    std::vector<const int64_t *> sig;     // sigma_ij row of each class once hit (process-wide cache)
    std::vector<int32_t> shapes;          // shape of every round so far
    int64_t drawn = 0, ncov = 0;
    int j = -1;                           // shape of the next round

    // the start shape is the one with the largest t_j (ties: smaller j);
    // EEMPTY when the table has no colourful k-treelet
    scc_status init(const scc_table *T, int64_t cbar, hipStream_t st);
    // a finished round of `n` samples of shape j with class histogram hist[S]
    void add_round(int64_t n, const unsigned long long *hist);
    bool covered() const { return ncov >= S; }
    // hits c_i, w_i (0 for classes never hit) and n_j
    void result(int64_t *hits, double *w_out, int64_t *n_j) const;
};

// sigma_ij rows (spanning trees of each unrooted shape) of classes `ids` of k,
// computed on host threads on first use and kept for the process
void class_sigma_rows(int k, const std::vector<int> &ids, std::vector<const int64_t *> &rows);
// the k-graphlet class lookup table on the device (built once per k)
scc_status class_lut(int k, hipStream_t st, const uint16_t **lut, int *num_classes);
