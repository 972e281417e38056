// Host driver of the bilinear split shared with the device assembly
// (paper_2604_11920_amd/csrc/split_path.h), for the CPU tests: per path,
// the records of its pieces in order, grouped by node (a stable sort by
// node), each group summed with sum_contributions, nodes with a positive
// sum kept, ascending.
// in:  int64 npaths, npoints, nx, ny; double h, km; int64 pt_ptr[npaths+1];
//      double px[npoints], py[npoints], plen[npoints]
// out: int64 node_ptr[npaths+1]; int64 total; int32 node_k[total]; double node_len[total]
// usage: split_check IN OUT
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "split_path.h"

template <class T>
static void get(FILE *f, T *p, size_t n)
{
    if (n && fread(p, sizeof(T), n, f) != n) { fprintf(stderr, "short read\n"); exit(2); }
}
template <class T>
static void put(FILE *f, const T *p, size_t n)
{
    if (n) fwrite(p, sizeof(T), n, f);
}

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    FILE *fi = fopen(argv[1], "rb");
    if (!fi) return 2;
    int64_t hdr[4];
    double gh[2];
    get(fi, hdr, 4);
    get(fi, gh, 2);
    const int64_t np = hdr[0], npt = hdr[1];
    lsqr::SplitGrid g{gh[0], gh[1], (int)hdr[2], (int)hdr[3]};
    std::vector<int64_t> pt((size_t)np + 1);
    std::vector<double> px((size_t)npt), py((size_t)npt), pl((size_t)npt);
    get(fi, pt.data(), pt.size());
    get(fi, px.data(), px.size());
    get(fi, py.data(), py.size());
    get(fi, pl.data(), pl.size());
    fclose(fi);
    std::vector<int64_t> node_ptr((size_t)np + 1, 0);
    std::vector<int32_t> node_k;
    std::vector<double> node_len;
    std::vector<int64_t> rn;
    std::vector<double> rv;
    for (int64_t p = 0; p < np; ++p) {
        rn.clear();
        rv.clear();
        int64_t nb[12];
        double vb[12];
        for (int64_t i = pt[(size_t)p]; i + 1 < pt[(size_t)p + 1]; ++i) {
            const int r = lsqr::split_piece(px[(size_t)i], py[(size_t)i], px[(size_t)i + 1],
                                            py[(size_t)i + 1], pl[(size_t)i], g, nb, vb);
            rn.insert(rn.end(), nb, nb + r);
            rv.insert(rv.end(), vb, vb + r);
        }
        std::vector<size_t> ord(rn.size());
        std::iota(ord.begin(), ord.end(), (size_t)0);
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return rn[a] < rn[b]; });
        for (size_t s = 0; s < ord.size();) {
            size_t e = s;
            while (e < ord.size() && rn[ord[e]] == rn[ord[s]]) ++e;
            const double sum = lsqr::sum_contributions((int)(e - s), [&](int j) { return rv[ord[s + j]]; });
            if (sum > 0.0) {
                node_k.push_back((int32_t)rn[ord[s]]);
                node_len.push_back(sum);
            }
            s = e;
        }
        node_ptr[(size_t)p + 1] = (int64_t)node_k.size();
    }
    FILE *fo = fopen(argv[2], "wb");
    if (!fo) return 2;
    const int64_t tot = (int64_t)node_k.size();
    put(fo, node_ptr.data(), node_ptr.size());
    put(fo, &tot, 1);
    put(fo, node_k.data(), node_k.size());
    put(fo, node_len.data(), node_len.size());
    fclose(fo);
    return 0;
}
