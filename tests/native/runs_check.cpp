// CPU driver for the host layout builders: reads a CSR structure from a
// binary file, runs the builders and writes their arrays back for checking.
//   in : int64 m, n, nz, nnz; int64 row_ptr[m+1]; int32 col[nnz]
//   out: int64 ok_nodes, nnruns, nnodes; int64 nrp[nnodes+1]; int64 nvq[4 nnodes+1];
//        uint32 row[]; uint32 src[]; uint32 dst[]; uint16 desc[]; int32 order[nnodes];
//        (node runs built) int64 rrp[m+1]; uint32 rrid[nnruns]  (row order of the runs)
//        int64 ok_groups, ngroups, ngcols; int32 gp[ngroups+1]; int64 gcp[ngroups+1];
//        int32 gcol[ngcols]; uint16 slot[nnz]   (row groups of at most CAP columns)
//        (node runs built, for W = 2, 4 then 8) int64 ok_pairs, total; uint32 dstp[nnruns];
//        int64 nvqp[4 nnodes+1]
// usage: runs_check IN OUT [CAP]   (CAP defaults to 4096)
#include <stdio.h>
#include <stdlib.h>

#include "runs_host.h"

template <class T>
static void put(FILE *f, const T *p, size_t n) { if (n) fwrite(p, sizeof(T), n, f); }

int main(int argc, char **argv)
{
    if (argc != 3 && argc != 4) { fprintf(stderr, "usage: runs_check IN OUT [CAP]\n"); return 2; }
    const int cap = argc == 4 ? atoi(argv[3]) : 4096;
    FILE *fi = fopen(argv[1], "rb");
    if (!fi) return 2;
    int64_t hdr[4];
    if (fread(hdr, 8, 4, fi) != 4) return 2;
    const int64_t m = hdr[0], n = hdr[1], nz = hdr[2], nnz = hdr[3];
    std::vector<int64_t> rp((size_t)m + 1);
    std::vector<int32_t> ci((size_t)nnz);
    if (fread(rp.data(), 8, (size_t)m + 1, fi) != (size_t)m + 1) return 2;
    if (nnz && fread(ci.data(), 4, (size_t)nnz, fi) != (size_t)nnz) return 2;
    fclose(fi);
    FILE *fo = fopen(argv[2], "wb");
    if (!fo) return 2;
    lsqr::NodeRuns R;
    const int64_t ok2 = lsqr::build_node_runs_host(m, n, (int)nz, rp.data(), ci.data(), R);
    const int64_t nr2 = ok2 ? (int64_t)R.row.size() : 0, nn = ok2 ? n / nz : 0;
    put(fo, &ok2, 1);
    put(fo, &nr2, 1);
    put(fo, &nn, 1);
    if (ok2) {
        put(fo, R.nrp.data(), R.nrp.size()); put(fo, R.nvq.data(), R.nvq.size());
        put(fo, R.row.data(), R.row.size()); put(fo, R.src.data(), R.src.size());
        put(fo, R.dst.data(), R.dst.size()); put(fo, R.desc.data(), R.desc.size());
        put(fo, R.order.data(), R.order.size());
    }
    // row order of the node runs
    if (ok2) {
        std::vector<int64_t> rrp;
        std::vector<uint32_t> rrid;
        lsqr::row_order_of_runs(R, m, rrp, rrid);
        put(fo, rrp.data(), rrp.size()); put(fo, rrid.data(), rrid.size());
    }
    lsqr::RowGroups G;
    const int64_t ok5 = lsqr::build_row_groups_host(m, n, rp.data(), ci.data(), cap, G);
    const int64_t ng5 = ok5 ? (int64_t)G.gp.size() - 1 : 0, nc5 = ok5 ? (int64_t)G.gcol.size() : 0;
    put(fo, &ok5, 1);
    put(fo, &ng5, 1);
    put(fo, &nc5, 1);
    if (ok5) {
        put(fo, G.gp.data(), G.gp.size()); put(fo, G.gcp.data(), G.gcp.size());
        put(fo, G.gcol.data(), G.gcol.size()); put(fo, G.slot.data(), G.slot.size());
    }
    for (int W : {2, 4, 8}) {
        if (!ok2) break;
        std::vector<uint32_t> dstp;
        std::vector<int64_t> nvqp;
        int64_t total = 0;
        const int64_t ok6 = lsqr::pair_layout_host(R, nn, dstp, nvqp, total, W);
        put(fo, &ok6, 1);
        put(fo, &total, 1);
        put(fo, dstp.data(), dstp.size()); put(fo, nvqp.data(), nvqp.size());
    }
    fclose(fo);
    return 0;
}
