// Host-side mesh and stencil setup of the library, run on its own so that it
// can be built with AddressSanitizer and UndefinedBehaviorSanitizer (the
// device code is not part of this program).  Usage:
//   host_setup_check MESH_FILE P,N_LO,N_HI,FLUX,BALANCE,CHARACTERISTIC,BC ...
// MESH_FILE: int32 dim, int64 n_vert, int64 n_cell, uint32 flags, then the
// vertex coordinates (double) and the cells' vertex ids (int32).  For every
// parameter set: mesh setup, stencil build and the transposed stencil tables;
// a parameter set the library refuses prints its message and counts as done.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.hpp"

using namespace wlseno;

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t dim = 0;
    int64_t nv = 0, nc = 0;
    uint32_t flags = 0;
    bool ok = std::fread(&dim, 4, 1, f) == 1 && std::fread(&nv, 8, 1, f) == 1 && std::fread(&nc, 8, 1, f) == 1 &&
              std::fread(&flags, 4, 1, f) == 1;
    std::vector<double> xyz(ok ? (size_t)(nv * dim) : 0);
    std::vector<int32_t> cells(ok ? (size_t)(nc * (dim + 1)) : 0);
    ok = ok && std::fread(xyz.data(), 8, xyz.size(), f) == xyz.size() &&
         std::fread(cells.data(), 4, cells.size(), f) == cells.size();
    std::fclose(f);
    if (!ok) return 2;
    HostMesh m;
    try {
        mesh_setup(m, dim, nv, xyz.data(), nc, cells.data(), flags);
    } catch (const Error &e) {
        std::printf("mesh refused: %s\n", e.msg.c_str());
        return 3;
    }
    for (int a = 2; a < argc; ++a) {
        wlseno_params prm{};
        int p = 3, lo = 12, hi = 20, flux = 0, bal = 0, chr = 0, bc = 0;
        if (std::sscanf(argv[a], "%d,%d,%d,%d,%d,%d,%d", &p, &lo, &hi, &flux, &bal, &chr, &bc) != 7) return 2;
        prm.p = p;
        prm.n_lo = lo;
        prm.n_hi = hi;
        prm.flux = flux;
        prm.weight_mode = 0;
        prm.lanes = 0;
        prm.eps = 1e-2;
        prm.alpha_w = 1.5;
        prm.rank_tol = 1e-12;
        prm.velocity[0] = 1.0;
        prm.velocity[1] = 0.5;
        prm.velocity[2] = 0.25;
        prm.gamma = 1.4;
        prm.bc = bc;
        prm.characteristic = chr;
        prm.balance = bal;
        for (int v = 0; v < 5; ++v) prm.far_state[v] = v == 0 ? 1.0 : 0.5;
        try {
            Build b;
            build_setup(m, prm, b);
            std::vector<int64_t> tptr;
            std::vector<int32_t> tpos;
            transpose_tables(b, m.nc, b.nf, tptr, tpos);
            std::printf("%s: %d-%d stencil rows, %zu transposed slots\n", argv[a], b.min_stencil, b.max_stencil,
                        tpos.size());
        } catch (const Error &e) {
            std::printf("%s refused: %s\n", argv[a], e.msg.c_str());
        }
    }
    return 0;
}
