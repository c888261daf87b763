// Driver of the host build of the exact and double-word tiers for sanitizer
// runs (address and undefined-behaviour sanitizers): reads decision requests
// from a binary file, writes (class, bin, double-word class, double-word bin)
// per request.
//
// Request layout (little endian): int32 count, then per request
//   double comps[16]; int32 is_f32, tag, sigma, naxes, kind[2], nbins[2],
//   slots[2]; double edges0[nbins[0] + 1] (if naxes > 0);
//   double edges1[nbins[1] + 1] (if naxes > 1).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "exact_harness.cpp"

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *in = std::fopen(argv[1], "rb");
    FILE *out = std::fopen(argv[2], "wb");
    if (!in || !out) return 2;
    int32_t count = 0;
    if (std::fread(&count, 4, 1, in) != 1) return 2;
    for (int32_t r = 0; r < count; ++r) {
        double comps[16];
        int32_t h[10];
        if (std::fread(comps, 8, 16, in) != 16 || std::fread(h, 4, 10, in) != 10) return 3;
        const int naxes = h[3];
        std::vector<double> e[2];
        for (int a = 0; a < naxes; ++a) {
            e[a].resize((size_t)h[6 + a] + 1);
            if (std::fread(e[a].data(), 8, e[a].size(), in) != e[a].size()) return 3;
        }
        const int32_t kind[2] = { h[4], h[5] }, nb[2] = { h[6], h[7] }, sl[2] = { h[8], h[9] };
        int bin = -1, bdw = -1;
        const double *e0 = naxes > 0 ? e[0].data() : nullptr, *e1 = naxes > 1 ? e[1].data() : nullptr;
        const int c = hx_decide(comps, h[0], h[1], h[2], naxes, kind, nb, sl, e0, e1, &bin);
        bool finite = true;
        for (double v : comps) finite = finite && v == v && v - v == 0.0;
        const int cdw = finite ? hx_decide_dw(comps, h[1], h[2], naxes, kind, nb, sl, e0, e1, &bdw) : -1;
        const int32_t res[4] = { c, bin, cdw, bdw };
        std::fwrite(res, 4, 4, out);
    }
    std::fclose(in);
    std::fclose(out);
    return 0;
}
