// Host build of the library's random-number header: writes, as raw float32,
//   ln of v * 2^-24 for every v in [1, 2^24]            (16 Mi values)
//   ln of the positive floats with bit patterns lo + 61 k up to 17.0
//   Box-Muller pairs (z0, z1) of the word pairs (a_i, b_i) read from stdin
//   the Gumbel deviates of the words w_i read from stdin
// so that a test can compare them bit for bit with the oracle's.  Nothing
// here touches a GPU.
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <vector>

#include "rng.h"

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    const size_t n_pairs = size_t(std::atoll(argv[1]));
    const size_t n_words = size_t(std::atoll(argv[2]));
    std::vector<uint32_t> in(2 * n_pairs + n_words);
    if (std::fread(in.data(), 4, in.size(), stdin) != in.size()) return 3;
    std::vector<float> out;
    out.reserve((size_t(1) << 24) + 4400000 + 2 * n_pairs + n_words);
    for (uint32_t v = 1; v <= (1u << 24); ++v) out.push_back(eco::ln_of_24bit(v));
    const float lo_f = 0x1p-24f, hi_f = 17.0f;
    uint32_t lo, hi;
    std::memcpy(&lo, &lo_f, 4);
    std::memcpy(&hi, &hi_f, 4);
    for (uint32_t b = lo; b <= hi; b += 61) {
        float x;
        std::memcpy(&x, &b, 4);
        out.push_back(eco::ln_positive(x));
    }
    for (size_t i = 0; i < n_pairs; ++i) {
        float z0, z1;
        eco::box_muller(in[2 * i], in[2 * i + 1], z0, z1);
        out.push_back(z0);
        out.push_back(z1);
    }
    for (size_t i = 0; i < n_words; ++i) out.push_back(eco::gumbel_of_word(in[2 * n_pairs + i]));
    if (std::fwrite(out.data(), 4, out.size(), stdout) != out.size()) return 4;
    return 0;
}
