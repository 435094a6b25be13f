// Host check of the sparse layout's slot image (built by the library's own
// compile code, included below): walks random texts, with bytes outside the
// alphabet mixed in, through the image exactly as the walk kernel reads it
// (uniform form: one slot and the shared default; general form: slot and
// header) and compares every state and the count of steps entering a final
// state with a walk of the dense table. Input file: Q, A, start, number of
// final states (u32 each), the alphabet (A bytes), the table (Q x A u32,
// row-major), the final states (u32). Prints "form=<uniform|general>
// slots=<n>" and exits 0 when every walk agrees, "no layout" and exits 3
// when the slots do not fit, 1 on a mismatch.
#include "../paper_1412_1741_amd/csrc/parem_api.cpp"

#include <cstdio>
#include <random>

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint32_t hdr[4];
    if (fread(hdr, 4, 4, f) != 4) return 2;
    const uint32_t Q = hdr[0], A = hdr[1], start = hdr[2], nacc = hdr[3];
    std::vector<uint8_t> alpha(A);
    std::vector<uint32_t> t((size_t)Q * A), acc(nacc);
    if (fread(alpha.data(), 1, A, f) != A || fread(t.data(), 4, t.size(), f) != t.size() ||
        fread(acc.data(), 4, nacc, f) != nacc)
        return 2;
    fclose(f);
    DeviceDfa d;
    d.Q = Q;
    d.A = A;
    d.sent = Q;
    d.start = start;
    d.cls.assign(256, (uint8_t)A);
    for (uint32_t a = 0; a < A; ++a) d.cls[alpha[a]] = (uint8_t)a;
    d.final_flag.assign(Q + 1, 0);
    for (uint32_t q : acc) d.final_flag[q] = 1;
    SparseImage im;
    if (!sparse_slots(d, t, im)) {
        printf("no layout\n");
        return 3;
    }
    const size_t slots = (im.image.size() - 256) / 4;
    const uint32_t *slot = reinterpret_cast<const uint32_t *>(im.image.data() + 256);
    bool raw = true;
    for (int x = 0; x < 256; ++x) raw &= d.cls[x] < A;
    auto at = [&](size_t i) -> uint32_t {
        if (i >= slots) {
            printf("slot %zu read beyond the image (%zu slots)\n", i, slots);
            exit(1);
        }
        return slot[i];
    };
    auto flag = [&](uint32_t s) { return im.uniform ? (s >> 16) & 0xffu : (at((s & 0xffffu) + 256) >> 16) & 0xffu; };
    std::mt19937_64 rng(1412);
    for (int trial = 0; trial < 2000; ++trial) {
        uint32_t q = (uint32_t)(rng() % (Q + 1)), s = im.walk[q];
        int64_t want = 0, got = -(int64_t)flag(s);
        for (int i = 0; i < 2000; ++i) {
            const uint32_t x = (rng() % 8 == 0) ? (uint32_t)(rng() % 256) : alpha[rng() % A];
            const uint32_t col = d.cls[x], key = raw ? x : col, b = s & 0xffffu;
            got += flag(s);
            if (im.uniform) {
                const uint32_t e = at(b + key);
                s = (e >> 24) == key ? e : im.d0;
            } else {
                const uint32_t e = at(b + key), h = at(b + 256);
                s = (e >> 16) == key ? (e & 0xffffu) : (h & 0xffffu);
            }
            q = (q < Q && col < A) ? t[(size_t)q * A + col] : Q;
            want += d.final_flag[q];
            if ((s & 0xffffu) >= im.sids.size() || im.sids[s & 0xffffu] != q) {
                printf("trial %d step %d: state %u, layout gives %u\n", trial, i, q,
                       (s & 0xffffu) < im.sids.size() ? im.sids[s & 0xffffu] : 0xffffffffu);
                return 1;
            }
        }
        got += flag(s);
        if (got != want) {
            printf("trial %d: count %lld, layout gives %lld\n", trial, (long long)want, (long long)got);
            return 1;
        }
    }
    printf("form=%s slots=%zu\n", im.uniform ? "uniform" : "general", slots);
    return 0;
}
