// Test-only known-answer generator: runs the Philox4x32-10 block function of
// rocRAND's open-source header (MIT licence, /opt/rocm/include/rocrand) on the
// host.  It is an implementation independent of the oracle's, used only to
// cross-check it; nothing in the product links this file.
// usage: philox_rocrand_kat  (reads lines "c0 c1 c2 c3 k0 k1" in hex on stdin)
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = e.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
