// Independent reference for the Philox4x32-10 block function: the rocRAND
// library's engine, evaluated on the host.  Used only by the oracle's tests.
// The engine is seeded with key = seed (low word key[0]); subsequence s moves
// counter words 2,3 to s; offset 4*o moves counter words 0,1 to o; the next
// four outputs are then the block for that counter.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void ref_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    unsigned long long subseq = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    unsigned long long offset = 4ull * ((unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    for (int i = 0; i < 4; i++) out[i] = eng.next();
}
