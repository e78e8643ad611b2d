// emu_ptr.hpp -- host stand-ins for the device's constant-address-space
// pointers, used only when walk_core.hpp is compiled for the CPU (the test
// emulation of the kernels).  Every read is bounds-checked against the
// registered buffer it belongs to; an out-of-bounds read aborts.
#pragma once

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace bbfg {

struct EmuRegion {
    const char* lo;
    const char* hi;
};

inline std::vector<EmuRegion>& emu_regions()
{
    static std::vector<EmuRegion> r;
    return r;
}

inline void emu_register(const void* p, size_t bytes)
{
    emu_regions().push_back({static_cast<const char*>(p), static_cast<const char*>(p) + bytes});
}

inline void emu_clear() { emu_regions().clear(); }

[[noreturn]] inline void emu_fail(const char* what)
{
    std::fprintf(stderr, "emu: %s\n", what);
    std::abort();
}

template <typename T>
struct kptr {
    const T* p;
    const char* lo;
    const char* hi;
    const T& operator[](int64_t i) const
    {
        const T* q = p + i;
        if (reinterpret_cast<const char*>(q) < lo || reinterpret_cast<const char*>(q + 1) > hi)
            emu_fail("out-of-bounds read");
        return *q;
    }
    kptr operator+(int64_t d) const { return kptr{p + d, lo, hi}; }
};

template <typename T>
inline kptr<T> kconst(const T* p)
{
    const char* c = reinterpret_cast<const char*>(p);
    for (const EmuRegion& r : emu_regions())
        if (c >= r.lo && c <= r.hi) return kptr<T>{p, r.lo, r.hi};
    emu_fail("pointer outside every registered buffer");
}

inline uint32_t uniform_u32(uint32_t x) { return x; }

}  // namespace bbfg
