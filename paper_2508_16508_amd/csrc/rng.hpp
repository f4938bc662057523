// rng.hpp -- device-side counter-based random draws for the predation and
// traffic models.
//
// A draw is keyed on (seed, step, agent, purpose) and carries no state, so a
// model resumes bit-exactly from its state and step counter.  The mixer is the
// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014): add the
// golden-ratio increment, then two xor-shift/multiply rounds with Stafford's
// "Mix13" constants and a closing xor-shift.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace abm {

__device__ __forceinline__ uint64_t splitmix64_out(uint64_t s) {
    uint64_t z = s + 0x9E3779B97F4A7C15ull;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// Per-(seed, step) stream key; hoisted out of per-agent loops.
__device__ __forceinline__ uint64_t stream_key(uint32_t seed, uint32_t step) {
    return splitmix64_out((static_cast<uint64_t>(seed) << 32) | step);
}

__device__ __forceinline__ uint32_t draw(uint64_t key, uint32_t agent, uint32_t purpose) {
    const uint64_t word = (static_cast<uint64_t>(agent) << 32) | purpose;
    return static_cast<uint32_t>(splitmix64_out(key ^ word) >> 32);
}

// floor(h * n / 2^32): multiply-shift range reduction onto [0, n).
__device__ __forceinline__ uint32_t scale(uint32_t h, uint32_t n) {
    return __umulhi(h, n);
}

// Draw purposes.
enum Purpose : uint32_t {
    kGrassGrown = 0x01, kGrassCountdown = 0x02,
    kSheepX = 0x10, kSheepY = 0x11, kSheepE = 0x12, kSheepMove = 0x13,
    kSheepGrassKey = 0x14, kSheepPreyKey = 0x15, kSheepBreed = 0x16,
    kWolfX = 0x20, kWolfY = 0x21, kWolfE = 0x22, kWolfMove = 0x23,
    kWolfEatKey = 0x24, kWolfBreed = 0x26,
    kTrafficLight = 0x30, kTrafficLane = 0x31, kTrafficSpawn = 0x32
};

constexpr uint32_t kInitStep = 0xFFFFFFFFu;

}  // namespace abm
