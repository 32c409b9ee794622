// Device memory arena of the library.
//
// Memory is reserved from the runtime in chunks (hipMalloc) and handed out
// by best fit; released blocks are merged with free neighbours of the same
// chunk.  There is one arena per (device, stream): a block released on a
// stream is handed out again only to later requests on that stream, which
// the stream orders after every use of the old contents.  A block released
// on another stream than the one it came from waits for that stream first.
// Chunks stay reserved until pauli_trim_memory; a new chunk is at least half
// the size of what the arena already holds, up to 1/16 of the device beyond
// the request (so growing sizes need few reservations).  When the runtime
// refuses a chunk, every idle chunk is returned and the request is retried
// once at the size it needs.
//
// The runtime's stream-ordered pool is not used: with outputs of many
// different sizes (batches, a growing propagation state) its allocation and
// release calls were seen to stall for seconds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace pauli {

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kChunkMin = size_t(256) << 20;

struct Arena {
  int dev = 0;
  hipStream_t s = nullptr;
  struct Free {
    size_t size;
    int chunk;
  };
  std::map<char*, Free> free_at;               // free blocks by address
  std::multimap<size_t, char*> free_by_size;   // the same blocks by size
  std::vector<char*> chunk_base;
  std::vector<size_t> chunk_size;              // 0 once returned
  std::vector<size_t> chunk_used;
};

struct Live {
  Arena* arena;
  size_t size;
  int chunk;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Arena>> g_arenas;
std::unordered_map<char*, Live> g_live;

void unlink_free(Arena& a, std::map<char*, Arena::Free>::iterator it) {
  auto range = a.free_by_size.equal_range(it->second.size);
  for (auto j = range.first; j != range.second; ++j)
    if (j->second == it->first) {
      a.free_by_size.erase(j);
      break;
    }
  a.free_at.erase(it);
}

// Adds [p, p + size) of chunk c to the free lists, merged with free
// neighbours of the same chunk.
void link_free(Arena& a, char* p, size_t size, int c) {
  auto next = a.free_at.lower_bound(p);
  if (next != a.free_at.end() && next->second.chunk == c && p + size == next->first) {
    size += next->second.size;
    unlink_free(a, next);
  }
  auto after = a.free_at.lower_bound(p);
  if (after != a.free_at.begin()) {
    auto prev = std::prev(after);
    if (prev->second.chunk == c && prev->first + prev->second.size == p) {
      p = prev->first;
      size += prev->second.size;
      unlink_free(a, prev);
    }
  }
  a.free_at.emplace(p, Arena::Free{size, c});
  a.free_by_size.emplace(size, p);
}

Arena& arena_for(int dev, hipStream_t s) {
  auto& slot = g_arenas[{dev, s}];
  if (!slot) {
    slot = std::make_unique<Arena>();
    slot->dev = dev;
    slot->s = s;
  }
  return *slot;
}

// Returns every chunk of device dev with nothing in use to the runtime.
// Caller holds g_mu.
void release_idle_chunks(int dev) {
  for (auto& kv : g_arenas) {
    Arena& a = *kv.second;
    if (a.dev != dev) continue;
    for (size_t c = 0; c < a.chunk_base.size(); ++c) {
      if (a.chunk_size[c] == 0 || a.chunk_used[c] != 0) continue;
      auto it = a.free_at.find(a.chunk_base[c]);
      if (it != a.free_at.end()) unlink_free(a, it);  // the whole chunk is one free block
      (void)hipFree(a.chunk_base[c]);
      a.chunk_size[c] = 0;
    }
  }
}

size_t chunk_bytes(size_t b) {
  if (b <= kChunkMin) return kChunkMin;
  // eight steps per octave, so that a returned chunk fits similar requests
  size_t base = kChunkMin;
  while (base * 2 <= b) base <<= 1;
  const size_t step = base / 8;
  return base + (b - base + step - 1) / step * step;
}

}  // namespace

void* arena_alloc(int dev, hipStream_t s, size_t bytes) {
  bytes = (bytes + kAlign - 1) / kAlign * kAlign;
  std::lock_guard<std::mutex> lk(g_mu);
  Arena& a = arena_for(dev, s);
  auto it = a.free_by_size.lower_bound(bytes);
  if (it == a.free_by_size.end()) {
    // chunks grow with the arena (at least half of what it holds), so sizes
    // that keep growing need few reservations
    size_t held = 0;
    for (size_t c = 0; c < a.chunk_size.size(); ++c) held += a.chunk_size[c];
    size_t cb = chunk_bytes(bytes);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      (void)hipGetLastError();
      total_b = 0;
    }
    const size_t grow = std::min(held / 2, total_b / 16);  // at most 1/16 of the device beyond need
    if (grow > cb) cb = chunk_bytes(grow);
    void* base = nullptr;
    hipError_t e = hipMalloc(&base, cb);
    if (e != hipSuccess || !base) {
      // return every idle chunk and ask for exactly what is needed
      (void)hipGetLastError();
      release_idle_chunks(dev);
      cb = chunk_bytes(bytes);
      base = nullptr;
      e = hipMalloc(&base, cb);
    }
    if (e != hipSuccess || !base) {
      (void)hipGetLastError();
      fail(PAULI_ERR_OOM, "device allocation of " + std::to_string(cb) + " bytes failed");
    }
    const int c = static_cast<int>(a.chunk_base.size());
    a.chunk_base.push_back(static_cast<char*>(base));
    a.chunk_size.push_back(cb);
    a.chunk_used.push_back(0);
    link_free(a, static_cast<char*>(base), cb, c);
    it = a.free_by_size.lower_bound(bytes);
  }
  char* p = it->second;
  auto fit = a.free_at.find(p);
  const Arena::Free f = fit->second;
  unlink_free(a, fit);
  if (f.size - bytes >= kAlign) link_free(a, p + bytes, f.size - bytes, f.chunk);
  else bytes = f.size;
  a.chunk_used[f.chunk] += bytes;
  g_live[p] = Live{&a, bytes, f.chunk};
  return p;
}

void arena_trim(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  release_idle_chunks(dev);
}

void arena_free(void* ptr, hipStream_t s) {
  char* p = static_cast<char*>(ptr);
  Live l;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    l = it->second;
    g_live.erase(it);
  }
  // uses on another stream must end before the owner's stream reuses it
  if (l.arena->s != s) (void)hipStreamSynchronize(s);
  std::lock_guard<std::mutex> lk(g_mu);
  l.arena->chunk_used[l.chunk] -= l.size;
  link_free(*l.arena, p, l.size, l.chunk);
}

}  // namespace pauli
