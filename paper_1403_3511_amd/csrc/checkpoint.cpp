// Checkpoint and resume of a propagation's state: the coefficient vector c^n with a
// caller-written JSON header (t_n, n, the index set and the configuration).  A file is
//   "HSCKPT01" | u64 header bytes | header | u64 data bytes | u64 FNV-1a 64 of the data | data
// all integers little-endian.  A save writes path + ".tmp" and renames it over path, so
// an interrupted save leaves the previous checkpoint intact.  Device data moves through
// one pinned staging buffer in chunks, so a 17 GB vector needs no host copy of its size.
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <string>

#include "hs_internal.h"

namespace hs {

static const char kMagic[8] = {'H', 'S', 'C', 'K', 'P', 'T', '0', '1'};
static const int64_t kStage = int64_t(64) << 20;  // pinned staging chunk

static uint64_t fnv1a(uint64_t h, const uint8_t *p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}
static const uint64_t kFnvBasis = 14695981039346656037ull;

struct File {
  FILE *f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

static bool put_u64(FILE *f, uint64_t v) {
  uint8_t b[8];
  for (int i = 0; i < 8; ++i) b[i] = (uint8_t)(v >> (8 * i));
  return std::fwrite(b, 1, 8, f) == 8;
}
static bool get_u64(FILE *f, uint64_t &v) {
  uint8_t b[8];
  if (std::fread(b, 1, 8, f) != 8) return false;
  v = 0;
  for (int i = 0; i < 8; ++i) v |= (uint64_t)b[i] << (8 * i);
  return true;
}

// pinned staging buffer for device transfers, freed on scope exit
struct Stage {
  void *p = nullptr;
  ~Stage() {
    if (p) (void)hipHostFree(p);
  }
};

// Opens path and checks the framing.  On success the file is positioned at the data.
static int32_t open_checked(const char *path, File &F, std::string *header, uint64_t &data_len,
                            uint64_t &sum, const char *who) {
  F.f = std::fopen(path, "rb");
  if (!F.f) return fail(HS_E_IO, std::string(who) + ": cannot open " + path + ": " + std::strerror(errno));
  char magic[8];
  if (std::fread(magic, 1, 8, F.f) != 8 || std::memcmp(magic, kMagic, 8) != 0)
    return fail(HS_E_IO, std::string(who) + ": " + path + " is not a checkpoint file");
  uint64_t hl = 0;
  if (!get_u64(F.f, hl) || hl > (uint64_t(1) << 30))
    return fail(HS_E_IO, std::string(who) + ": bad header length in " + path);
  std::string h(hl, '\0');
  if (hl && std::fread(&h[0], 1, hl, F.f) != hl)
    return fail(HS_E_IO, std::string(who) + ": truncated header in " + path);
  if (!get_u64(F.f, data_len) || !get_u64(F.f, sum))
    return fail(HS_E_IO, std::string(who) + ": truncated file " + path);
  // the data must be exactly what is left of the file
  const long here = std::ftell(F.f);
  if (here < 0 || std::fseek(F.f, 0, SEEK_END) != 0)
    return fail(HS_E_IO, std::string(who) + ": cannot seek in " + path);
  const long end = std::ftell(F.f);
  if (end < here || (uint64_t)(end - here) != data_len)
    return fail(HS_E_IO, std::string(who) + ": " + path + " holds " + std::to_string(end - here) +
                             " data bytes, its header says " + std::to_string(data_len));
  if (std::fseek(F.f, here, SEEK_SET) != 0) return fail(HS_E_IO, std::string(who) + ": cannot seek in " + path);
  if (header) header->swap(h);
  return HS_OK;
}

}  // namespace hs

extern "C" int32_t hs_checkpoint_save(const char *path, const char *header_json, const void *src, int64_t bytes,
                                      int32_t src_on_device, void *stream) {
  using namespace hs;
  if (!path || !header_json || (!src && bytes > 0) || bytes < 0)
    return fail(HS_E_INVALID, "hs_checkpoint_save: NULL argument or negative size");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string tmp = std::string(path) + ".tmp";
  const size_t hl = std::strlen(header_json);
  uint64_t sum = kFnvBasis;
  Stage st;
  const uint8_t *hsrc = static_cast<const uint8_t *>(src);
  if (src_on_device && bytes > 0) {
    HS_HIP(hipHostMalloc(&st.p, (size_t)std::min(bytes, kStage), hipHostMallocDefault));
    // everything already enqueued that writes src finishes first
    HS_HIP(hipStreamSynchronize(s));
  }
  {
    File F;
    F.f = std::fopen(tmp.c_str(), "wb");
    if (!F.f) return fail(HS_E_IO, "hs_checkpoint_save: cannot create " + tmp + ": " + std::strerror(errno));
    // the checksum sits before the data: reserve its place, fill it in after the data
    if (std::fwrite(kMagic, 1, 8, F.f) != 8 || !put_u64(F.f, hl) ||
        (hl && std::fwrite(header_json, 1, hl, F.f) != hl) || !put_u64(F.f, (uint64_t)bytes))
      return fail(HS_E_IO, "hs_checkpoint_save: write failed on " + tmp);
    const long sum_at = std::ftell(F.f);
    if (sum_at < 0 || !put_u64(F.f, 0)) return fail(HS_E_IO, "hs_checkpoint_save: write failed on " + tmp);
    for (int64_t off = 0; off < bytes;) {
      const int64_t n = std::min(bytes - off, src_on_device ? kStage : bytes);
      const uint8_t *chunk = hsrc + off;
      if (src_on_device) {
        HS_HIP(hipMemcpyAsync(st.p, hsrc + off, (size_t)n, hipMemcpyDeviceToHost, s));
        HS_HIP(hipStreamSynchronize(s));
        chunk = static_cast<const uint8_t *>(st.p);
      }
      sum = fnv1a(sum, chunk, (size_t)n);
      if (std::fwrite(chunk, 1, (size_t)n, F.f) != (size_t)n)
        return fail(HS_E_IO, "hs_checkpoint_save: write failed on " + tmp);
      off += n;
    }
    if (std::fseek(F.f, sum_at, SEEK_SET) != 0 || !put_u64(F.f, sum) || std::fflush(F.f) != 0)
      return fail(HS_E_IO, "hs_checkpoint_save: write failed on " + tmp);
    const int rc = std::fclose(F.f);
    F.f = nullptr;
    if (rc != 0) return fail(HS_E_IO, "hs_checkpoint_save: close failed on " + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0)
    return fail(HS_E_IO, "hs_checkpoint_save: cannot rename " + tmp + " to " + path + ": " + std::strerror(errno));
  return HS_OK;
}

extern "C" int32_t hs_checkpoint_info(const char *path, char *header_out, int64_t cap, int64_t *header_len,
                                      int64_t *data_bytes) {
  using namespace hs;
  if (!path) return fail(HS_E_INVALID, "hs_checkpoint_info: NULL path");
  File F;
  std::string h;
  uint64_t dl = 0, sum = 0;
  const int32_t st = open_checked(path, F, &h, dl, sum, "hs_checkpoint_info");
  if (st != HS_OK) return st;
  if (header_len) *header_len = (int64_t)h.size();
  if (data_bytes) *data_bytes = (int64_t)dl;
  if (header_out && cap > 0) {
    const size_t n = std::min((size_t)(cap - 1), h.size());
    std::memcpy(header_out, h.data(), n);
    header_out[n] = 0;
  }
  return HS_OK;
}

extern "C" int32_t hs_checkpoint_load(const char *path, void *dst, int64_t bytes, int32_t dst_on_device,
                                      void *stream) {
  using namespace hs;
  if (!path || (!dst && bytes > 0) || bytes < 0)
    return fail(HS_E_INVALID, "hs_checkpoint_load: NULL argument or negative size");
  hipStream_t s = static_cast<hipStream_t>(stream);
  File F;
  uint64_t dl = 0, sum = 0;
  int32_t st = open_checked(path, F, nullptr, dl, sum, "hs_checkpoint_load");
  if (st != HS_OK) return st;
  if ((uint64_t)bytes != dl)
    return fail(HS_E_INVALID, "hs_checkpoint_load: " + std::string(path) + " holds " + std::to_string(dl) +
                                  " data bytes, the destination " + std::to_string(bytes));
  // read and check everything before touching the destination
  uint64_t got = kFnvBasis;
  Stage stg;
  uint8_t *hdst = static_cast<uint8_t *>(dst);
  if (dst_on_device && bytes > 0) {
    // a device destination: verify the whole file first, then copy in a second pass
    HS_HIP(hipHostMalloc(&stg.p, (size_t)std::min(bytes, kStage), hipHostMallocDefault));
    const long data_at = std::ftell(F.f);
    for (int64_t off = 0; off < bytes;) {
      const int64_t n = std::min(bytes - off, kStage);
      if (std::fread(stg.p, 1, (size_t)n, F.f) != (size_t)n)
        return fail(HS_E_IO, "hs_checkpoint_load: read failed on " + std::string(path));
      got = fnv1a(got, static_cast<const uint8_t *>(stg.p), (size_t)n);
      off += n;
    }
    if (got != sum) return fail(HS_E_IO, "hs_checkpoint_load: checksum mismatch in " + std::string(path));
    if (data_at < 0 || std::fseek(F.f, data_at, SEEK_SET) != 0)
      return fail(HS_E_IO, "hs_checkpoint_load: cannot seek in " + std::string(path));
    // the copies are ordered after the work already enqueued on the stream
    for (int64_t off = 0; off < bytes;) {
      const int64_t n = std::min(bytes - off, kStage);
      HS_HIP(hipStreamSynchronize(s));  // the staging buffer is free again
      if (std::fread(stg.p, 1, (size_t)n, F.f) != (size_t)n)
        return fail(HS_E_IO, "hs_checkpoint_load: read failed on " + std::string(path));
      HS_HIP(hipMemcpyAsync(hdst + off, stg.p, (size_t)n, hipMemcpyHostToDevice, s));
      off += n;
    }
    HS_HIP(hipStreamSynchronize(s));
    return HS_OK;
  }
  std::string buf((size_t)bytes, '\0');
  if (bytes > 0 && std::fread(&buf[0], 1, (size_t)bytes, F.f) != (size_t)bytes)
    return fail(HS_E_IO, "hs_checkpoint_load: read failed on " + std::string(path));
  got = fnv1a(got, reinterpret_cast<const uint8_t *>(buf.data()), buf.size());
  if (got != sum) return fail(HS_E_IO, "hs_checkpoint_load: checksum mismatch in " + std::string(path));
  if (bytes > 0) std::memcpy(hdst, buf.data(), (size_t)bytes);
  return HS_OK;
}
