// Page images of a streamed scene (host logic, no device calls): one image
// per cluster, kept in host memory or in a file on disk.
//
// The file tier writes every image at a multiple of slot_bytes (the image
// size rounded up to 4 KiB), so that reads can bypass the page cache
// (O_DIRECT) where the file system allows it; otherwise reads are buffered.
// A batch of images is read with one positioned read per run of consecutive
// clusters: the caller passes the clusters in ascending order, so a run of
// neighbouring clusters (a cut is spatially coherent, and cluster ids follow
// the build order) lands in consecutive staging slots in one system call.
// Direct reads go through an aligned bounce buffer of the store's own (the
// kernel cannot always transfer straight into memory pinned for the GPU).
#pragma once

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace v3dg {

class PageStore {
public:
    enum Tier : uint32_t { kMemory = 0, kFileBuffered = 1, kFileDirect = 2 };
    static constexpr uint64_t kAlign = 4096;
    static constexpr uint64_t kBounceBytes = 4u << 20;  // direct reads of up to 4 MiB at a time

    PageStore() = default;
    PageStore(const PageStore &) = delete;
    PageStore &operator=(const PageStore &) = delete;
    ~PageStore() { close(); }

    void init_memory(uint32_t n_pages, uint32_t page_bytes)
    {
        close();
        tier_ = kMemory;
        page_bytes_ = page_bytes;
        slot_bytes_ = page_bytes;
        mem_.assign((uint64_t)n_pages * page_bytes, 0);
    }

    // Creates (or truncates) path.  direct asks for O_DIRECT reads; when the
    // file system refuses them the store reads through the page cache.
    bool init_file(const char *path, uint32_t n_pages, uint32_t page_bytes, bool direct, bool keep, std::string *err)
    {
        close();
        page_bytes_ = page_bytes;
        slot_bytes_ = (page_bytes + kAlign - 1) / kAlign * kAlign;
        path_ = path;
        keep_ = keep;
        wfd_ = ::open(path, O_CREAT | O_TRUNC | O_RDWR | O_CLOEXEC, 0600);
        if (wfd_ < 0) return fail(err, "cannot create the page file");
        if (::ftruncate(wfd_, (off_t)((uint64_t)n_pages * slot_bytes_)) != 0) return fail(err, "cannot size the page file");
        tier_ = kFileBuffered;
        if (direct) {
            const int fd = ::open(path, O_RDONLY | O_DIRECT | O_CLOEXEC);
            if (fd >= 0) {
                rfd_ = fd;
                tier_ = kFileDirect;
            }
        }
        if (rfd_ < 0) rfd_ = ::open(path, O_RDONLY | O_CLOEXEC);
        if (rfd_ < 0) return fail(err, "cannot open the page file for reading");
        return true;
    }

    // Writes the image of cluster k (page_bytes bytes).
    bool put(uint32_t k, const uint8_t *img, std::string *err)
    {
        if (tier_ == kMemory) {
            std::memcpy(mem_.data() + (uint64_t)k * page_bytes_, img, page_bytes_);
            return true;
        }
        if (!write_all(wfd_, img, page_bytes_, (uint64_t)k * slot_bytes_)) return fail(err, "writing the page file failed");
        return true;
    }

    // Done writing: the file's pages are flushed so that direct reads see them.
    bool seal(std::string *err)
    {
        if (tier_ == kMemory) return true;
        if (::fsync(wfd_) != 0) return fail(err, "flushing the page file failed");
        return true;
    }

    // Copies the images of clusters ks[0 .. m) (strictly ascending) to
    // dst + j * stride() (dst aligned to kAlign for the direct tier).
    bool get(const uint32_t *ks, uint32_t m, uint8_t *dst, std::string *err)
    {
        if (tier_ == kMemory) {
            for (uint32_t j = 0; j < m; ++j)
                std::memcpy(dst + (uint64_t)j * slot_bytes_, mem_.data() + (uint64_t)ks[j] * page_bytes_, page_bytes_);
            return true;
        }
        const uint32_t bounce_slots = (uint32_t)(kBounceBytes / slot_bytes_);
        if (tier_ == kFileDirect && !bounce_) {
            void *b = nullptr;
            if (bounce_slots == 0 || posix_memalign(&b, kAlign, (size_t)bounce_slots * slot_bytes_) != 0)
                return fail(err, "no bounce buffer for direct reads");
            bounce_ = static_cast<uint8_t *>(b);
        }
        for (uint32_t j = 0; j < m;) {
            uint32_t e = j + 1;
            const uint32_t lim = tier_ == kFileDirect ? bounce_slots : m;
            while (e < m && ks[e] == ks[e - 1] + 1 && e - j < lim) ++e;
            // a run of consecutive clusters: one read into consecutive slots
            const uint64_t bytes = (uint64_t)(e - j) * slot_bytes_, off = (uint64_t)ks[j] * slot_bytes_;
            uint8_t *to = dst + (uint64_t)j * slot_bytes_;
            if (tier_ == kFileDirect) {
                if (!read_all(rfd_, bounce_, bytes, off)) return fail(err, "reading the page file failed");
                std::memcpy(to, bounce_, bytes);
            } else if (!read_all(rfd_, to, bytes, off)) {
                return fail(err, "reading the page file failed");
            }
            ++reads_;
            j = e;
        }
        return true;
    }

    uint64_t stride() const { return slot_bytes_; }
    uint32_t tier() const { return tier_; }
    uint64_t reads() const { return reads_; }

    void close()
    {
        if (rfd_ >= 0) ::close(rfd_);
        if (wfd_ >= 0) ::close(wfd_);
        if (!path_.empty() && !keep_) ::unlink(path_.c_str());
        rfd_ = wfd_ = -1;
        free(bounce_);
        bounce_ = nullptr;
        path_.clear();
        mem_.clear();
        tier_ = kMemory;
        reads_ = 0;
    }

private:
    static bool fail(std::string *err, const char *what)
    {
        if (err) *err = std::string(what) + ": " + std::strerror(errno);
        return false;
    }
    static bool write_all(int fd, const uint8_t *p, uint64_t n, uint64_t off)
    {
        while (n) {
            const ssize_t w = ::pwrite(fd, p, n, (off_t)off);
            if (w < 0 && errno == EINTR) continue;
            if (w <= 0) return false;
            p += w;
            n -= (uint64_t)w;
            off += (uint64_t)w;
        }
        return true;
    }
    static bool read_all(int fd, uint8_t *p, uint64_t n, uint64_t off)
    {
        while (n) {
            const ssize_t r = ::pread(fd, p, n, (off_t)off);
            if (r < 0 && errno == EINTR) continue;
            if (r <= 0) return false;
            p += r;
            n -= (uint64_t)r;
            off += (uint64_t)r;
        }
        return true;
    }

    uint32_t tier_ = kMemory;
    uint64_t page_bytes_ = 0, slot_bytes_ = 0, reads_ = 0;
    std::vector<uint8_t> mem_;
    int rfd_ = -1, wfd_ = -1;
    uint8_t *bounce_ = nullptr;
    std::string path_;
    bool keep_ = false;
};

}  // namespace v3dg
