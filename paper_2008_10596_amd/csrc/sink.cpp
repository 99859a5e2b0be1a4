// sink.cpp -- images to and from files.  The paper's checkpoints end on
// durable storage (DMTCP writes each process's image to a file, Sec. 2.2 and
// Sec. 4); here the serialized image (ckpt_image_serialize's bytes) is written
// and read in large blocks.  Writes bypass the page cache (O_DIRECT) where the
// file system allows it: the image is staged through aligned blocks, one
// thread fills a block while another writes the previous one.
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "ckpt_runtime.h"

using namespace ckpt;

namespace {

constexpr size_t kBlock = size_t(64) << 20;   // bytes per write
constexpr size_t kAlign = 4096;               // O_DIRECT alignment of buffer, offset and length

// The image's serialized bytes as a list of (pointer, length) pieces in file
// order, without copying the large DATA section.
struct Pieces {
    std::vector<uint8_t> head;   // header and tables
    const uint8_t *data = nullptr;
    size_t data_bytes = 0;
};

int image_pieces(const ckpt_image *img, Pieces *out)
{
    if (!img->drained)
        return set_error(CKPT_E_INVAL, "image holds no host data");
    out->head.resize(serialized_head_bytes(img));
    serialize_head(img, out->head.data());
    out->data = (const uint8_t *)img->data.p;
    out->data_bytes = img->ser_bytes;
    return CKPT_OK;
}

// 0, or the errno of the failing write
int write_all(int fd, const uint8_t *p, size_t n, off_t off)
{
    while (n) {
        const ssize_t w = pwrite(fd, p, n, off);
        if (w < 0) {
            if (errno == EINTR)
                continue;
            return errno;
        }
        p += w;
        n -= (size_t)w;
        off += w;
    }
    return 0;
}

}  // namespace

extern "C" int ckpt_image_write_file(const ckpt_image *img, const char *path, uint32_t flags, uint64_t *bytes)
{
    if (!img || !path)
        return set_error(CKPT_E_INVAL, "NULL argument");
    if (flags & ~(uint32_t)CKPT_FILE_BUFFERED)
        return set_error(CKPT_E_INVAL, "unknown file flags 0x%x", flags);
    image_wait(img);
    Pieces pc;
    CKPT_TRY(image_pieces(img, &pc));
    const size_t total = pc.head.size() + pc.data_bytes;
    const std::string tmp_path = std::string(path) + ".partial";

    bool direct = !(flags & CKPT_FILE_BUFFERED);
    int fd = -1;
    if (direct) {
        fd = open(tmp_path.c_str(), O_WRONLY | O_CREAT | O_TRUNC | O_DIRECT, 0644);
        if (fd < 0)
            direct = false;   // the file system has no direct I/O (e.g. tmpfs)
    }
    if (fd < 0)
        fd = open(tmp_path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (fd < 0)
        return set_error(CKPT_E_IO, "cannot create %s: %s", tmp_path.c_str(), strerror(errno));

    // Two aligned blocks: the copier fills one while the writer writes the
    // other.  The file is the concatenation head + DATA; each block is a
    // contiguous file range.
    const size_t nblocks = (total + kBlock - 1) / kBlock;
    uint8_t *buf[2] = {nullptr, nullptr};
    for (auto &b : buf)
        if (posix_memalign((void **)&b, kAlign, kBlock) != 0) {
            free(buf[0]);
            close(fd);
            unlink(tmp_path.c_str());
            return set_error(CKPT_E_NOMEM, "no memory for write blocks");
        }
    auto fill = [&](size_t blk, uint8_t *dst) -> size_t {
        const size_t lo = blk * kBlock, hi = std::min(total, lo + kBlock);
        size_t o = lo;
        if (o < pc.head.size()) {
            const size_t n = std::min(hi, pc.head.size()) - o;
            memcpy(dst, pc.head.data() + o, n);
            o += n;
        }
        if (o < hi)
            memcpy(dst + (o - lo), pc.data + (o - pc.head.size()), hi - o);
        return hi - lo;
    };
    std::mutex mu;
    std::condition_variable cv;
    size_t filled = 0, written = 0;   // blocks filled / written so far
    size_t len[2] = {0, 0};
    int rc = CKPT_OK;
    std::thread copier([&] {
        for (size_t b = 0; b < nblocks; b++) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return b < written + 2 || rc != CKPT_OK; });
                if (rc != CKPT_OK)
                    return;
            }
            const size_t n = fill(b, buf[b & 1]);
            std::lock_guard<std::mutex> lk(mu);
            len[b & 1] = n;
            filled = b + 1;
            cv.notify_all();
        }
    });
    for (size_t b = 0; b < nblocks && rc == CKPT_OK; b++) {
        size_t n;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return filled > b; });
            n = len[b & 1];
        }
        // direct I/O writes whole aligned blocks; the last one is padded and
        // the file cut back to size afterwards
        const size_t wn = direct ? (n + kAlign - 1) / kAlign * kAlign : n;
        if (wn > n)
            memset(buf[b & 1] + n, 0, wn - n);
        int err = write_all(fd, buf[b & 1], wn, (off_t)(b * kBlock));
        if (err == EINVAL && direct) {
            // direct I/O refused at write time: go on through the page cache
            direct = false;
            const int fl = fcntl(fd, F_GETFL);
            if (fl != -1 && fcntl(fd, F_SETFL, fl & ~O_DIRECT) == 0)
                err = write_all(fd, buf[b & 1], n, (off_t)(b * kBlock));
        }
        std::lock_guard<std::mutex> lk(mu);
        if (err)
            rc = set_error(CKPT_E_IO, "write of %s failed: %s", tmp_path.c_str(), strerror(err));
        written = b + 1;
        cv.notify_all();
    }
    copier.join();
    free(buf[0]);
    free(buf[1]);
    if (rc == CKPT_OK && ftruncate(fd, (off_t)total) != 0)
        rc = set_error(CKPT_E_IO, "truncate failed: %s", strerror(errno));
    if (rc == CKPT_OK && fsync(fd) != 0)
        rc = set_error(CKPT_E_IO, "fsync failed: %s", strerror(errno));
    close(fd);
    // the image appears under its name only once complete
    if (rc == CKPT_OK && rename(tmp_path.c_str(), path) != 0)
        rc = set_error(CKPT_E_IO, "rename to %s failed: %s", path, strerror(errno));
    if (rc != CKPT_OK) {
        unlink(tmp_path.c_str());
        return rc;
    }
    if (bytes)
        *bytes = total;
    return CKPT_OK;
}

ImageFile::~ImageFile()
{
    if (fd >= 0)
        close(fd);
}

namespace {

// n bytes at file offset off into p; CKPT_E_IO on an error or a short file
int read_all(int fd, uint8_t *p, size_t n, uint64_t off, const char *path)
{
    while (n) {
        const ssize_t r = pread(fd, p, std::min(n, kBlock), (off_t)off);
        if (r < 0 && errno == EINTR)
            continue;
        if (r < 0)
            return set_error(CKPT_E_IO, "read of %s failed: %s", path, strerror(errno));
        if (r == 0)
            return set_error(CKPT_E_INVAL, "truncated image file %s", path);
        p += r;
        n -= (size_t)r;
        off += (uint64_t)r;
    }
    return CKPT_OK;
}

}  // namespace

int ckpt::open_image_file(const char *path, ImageFile *f)
{
    f->path = path;
    f->fd = open(path, O_RDONLY);
    if (f->fd < 0)
        return set_error(CKPT_E_NOTFOUND, "cannot open %s: %s", path, strerror(errno));
    struct stat st;
    if (fstat(f->fd, &st) != 0)
        return set_error(CKPT_E_IO, "cannot stat %s", path);
    const uint64_t size = (uint64_t)st.st_size;
    // the fixed header gives the size of the head; a short file fails here
    uint8_t hdr[128];
    const size_t nh = (size_t)std::min<uint64_t>(size, sizeof hdr);
    CKPT_TRY(read_all(f->fd, hdr, nh, 0, path));
    uint64_t head = 0, ser = 0;
    CKPT_TRY(head_layout(hdr, nh, size, &head, &ser));
    f->head.resize(head);
    CKPT_TRY(read_all(f->fd, f->head.data(), head, 0, path));
    return parse_head(f->head.data(), head, &f->h, ser);
}

int ckpt::load_image_file(ckpt_ctx *ctx, ImageFile *f, ckpt_image **out)
{
    const uint64_t off = f->h.head_bytes, ser = f->h.ser_bytes;
    ckpt_image *img = nullptr;
    CKPT_TRY(image_from_head(ctx, &f->h, &img));
    std::unique_ptr<ckpt_image> guard(img);
    // DATA in kBlock pieces, dealt round-robin to up to 8 readers, each
    // reading straight into the pinned buffer (no staging copy)
    const uint64_t nblocks = (ser + kBlock - 1) / kBlock;
    const unsigned nt = (unsigned)std::min<uint64_t>({nblocks, 8, std::max(1u, std::thread::hardware_concurrency())});
    std::vector<int> rcs(nt, CKPT_OK);
    std::vector<std::string> errs(nt);
    auto reader = [&](unsigned t) {
        for (uint64_t b = t; b < nblocks; b += nt) {
            const uint64_t lo = b * kBlock, n = std::min<uint64_t>(kBlock, ser - lo);
            const int rc = read_all(f->fd, (uint8_t *)img->data.p + lo, n, off + lo, f->path.c_str());
            if (rc != CKPT_OK) {
                rcs[t] = rc;
                errs[t] = ckpt_last_error();
                return;
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; t++)
        th.emplace_back(reader, t);
    if (nt)
        reader(0);
    for (auto &x : th)
        x.join();
    for (unsigned t = 0; t < nt; t++)
        if (rcs[t] != CKPT_OK)
            return set_error(rcs[t], "%s", errs[t].c_str());
    *out = guard.release();
    return CKPT_OK;
}

extern "C" int ckpt_image_read_file(ckpt_ctx *ctx, const char *path, ckpt_image **out)
{
    if (!path || !out)
        return set_error(CKPT_E_INVAL, "NULL argument");
    ImageFile f;
    CKPT_TRY(open_image_file(path, &f));
    return load_image_file(ctx, &f, out);
}
