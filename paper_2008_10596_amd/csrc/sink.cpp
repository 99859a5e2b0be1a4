// sink.cpp -- images to and from files.  The paper's checkpoints end on
// durable storage (DMTCP writes each process's image to a file, Sec. 2.2 and
// Sec. 4); here the serialized image (ckpt_image_serialize's bytes) is written
// and read in large blocks.  Writes bypass the page cache (O_DIRECT) where the
// file system allows it: the image is staged through aligned blocks, one
// thread fills a block while another writes the previous one.
//
// With CKPT_FILE_DEFLATE the file is a compressed container instead.  DMTCP
// gzips its images by default (the paper turns that off for its timings,
// Sec. 4.4); here DATA is cut into 4 MiB blocks that a pool of threads
// compresses, each block kept raw when it does not shrink, and read back by a
// pool that inflates straight into pinned memory.  Device memory is mostly
// arrays of 2- or 4-byte numbers, whose high bytes (sign and exponent) repeat
// far more than the low ones: a block may first be split into byte planes
// (byte j of every w-byte element together) and then entropy-coded only
// (zlib's Huffman-only deflate, no string matching), or be deflated as it is
// at zlib's fastest level.  A 64 KiB trial of each picks the block's form.
// Container layout, little-endian:
//   magic "CKPTZIP1", u32 version (1), u32 block bytes, u64 head bytes,
//   u64 DATA bytes, u64 block count, one u64 per block (bits 0-60: stored
//   bytes; bits 61-62: planes, 0 none, 1 two, 2 four; bit 63: stored raw),
//   the serialized head (header and tables, as in ckpt_image_serialize), then
//   the blocks back to back, each a zlib stream of the (split) block.
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>
#include <zlib.h>

#include <atomic>
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

constexpr char kZipMagic[8] = {'C', 'K', 'P', 'T', 'Z', 'I', 'P', '1'};
constexpr uint32_t kZipVersion = 1;
constexpr size_t kZipHeader = 8 + 4 + 4 + 8 + 8 + 8;
constexpr uint32_t kZipBlock = 4u << 20;          // DATA bytes per compressed block
constexpr uint64_t kZipRawBit = uint64_t(1) << 63;
constexpr int kZipPlaneShift = 61;
constexpr uint64_t kZipSizeMask = (uint64_t(1) << kZipPlaneShift) - 1;
constexpr unsigned kZipPlanes[3] = {1, 2, 4};   // element width for plane codes 0, 1, 2

// Byte planes of w-byte elements: out[j * m + i] = in[i * w + j] for the m
// whole elements; the n - w m trailing bytes follow as they are.
void split_planes(const uint8_t *in, uint64_t n, unsigned w, uint8_t *out)
{
    const uint64_t m = n / w;
    for (unsigned j = 0; j < w; j++) {
        uint8_t *o = out + j * m;
        const uint8_t *p = in + j;
        for (uint64_t i = 0; i < m; i++)
            o[i] = p[i * w];
    }
    memcpy(out + w * m, in + w * m, n - w * m);
}

void join_planes(const uint8_t *in, uint64_t n, unsigned w, uint8_t *out)
{
    const uint64_t m = n / w;
    for (unsigned j = 0; j < w; j++) {
        const uint8_t *p = in + j * m;
        uint8_t *o = out + j;
        for (uint64_t i = 0; i < m; i++)
            o[i * w] = p[i];
    }
    memcpy(out + w * m, in + w * m, n - w * m);
}

// One zlib stream of src[0, n) in out (cap bytes) at level 1 with the given
// strategy; its size, or 0 when it does not fit.
uint64_t zlib_pack(const uint8_t *src, uint64_t n, uint8_t *out, uint64_t cap, int strategy)
{
    z_stream zs;
    memset(&zs, 0, sizeof(zs));
    if (deflateInit2(&zs, Z_BEST_SPEED, Z_DEFLATED, 15, 8, strategy) != Z_OK)
        return 0;
    zs.next_in = const_cast<Bytef *>(src);
    zs.avail_in = (uInt)n;
    zs.next_out = out;
    zs.avail_out = (uInt)cap;
    const int r = deflate(&zs, Z_FINISH);
    const uint64_t got = zs.total_out;
    deflateEnd(&zs);
    return r == Z_STREAM_END ? got : 0;
}
constexpr size_t kZipProbe = 64 << 10;            // bytes tried first
constexpr double kZipProbeKeep = 0.97;            // a probe above this ratio: the block stays raw
constexpr unsigned kZipThreads = 16;

unsigned pool_threads(uint64_t jobs, unsigned cap)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>({jobs, cap, hw}));
}

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

// The compressed container of pc at fd (buffered I/O).  Threads take blocks
// in order, compress them, and write them in block order as their turn comes;
// the block table is written last.  *total receives the file size.
int write_deflated(int fd, const Pieces &pc, const std::string &tmp_path, uint64_t *total)
{
    const uint64_t nb = (pc.data_bytes + kZipBlock - 1) / kZipBlock;
    std::vector<uint8_t> hdr(kZipHeader);
    memcpy(hdr.data(), kZipMagic, 8);
    const uint32_t h32[2] = {kZipVersion, kZipBlock};
    const uint64_t h64[3] = {pc.head.size(), pc.data_bytes, nb};
    memcpy(hdr.data() + 8, h32, 8);
    memcpy(hdr.data() + 16, h64, 24);
    const uint64_t table_off = kZipHeader, head_off = table_off + 8 * nb;
    int err = write_all(fd, hdr.data(), hdr.size(), 0);
    if (!err)
        err = write_all(fd, pc.head.data(), pc.head.size(), (off_t)head_off);
    if (err)
        return set_error(CKPT_E_IO, "write of %s failed: %s", tmp_path.c_str(), strerror(err));
    std::vector<uint64_t> table(nb, 0);
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<uint64_t> next{0};
    uint64_t turn = 0, pos = head_off + pc.head.size();
    int rc = CKPT_OK;
    std::string msg;
    auto worker = [&] {
        const uint64_t cap = compressBound(kZipBlock);
        std::vector<uint8_t> out(cap), planes(kZipBlock), probe(compressBound(kZipProbe)), pplanes(kZipProbe);
        for (;;) {
            const uint64_t b = next.fetch_add(1);
            if (b >= nb)
                return;
            const uint8_t *src = pc.data + b * kZipBlock;
            const uint64_t n = std::min<uint64_t>(kZipBlock, pc.data_bytes - b * kZipBlock);
            // the form that codes the first 64 KiB smallest: as it is at
            // level 1, or split into 2 or 4 planes and Huffman-coded
            const uint64_t pn = std::min<uint64_t>(n, kZipProbe);
            int code = -1;
            uint64_t best = pn;
            for (int c = 0; c < 3; c++) {
                const uint8_t *in = src;
                if (c > 0) {
                    split_planes(src, pn, kZipPlanes[c], pplanes.data());
                    in = pplanes.data();
                }
                const uint64_t g = zlib_pack(in, pn, probe.data(), probe.size(), c ? Z_HUFFMAN_ONLY : Z_DEFAULT_STRATEGY);
                if (g && g < best) {
                    best = g;
                    code = c;
                }
            }
            // a block whose trial does not shrink below 97% is stored as it is
            bool raw = code < 0 || best >= kZipProbeKeep * pn;
            uint64_t got = 0;
            if (!raw) {
                const uint8_t *in = src;
                if (code > 0) {
                    split_planes(src, n, kZipPlanes[code], planes.data());
                    in = planes.data();
                }
                got = zlib_pack(in, n, out.data(), cap, code ? Z_HUFFMAN_ONLY : Z_DEFAULT_STRATEGY);
                raw = got == 0 || got >= n;
            }
            const uint8_t *w = raw ? src : out.data();
            const uint64_t wn = raw ? n : got;
            // blocks take their file offsets in order; the write itself can
            // overlap the next blocks' writes
            uint64_t at = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return turn == b || rc != CKPT_OK; });
                if (rc != CKPT_OK)
                    return;
                at = pos;
                pos += wn;
                turn = b + 1;
                table[b] = wn | (raw ? kZipRawBit : (uint64_t)code << kZipPlaneShift);
            }
            cv.notify_all();
            const int e = write_all(fd, w, wn, (off_t)at);
            if (e) {
                std::lock_guard<std::mutex> lk2(mu);
                if (rc == CKPT_OK) {
                    rc = CKPT_E_IO;
                    msg = std::string("write of ") + tmp_path + " failed: " + strerror(e);
                }
                cv.notify_all();
                return;
            }
        }
    };
    std::vector<std::thread> th;
    const unsigned nt = pool_threads(nb, kZipThreads);
    for (unsigned t = 1; t < nt; t++)
        th.emplace_back(worker);
    worker();
    for (auto &x : th)
        x.join();
    if (rc != CKPT_OK)
        return set_error(rc, "%s", msg.c_str());
    if (nb && (err = write_all(fd, (const uint8_t *)table.data(), 8 * nb, (off_t)table_off)))
        return set_error(CKPT_E_IO, "write of %s failed: %s", tmp_path.c_str(), strerror(err));
    *total = pos;
    return CKPT_OK;
}

// The file's block table checked against its size and DATA bytes; fills the
// container fields of f.
int parse_zip(const uint8_t *hdr, uint64_t size, ImageFile *f, uint64_t *head_off, uint64_t *head_bytes,
              uint64_t *data_bytes)
{
    uint32_t h32[2];
    uint64_t h64[3];
    memcpy(h32, hdr + 8, 8);
    memcpy(h64, hdr + 16, 24);
    const uint64_t nb = h64[2];
    if (h32[0] != kZipVersion || h32[1] == 0 || h32[1] > (1u << 30) || h64[1] >= (uint64_t(1) << 62))
        return set_error(CKPT_E_INVAL, "bad compressed container header");
    if (nb > size / 8 || nb != (h64[1] + h32[1] - 1) / h32[1] || h64[0] > size)
        return set_error(CKPT_E_INVAL, "truncated compressed container");
    std::vector<uint64_t> table(nb);
    if (nb && pread(f->fd, table.data(), 8 * nb, (off_t)kZipHeader) != (ssize_t)(8 * nb))
        return set_error(CKPT_E_INVAL, "truncated compressed container");
    *head_off = kZipHeader + 8 * nb;
    *head_bytes = h64[0];
    *data_bytes = h64[1];
    f->deflated = true;
    f->zblock = h32[1];
    f->zoff.resize(nb);
    f->zlen.resize(nb);
    f->zraw.resize(nb);
    f->zplanes.resize(nb);
    uint64_t pos = *head_off + h64[0];
    for (uint64_t b = 0; b < nb; b++) {
        const uint64_t want = std::min<uint64_t>(h32[1], h64[1] - b * h32[1]);
        const bool raw = table[b] & kZipRawBit;
        const unsigned code = (unsigned)((table[b] >> kZipPlaneShift) & 3);
        const uint64_t len = table[b] & kZipSizeMask;
        if ((raw && (len != want || code != 0)) || (!raw && (len == 0 || len > compressBound((uLong)want))) ||
            code > 2 || len > size || pos > size - len)
            return set_error(CKPT_E_INVAL, "bad block %llu of the compressed container", (unsigned long long)b);
        f->zoff[b] = pos;
        f->zlen[b] = len;
        f->zraw[b] = raw;
        f->zplanes[b] = (uint8_t)kZipPlanes[code];
        pos += len;
    }
    if (pos != size)
        return set_error(CKPT_E_INVAL, "compressed container is %llu bytes, its table says %llu",
                         (unsigned long long)size, (unsigned long long)pos);
    return CKPT_OK;
}

}  // namespace

extern "C" int ckpt_image_write_file(const ckpt_image *img, const char *path, uint32_t flags, uint64_t *bytes)
{
    if (!img || !path)
        return set_error(CKPT_E_INVAL, "NULL argument");
    if (flags & ~(uint32_t)(CKPT_FILE_BUFFERED | CKPT_FILE_DEFLATE))
        return set_error(CKPT_E_INVAL, "unknown file flags 0x%x", flags);
    image_wait(img);
    Pieces pc;
    CKPT_TRY(image_pieces(img, &pc));
    const size_t total = pc.head.size() + pc.data_bytes;
    const std::string tmp_path = std::string(path) + ".partial";
    if (flags & CKPT_FILE_DEFLATE) {
        const int fd = open(tmp_path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
        if (fd < 0)
            return set_error(CKPT_E_IO, "cannot create %s: %s", tmp_path.c_str(), strerror(errno));
        uint64_t n = 0;
        int rc = write_deflated(fd, pc, tmp_path, &n);
        if (rc == CKPT_OK && ftruncate(fd, (off_t)n) != 0)
            rc = set_error(CKPT_E_IO, "truncate failed: %s", strerror(errno));
        if (rc == CKPT_OK && fsync(fd) != 0)
            rc = set_error(CKPT_E_IO, "fsync failed: %s", strerror(errno));
        close(fd);
        if (rc == CKPT_OK && rename(tmp_path.c_str(), path) != 0)
            rc = set_error(CKPT_E_IO, "rename to %s failed: %s", path, strerror(errno));
        if (rc != CKPT_OK) {
            unlink(tmp_path.c_str());
            return rc;
        }
        if (bytes)
            *bytes = n;
        return CKPT_OK;
    }

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
    if (nh >= kZipHeader && memcmp(hdr, kZipMagic, 8) == 0) {
        uint64_t head_off = 0, head_bytes = 0, data_bytes = 0;
        CKPT_TRY(parse_zip(hdr, size, f, &head_off, &head_bytes, &data_bytes));
        f->head.resize(head_bytes);
        CKPT_TRY(read_all(f->fd, f->head.data(), head_bytes, head_off, path));
        CKPT_TRY(parse_head(f->head.data(), head_bytes, &f->h, data_bytes));
        if (f->h.head_bytes != head_bytes || f->h.ser_bytes != data_bytes)
            return set_error(CKPT_E_INVAL, "compressed container does not match its image header");
        return CKPT_OK;
    }
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
    if (f->deflated) {
        // each block read and inflated straight into its place in the pinned buffer
        const uint64_t nb = f->zoff.size();
        std::atomic<uint64_t> next{0};
        std::mutex mu;
        int rc = CKPT_OK;
        std::string msg;
        auto worker = [&] {
            std::vector<uint8_t> cbuf, planes;
            for (;;) {
                const uint64_t b = next.fetch_add(1);
                if (b >= nb)
                    return;
                uint8_t *dst = (uint8_t *)img->data.p + b * f->zblock;
                const uint64_t want = std::min<uint64_t>(f->zblock, ser - b * f->zblock);
                int r = CKPT_OK;
                if (f->zraw[b]) {
                    r = read_all(f->fd, dst, want, f->zoff[b], f->path.c_str());
                } else {
                    cbuf.resize(f->zlen[b]);
                    r = read_all(f->fd, cbuf.data(), f->zlen[b], f->zoff[b], f->path.c_str());
                    // planes are inflated aside and joined into place
                    const unsigned w = f->zplanes[b];
                    if (w > 1)
                        planes.resize(want);
                    uint8_t *to = w > 1 ? planes.data() : dst;
                    uLongf got = (uLongf)want;
                    if (r == CKPT_OK && (uncompress(to, &got, cbuf.data(), (uLong)f->zlen[b]) != Z_OK || got != want))
                        r = set_error(CKPT_E_INVAL, "block %llu of %s does not inflate to %llu bytes",
                                      (unsigned long long)b, f->path.c_str(), (unsigned long long)want);
                    if (r == CKPT_OK && w > 1)
                        join_planes(planes.data(), want, w, dst);
                }
                if (r != CKPT_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    if (rc == CKPT_OK) {
                        rc = r;
                        msg = ckpt_last_error();
                    }
                    next.store(nb);   // the other workers stop at their next block
                    return;
                }
            }
        };
        std::vector<std::thread> th;
        const unsigned nt = pool_threads(nb, kZipThreads);
        for (unsigned t = 1; t < nt; t++)
            th.emplace_back(worker);
        worker();
        for (auto &x : th)
            x.join();
        if (rc != CKPT_OK)
            return set_error(rc, "%s", msg.c_str());
        *out = guard.release();
        return CKPT_OK;
    }
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

extern "C" int ckpt_image_file_info(const char *path, ckpt_image_meta *out)
{
    if (!path || !out)
        return set_error(CKPT_E_INVAL, "NULL argument");
    ImageFile f;
    CKPT_TRY(open_image_file(path, &f));
    const ImageHead &h = f.h;
    if (crc_digest(h.rest, h.N * 4) != h.digest)
        return set_error(CKPT_E_INVAL, "CRC section digest mismatch");
    memset(out, 0, sizeof(*out));
    out->mode = h.mode;
    out->chunk_bytes = h.C;
    out->n_allocs = h.allocs.size();
    out->n_chunks = h.N;
    out->data_bytes = h.data_bytes;
    out->serialized_bytes = h.ser_bytes;
    out->n_dirty = h.n_dirty;
    out->serial = h.serial;
    out->base_serial = h.base_serial;
    out->crc_digest = h.digest;
    out->drained = 1;
    return CKPT_OK;
}
