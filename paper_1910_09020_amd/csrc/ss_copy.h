// Host copies of large buffers split over a few threads.  ss_server_submit
// stages each request's bases with it: one host thread copies about 9 GB/s, so
// a request of ten million bases per side spent longer in its submission copy
// than on the device.  Several threads may call copy() at once: the pieces of
// every call go to whichever threads are free, the caller among them, and a
// call returns once all of its own pieces are done.
//
// Every field of a job that changes is read and written under the one mutex;
// a piece is copied outside it, from fields fixed before the job was queued.
// A job lives on its caller's stack: it leaves the queue when its last piece
// is taken, and its caller returns only after seeing, under the mutex, the
// count of finished pieces reach the total, so no thread touches it after.
#pragma once
#include <algorithm>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace ss {

class CopyCrew {
public:
    static constexpr size_t kPiece = (size_t)1 << 20;   // bytes per piece
    static constexpr size_t kMin = (size_t)2 << 20;     // smaller copies run on the caller alone

    // helpers: threads besides the callers (fewer if the system refuses some; none: plain copies)
    explicit CopyCrew(int helpers)
    {
        for (int i = 0; i < helpers; i++) {
            try {
                th_.emplace_back([this] { run(); });
            } catch (...) {
                break;
            }
        }
    }
    ~CopyCrew()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    CopyCrew(const CopyCrew&) = delete;
    CopyCrew& operator=(const CopyCrew&) = delete;

    void copy(void* dst, const void* src, size_t n)
    {
        if (n < kMin || th_.empty()) {
            if (n) std::memcpy(dst, src, n);
            return;
        }
        Job job;
        job.dst = static_cast<uint8_t*>(dst);
        job.src = static_cast<const uint8_t*>(src);
        job.n = n;
        job.pieces = (n + kPiece - 1) / kPiece;
        std::unique_lock<std::mutex> lk(mu_);
        jobs_.push_back(&job);
        cv_.notify_all();
        while (job.next < job.pieces) {
            const size_t p = take(job);
            lk.unlock();
            piece(job, p);
            lk.lock();
            job.done++;
        }
        cv_.wait(lk, [&] { return job.done == job.pieces; });
    }

    int helpers() const { return (int)th_.size(); }

private:
    struct Job {
        uint8_t* dst = nullptr;          // fixed before the job is queued
        const uint8_t* src = nullptr;
        size_t n = 0, pieces = 0;
        size_t next = 0, done = 0;       // under mu_
    };

    // the job's next piece (mu_ held); the job leaves the queue with its last one
    size_t take(Job& job)
    {
        const size_t p = job.next++;
        if (job.next == job.pieces) {
            const auto it = std::find(jobs_.begin(), jobs_.end(), &job);
            if (it != jobs_.end()) jobs_.erase(it);
        }
        return p;
    }

    static void piece(const Job& job, size_t p)
    {
        const size_t a = p * kPiece, e = std::min(job.n, a + kPiece);
        std::memcpy(job.dst + a, job.src + a, e - a);
    }

    void run()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !jobs_.empty(); });
            if (jobs_.empty()) return;   // stopping, nothing left
            Job* job = jobs_.front();
            const size_t p = take(*job);
            lk.unlock();
            piece(*job, p);
            lk.lock();
            if (++job->done == job->pieces) cv_.notify_all();
        }
    }

    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Job*> jobs_;
    std::vector<std::thread> th_;
    bool stop_ = false;
};

}  // namespace ss
